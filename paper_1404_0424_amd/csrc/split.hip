// Split forms of CG-D detection and CG-P precoding (Sec. III-B, III-C-2,
// III-D, Algorithm 1) for complex64 storage, U <= 32, S <= 16: the four
// wavefronts of a workgroup share one subcarrier.  Wave w accumulates the
// Gram (and, for detection, the matched filter) over its quarter of the
// antennas, the partial sums meet in LDS (added in the fixed order
// 0 + 1 + 2 + 3), and wave 0 runs the CG, the SINR and the LLRs; for
// precoding every wave then forms q = H v for its own antennas, with its
// quarter of H kept in registers since the Gram, so H crosses HBM once.
//
// A launch with few subcarriers per SIMD (3,300 subcarriers of 256 x 32,
// one frame) runs four wavefronts per subcarrier instead of one, and the
// Gram, which dominates the arithmetic, is spread over four SIMDs.  The
// antenna split changes the summation order of the Gram: results match the
// other schedules to rounding, not bitwise.
#include "detect_core.hpp"
#include "gram_stream.hpp"
#include "launch.hpp"
#include "precode_out.hpp"

namespace mimo {

constexpr int kSplitWaves = 4;

// Antenna range [a0, a1) of wave wv: consecutive runs of ceil(B / 16)
// k-steps (4 antennas each).
struct SplitRange {
  int a0, a1, kq;
  __device__ SplitRange(int B, int wv) {
    const int nks = (B + 3) >> 2;
    kq = (nks + kSplitWaves - 1) / kSplitWaves;
    a0 = 4 * kq * wv < B ? 4 * kq * wv : B;
    a1 = 4 * kq * (wv + 1) < B ? 4 * kq * (wv + 1) : B;
  }
};

// f4 values per lane of one partial accumulator
template <int W, bool DO_MF>
constexpr int split_acc_f4() { return 2 * GramAcc<W>::NT + (DO_MF ? 3 * W : 0); }

// Sums the four waves' partial accumulators into wave 0's `acc` through
// R (3 x split_acc_f4 x 64 f4 of LDS).  Called by all four waves.
template <int W, bool DO_MF>
__device__ __forceinline__ void split_reduce(GramAcc<W>& acc, f4* R, int wv, int lane) {
  constexpr int NT = GramAcc<W>::NT, NQ = split_acc_f4<W, DO_MF>();
  if (wv > 0) {
    f4* r = R + (wv - 1) * NQ * kWave + lane;
    int q = 0;
#pragma unroll
    for (int t = 0; t < NT; ++t) { r[kWave * q++] = acc.gr[t]; r[kWave * q++] = acc.gi[t]; }
    if (DO_MF) {
#pragma unroll
      for (int w = 0; w < W; ++w) {
        r[kWave * q++] = acc.dr[w];
        r[kWave * q++] = acc.di[w];
        r[kWave * q++] = acc.p3[w];
      }
    }
  }
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int k = 0; k < kSplitWaves - 1; ++k) {
      const f4* r = R + k * NQ * kWave + lane;
      int q = 0;
#pragma unroll
      for (int t = 0; t < NT; ++t) { acc.gr[t] += r[kWave * q++]; acc.gi[t] += r[kWave * q++]; }
      if (DO_MF) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          acc.dr[w] += r[kWave * q++];
          acc.di[w] += r[kWave * q++];
          acc.p3[w] += r[kWave * q++];
        }
      }
    }
  }
  __syncthreads();          // R is free for the next subcarrier's partial sums
}

template <int W, typename ST, int M_BITS>
__global__ __launch_bounds__(256, 2) void detect_split_kernel(DetectParams prm) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;
  constexpr int AP = 2 * (NU * AST + NU * kPST);   // wave 0: A then P (floats)
  constexpr int STG = NU * 16 * M_BITS;            // wave 0: LLR tile
  constexpr int NQ = split_acc_f4<W, true>();
  using Sub = SubC32<W>;
  using Blk = typename Storage<InC32, W>::SmallBlock;
  __shared__ __align__(16) f4 R_s[(kSplitWaves - 1) * NQ * kWave];
  __shared__ __align__(16) float W_s[AP > STG ? AP : STG];
  __shared__ float G_s[NU];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = lane & 15, g = lane >> 4;
  float2* As = (float2*)W_s;
  float2* Ps = As + NU * AST;
  const int B = prm.B, U = prm.U, S = prm.S;
  const SplitRange rg(B, wv);
  const int rows = rg.a1 - rg.a0;
  const float2* H = (const float2*)prm.H;
  const float2* Y = (const float2*)prm.Y;
  auto part = [&](Sub& sb, int64_t m) {       // this wave's rows of subcarrier m
    sb.init(H + ((size_t)m * B + rg.a0) * U, Y + ((size_t)m * B + rg.a0) * S, rows, U, S, 0, c, g);
  };

  int64_t n = blockIdx.x;
  Sub cur;
  Blk blk;
  if (n < prm.n_sc) {
    part(cur, n);
    blk.template load<true>(cur, 0);
  }
  while (n < prm.n_sc) {
    const int64_t nn = n + gridDim.x;
    Sub nxt;
    part(nxt, nn < prm.n_sc ? nn : n);
    if (nn >= prm.n_sc) nxt.disable();
    // ---- partial A and b over this wave's antennas (Algorithm 1, initialization)
    GramAcc<W> acc;
    acc.clear();
    gram_stream<W, true>(InC32{}, blk, cur, nxt, rows, acc);
    split_reduce<W, true>(acc, R_s, wv, lane);
    if (wv == 0) {
      AOperand<W> at;
      float d[W];
      gram_to_operands<W>(InC32{}, acc, As, G_s, Ps, AST, prm.reg, U, c, g, at, d);
      cg_llr_epilogue<W, ST, M_BITS, true, true>(prm, n, 0, acc, at, d, G_s, Ps, c, g, W_s);
    }
    n = nn;
    cur = nxt;
  }
}

// Output tile (16 antennas) of this wave's resident channel to LDS as
// Ts[antenna][slot] (row stride HST), user 16 w + u in slot 16 w + 4 (u % 4)
// + u / 4: the contraction's k-step t of tile w takes users 16 w + 4 t + g,
// which sit in the four adjacent slots 16 w + 4 g .. + 3 of a row.
template <int W, int KQ>
__device__ __forceinline__ void split_stage_tile(const BlockC32<W, 1> (&hb)[KQ], int i,
                                                 float2* __restrict__ Ts, int hst, int c,
                                                 int g) {
  const int sl = ((c & 3) << 2) | (c >> 2);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int w = 0; w < W; ++w) Ts[(4 * t + g) * hst + 16 * w + sl] = hb[4 * i + t].h[0][w];
}

// Precoding with the channel resident: wave w keeps its KQ k-steps of H in
// registers from the Gram to q = H v, and reloads them with the next
// subcarrier's while the output stage runs.
template <int W, typename ST>
__global__ __launch_bounds__(256, 2) void precode_split_kernel(PrecodeParams prm) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;
  constexpr int HST = NU + 2;                      // staged tile row stride (complex)
  constexpr int KQ = 16;                           // k-steps in registers: B <= 256
  constexpr int NQ = split_acc_f4<W, false>();
  using Sub = SubC32<W>;
  using RB = BlockC32<W, 1>;
  __shared__ __align__(16) f4 R_s[(kSplitWaves - 1) * NQ * kWave];
  __shared__ __align__(16) float2 A_s[NU * AST];
  __shared__ __align__(16) float2 P_s[NU * kPST];  // V for every wave's output stage
  __shared__ __align__(16) float2 T_s[kSplitWaves][16 * HST];
  __shared__ float G_s[NU];
  __shared__ float N_s[16];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = lane & 15, g = lane >> 4;
  const int B = prm.B, U = prm.U, S = prm.S;
  const SplitRange rg(B, wv);
  const int rows = rg.a1 - rg.a0;
  const float2* H = (const float2*)prm.H;
  float2* Ts = T_s[wv];
  auto part = [&](Sub& sb, int64_t m) {
    sb.init(H + ((size_t)m * B + rg.a0) * U, nullptr, rows, U, S, 0, c, g);
  };

  int64_t n = blockIdx.x;
  RB hb[KQ];
  {
    Sub cur;
    part(cur, n < prm.n_sc ? n : 0);
    if (n >= prm.n_sc) cur.disable();
#pragma unroll
    for (int t = 0; t < KQ; ++t) hb[t].template load<false>(cur, 4 * t);
  }
  while (n < prm.n_sc) {
    const int64_t nn = n + gridDim.x;
    // ---- partial G over this wave's antennas (Algorithm 1, initialization)
    GramAcc<W> acc;
    acc.clear();
#pragma unroll
    for (int t = 0; t < KQ; ++t)
      if (4 * t < rows) hb[t].template mma<true, false>(acc);
    split_reduce<W, false>(acc, R_s, wv, lane);
    if (wv == 0) {
      store_gram(InC32{}, acc, A_s, G_s, (float*)P_s, AST, prm.beta, c, g);
      wave_lds_sync();
      AOperand<W> at;
      at.load(A_s, AST, c, g, U);
      float2 b[W][4];                                 // b = t
      const __amdgpu_buffer_rsrc_t rt =
          make_rsrc(prm.T + (size_t)n * U * S, (uint32_t)U * S * 8u);
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int u = 16 * w + c, s = 4 * g + j;
          b[w][j] = bload2(rt, (u < U && s < S) ? (uint32_t)(u * S + s) * 8u : kOOB, 0u);
        }
      CGState<W, ST> st;
      cg_init<W, ST>(st, b);
      for (int k = 0; k < prm.K; ++k) {
        ST al[4], be[4];
        cg_step<W, ST>(st, at, P_s, c, g, al, be);
      }
      // ||q||^2 = v^H G v; V stays staged in P_s for every wave
      stage_vec<W>(P_s, c, g, st.v);
      wave_lds_sync();
      qnorm2_lds<W, ST>(at, G_s, st.v, P_s, N_s, c, g);
      const __amdgpu_buffer_rsrc_t rn =
          prm.qnorm ? make_rsrc(prm.qnorm + (size_t)n * S, (uint32_t)S * 4u)
                    : make_rsrc(nullptr, 0u);
      wave_lds_sync();
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int ss = 4 * g + j;
        bstore1(rn, (c == 0 && ss < S) ? (uint32_t)ss * 4u : kOOB, sqrtf(N_s[ss]));
      }
    }
    __syncthreads();                                  // V and the norms are in LDS
    // ---- q = H_u v for this wave's antennas (MFMA: rows = antennas,
    // columns = right-hand sides, k = users), H from registers
    const float nrm2 = N_s[c];
    const float scl = prm.normalize ? (nrm2 > 0.f ? __builtin_amdgcn_rsqf(nrm2) : 0.f) : 1.0f;
    float2 vv[W][4];
    float vs[W][4];
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        vv[w][t] = P_s[(16 * w + 4 * t + g) * kPST + c];
        vs[w][t] = vv[w][t].x + vv[w][t].y;
      }
    Sub nxt;                                          // empty past the last subcarrier
    part(nxt, nn < prm.n_sc ? nn : n);
    if (nn >= prm.n_sc) nxt.disable();
    const __amdgpu_buffer_rsrc_t rq =
        make_rsrc(prm.Q + ((size_t)n * B + rg.a0) * S, (uint32_t)(rows * S) * 8u);
#pragma unroll
    for (int i = 0; i < KQ / 4; ++i) {
      if (16 * i < rows) {
        wave_lds_sync();                              // previous tile's reads are done
        split_stage_tile<W, KQ>(hb, i, Ts, HST, c, g);
        wave_lds_sync();
        f4 p1 = zero4(), p2 = zero4(), p3 = zero4();
#pragma unroll
        for (int w = 0; w < W; ++w) {
          float2 hv[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) hv[t] = Ts[c * HST + 16 * w + 4 * g + t];   // user 16 w + 4 t + g
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            if (16 * w + 4 * t >= U) break;           // users past U: v is zero
            p1 = mfma4(hv[t].x, vv[w][t].x, p1);
            p2 = mfma4(hv[t].y, vv[w][t].y, p2);
            p3 = mfma4(hv[t].x + hv[t].y, vs[w][t], p3);
          }
        }
        const f4 qr = p1 - p2;
        const f4 qi = p3 - p1 - p2;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = 16 * i + 4 * g + j;           // antenna a0 + r, rhs c
          bstore2<0>(rq, (r < rows && c < S) ? (uint32_t)(r * S + c) * 8u : kOOB, qr[j] * scl,
                     qi[j] * scl);
        }
      }
      // the staged tile's k-steps receive the next subcarrier's
#pragma unroll
      for (int t = 4 * i; t < 4 * i + 4; ++t) hb[t].template load<false>(nxt, 4 * t);
    }
    n = nn;
  }
}

bool split_eligible(int in_dtype, int U, int S, int B, bool precode) {
  return in_dtype == 0 && U <= 32 && S <= 16 && (!precode || B <= 256);
}

static unsigned int split_grid(int64_t n_sc, const Schedule& sch) {
  int64_t blocks = n_sc;
  if (sch.blocks_per_cu > 0) {
    const int64_t cap = (int64_t)num_compute_units() * sch.blocks_per_cu;
    if (blocks > cap) blocks = cap;
  }
  if (blocks > (1 << 20)) blocks = 1 << 20;
  if (blocks < 1) blocks = 1;
  return (unsigned int)blocks;
}

template <int W, typename ST>
static hipError_t launch_detect_split_m(const DetectParams& p, int m_bits, const Schedule& sch,
                                        hipStream_t stream) {
  const dim3 grid(split_grid(p.n_sc, sch)), block(kWave * kSplitWaves);
  switch (m_bits) {
    case 2: hipLaunchKernelGGL((detect_split_kernel<W, ST, 2>), grid, block, 0, stream, p); break;
    case 4: hipLaunchKernelGGL((detect_split_kernel<W, ST, 4>), grid, block, 0, stream, p); break;
    case 6: hipLaunchKernelGGL((detect_split_kernel<W, ST, 6>), grid, block, 0, stream, p); break;
    case 8: hipLaunchKernelGGL((detect_split_kernel<W, ST, 8>), grid, block, 0, stream, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_detect_split(const DetectParams& p, int scalar_f64, int m_bits,
                               const Schedule& sch, hipStream_t stream) {
  if (p.U <= 16)
    return scalar_f64 ? launch_detect_split_m<1, double>(p, m_bits, sch, stream)
                      : launch_detect_split_m<1, float>(p, m_bits, sch, stream);
  return scalar_f64 ? launch_detect_split_m<2, double>(p, m_bits, sch, stream)
                    : launch_detect_split_m<2, float>(p, m_bits, sch, stream);
}

hipError_t launch_precode_split(const PrecodeParams& p, int scalar_f64, const Schedule& sch,
                                hipStream_t stream) {
  const dim3 grid(split_grid(p.n_sc, sch)), block(kWave * kSplitWaves);
  if (p.U <= 16) {
    if (scalar_f64) hipLaunchKernelGGL((precode_split_kernel<1, double>), grid, block, 0, stream, p);
    else hipLaunchKernelGGL((precode_split_kernel<1, float>), grid, block, 0, stream, p);
  } else {
    if (scalar_f64) hipLaunchKernelGGL((precode_split_kernel<2, double>), grid, block, 0, stream, p);
    else hipLaunchKernelGGL((precode_split_kernel<2, float>), grid, block, 0, stream, p);
  }
  return hipGetLastError();
}

}  // namespace mimo

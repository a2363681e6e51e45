// Fused CG-D kernel: Gram + matched filter (MFMA) -> K CG iterations with the
// approximate in-loop SINR tracker -> max-log LLR epilogue, one wavefront per
// subcarrier (Sec. III-B, III-C-2, Algorithm 1, eqs. (4), (13)-(15)).
#include <type_traits>

#include "cg_core.hpp"
#include "gram_phase.hpp"
#include "launch.hpp"
#include "llr.hpp"

namespace mimo {

// Output descriptors of one subcarrier: LLR, xhat, mu and sinr as buffer
// resources over that subcarrier's [U][S] entries (zero-size when the
// optional output is absent), so every lane issues the same stores and
// masked entries are dropped by the range check: no branches around the
// stores, and the compiler's memory-counter waits stay exact.
template <int M_BITS>
struct DetectStore {
  __amdgpu_buffer_rsrc_t llr, xhat, mu, sinr;
  __device__ void init(const DetectParams& p, int64_t n) {
    const uint32_t per = (uint32_t)(p.U * p.S);
    llr = make_rsrc(p.llr + (size_t)n * per * M_BITS, per * M_BITS * 4u);
    xhat = make_rsrc(p.xhat ? (const void*)(p.xhat + (size_t)n * per) : p.llr,
                     p.xhat ? per * 8u : 0u);
    mu = make_rsrc(p.mu ? (const void*)(p.mu + (size_t)n * per) : p.llr, p.mu ? per * 4u : 0u);
    sinr = make_rsrc(p.sinr ? (const void*)(p.sinr + (size_t)n * per) : p.llr,
                     p.sinr ? per * 4u : 0u);
  }
  // xhat, mu, sinr of entry e = u * S + s (or -1 for a masked lane)
  __device__ void store_aux(int e, float2 x, float m, float rho) const {
    const bool ok = e >= 0;
    bstore2<0>(xhat, ok ? (uint32_t)e * 8u : kOOB, x.x, x.y);
    const uint32_t o4 = ok ? (uint32_t)e * 4u : kOOB;
    bstore1<0>(mu, o4, m);
    bstore1<0>(sinr, o4, rho);
  }
  // entry e = u * S + s, or -1 for a masked lane
  __device__ void store(int e, const float (&out)[M_BITS], float2 x, float m, float rho) const {
    const bool ok = e >= 0;
    const uint32_t ol = ok ? (uint32_t)e * (M_BITS * 4u) : kOOB;
    if constexpr (M_BITS == 2) {
      bstore2(llr, ol, out[0], out[1]);
    } else if constexpr (M_BITS == 4) {
      bstore4(llr, ol, out[0], out[1], out[2], out[3]);
    } else if constexpr (M_BITS == 6) {
      bstore3(llr, ol, out[0], out[1], out[2]);
      bstore3(llr, ol + 12u, out[3], out[4], out[5]);
    } else {
      bstore4(llr, ol, out[0], out[1], out[2], out[3]);
      bstore4(llr, ol + 16u, out[4], out[5], out[6], out[7]);
    }
    bstore2<0>(xhat, ok ? (uint32_t)e * 8u : kOOB, x.x, x.y);
    const uint32_t o4 = ok ? (uint32_t)e * 4u : kOOB;
    bstore1<0>(mu, o4, m);
    bstore1<0>(sinr, o4, rho);
  }
};

// Memory-op form per storage type, chosen by measurement on MI355X: with
// complex64 storage the unconditional prefetch and buffer-descriptor stores
// are faster (the compiler's load-counter waits then cover exactly the
// block consumed); with 16-bit storage the branchy form is faster.
template <typename IN>
constexpr bool kUncondMem = std::is_same<IN, InC32>::value || std::is_same<IN, InC32P>::value;

// K iterations of Algorithm 1 with the tracker of eq. (13), then mu (eq. (14)),
// rho (eq. (15)), z = xhat / mu and the LLRs (eq. (4)) of right-hand sides
// s0 + 4 g + j of subcarrier n.  A^T, d and G_ii come from the Gram phase.
// BUF: stores through buffer descriptors (no branches) or plain stores.
// STAGE (all right-hand sides in this chunk): the subcarrier's LLR
// tile, U x S x M_BITS floats contiguous in memory, is assembled in `stg`
// (wave-private LDS, free once the CG is done) and written with one
// contiguous 16-byte (or 8-byte) piece per lane, so every store instruction
// covers whole cache lines; scattered 12-byte pieces let partly written lines
// leave L2 under load and reach HBM more than once.
template <int W, typename ST, int M_BITS, bool BUF, bool STAGE = false>
__device__ __forceinline__ void cg_llr_epilogue(const DetectParams& prm, int64_t n, int s0,
                                                const GramAcc<W>& acc, const AOperand<W>& at,
                                                const float (&d)[W], const float* Gs,
                                                float2* Ps, int c, int g,
                                                float* __restrict__ stg = nullptr) {
  const int U = prm.U, S = prm.S;
  float2 b[W][4];
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int j = 0; j < 4; ++j) b[w][j] = make_float2(acc.dr[w][j], acc.di[w][j]);
  CGState<W, ST> st;
  cg_init<W, ST>(st, b);
  Tracker<W, ST> tk;
  tk.init();
  for (int k = 0; k < prm.K; ++k) {
    ST al[4], be[4];
    cg_step<W, ST>(st, at, Ps, c, g, al, be);
    tracker_step<W, ST>(tk, d, al, be);
  }
  DetectStore<M_BITS> os;
  if (BUF || STAGE) os.init(prm, n);
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int u = 16 * w + c;
    const float Guu = Gs[u < U ? u : 0];
    const float rho = Guu / prm.n0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int s = s0 + 4 * g + j;
      const float mu = (float)(tk.tv[w][j] * (ST)Guu);
      const float2 x = st.v[w][j];
      // |mu| < FLT_MIN only when the right-hand side froze at (near) zero:
      // z = 0 as for b = 0.
      const float imu = fabsf(mu) >= __FLT_MIN__ ? __builtin_amdgcn_rcpf(mu) : 0.f;
      const float2 z = make_float2(x.x * imu, x.y * imu);
      float out[M_BITS];
      llr_maxlog<M_BITS>(z, rho, prm.scale, prm.inv_scale, out);
      if (STAGE) {
        if (u < U && s < S) {
          float* sp = stg + (u * S + s) * M_BITS;
#pragma unroll
          for (int q = 0; q < M_BITS; ++q) sp[q] = out[q];
        }
        os.store_aux((u < U && s < S) ? u * S + s : -1, x, mu, rho);
      } else if (BUF) {
        os.store((u < U && s < S) ? u * S + s : -1, out, x, mu, rho);
      } else if (u < U && s < S) {
        const size_t idx = ((size_t)n * U + u) * S + s;
        float* lp = prm.llr + idx * M_BITS;
#pragma unroll
        for (int q = 0; q < M_BITS; ++q) lp[q] = out[q];
        if (prm.xhat) prm.xhat[idx] = x;
        if (prm.mu) prm.mu[idx] = mu;
        if (prm.sinr) prm.sinr[idx] = rho;
      }
    }
  }
  if (STAGE) {
    wave_lds_sync();
    const int lane = 16 * g + c;
    const int total = U * S * M_BITS;             // floats, even (M_BITS is even)
    if ((total & 3) == 0) {                       // 16-byte aligned tile
      const float4* src = (const float4*)stg;
      for (int o = lane; o < total / 4; o += kWave) {
        const float4 v = src[o];
        bstore4(os.llr, (uint32_t)o * 16u, v.x, v.y, v.z, v.w);
      }
    } else {
      const float2* src = (const float2*)stg;
      for (int o = lane; o < total / 2; o += kWave) {
        const float2 v = src[o];
        bstore2(os.llr, (uint32_t)o * 8u, v.x, v.y);
      }
    }
    wave_lds_sync();                              // stg is A / P of the next subcarrier
  }
}

// Gram tiles -> LDS A, A^T operand and diagonal d = A_ii.
template <int W, typename IN>
__device__ __forceinline__ void gram_to_operands(IN tag, const GramAcc<W>& acc, float2* As,
                                                 float* Gs, float2* Ps, int ast, float reg, int U,
                                                 int c, int g, AOperand<W>& at, float (&d)[W]) {
  store_gram(tag, acc, As, Gs, (float*)Ps, ast, reg, c, g);
  wave_lds_sync();
  at.load(As, ast, c, g, U);
#pragma unroll
  for (int w = 0; w < W; ++w) d[w] = As[(16 * w + c) * ast + 16 * w + c].x;
}

// Streaming kernel for S <= 16 (one right-hand-side chunk).  Each wavefront
// keeps the next block of H / Y loads in flight while the MFMAs of the
// current block run, and issues the first block of its next subcarrier
// before the CG / LLR phase of the current one, so HBM latency overlaps
// compute within the wave as well as across waves.
template <int W, typename IN, typename ST, int M_BITS, bool SMALL>
__global__ __launch_bounds__(256, 2) void detect_stream_kernel(DetectParams prm) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;   // LDS row stride (complex) of A
  using Sub = typename Storage<IN, W>::Sub;
  using Blk = typename std::conditional<SMALL, typename Storage<IN, W>::SmallBlock,
                                        typename Storage<IN, W>::Block>::type;
  // per wave: A then P (float2), reused as the LLR staging tile
  constexpr int AP = 2 * (NU * AST + NU * kPST);                     // floats
  constexpr int STG = NU * 16 * M_BITS;
  __shared__ __align__(16) float W_s[kWavesPerBlock][AP > STG ? AP : STG];
  __shared__ float G_s[kWavesPerBlock][NU];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  float2* As = (float2*)W_s[wv];
  float2* Ps = As + NU * AST;
  float* Gs = G_s[wv];
  const int B = prm.B, U = prm.U, S = prm.S;
  const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;

  int64_t n = (int64_t)blockIdx.x * kWavesPerBlock + wv;
  Sub cur;
  Blk blk;
  if (n < prm.n_sc) {
    cur.init(offset_sc(IN{}, prm.H, n, B, U), offset_sc(IN{}, prm.Y, n, B, S), B, U, S, 0, c, g);
    blk.template load<true>(cur, 0);
  }
  while (n < prm.n_sc) {
    const int64_t nn = n + stride;
    const int64_t nc = nn < prm.n_sc ? nn : n;        // descriptors only used if nn < n_sc
    Sub nxt;
    nxt.init(offset_sc(IN{}, prm.H, nc, B, U), offset_sc(IN{}, prm.Y, nc, B, S), B, U, S, 0, c, g);
    if (nn >= prm.n_sc) nxt.disable();       // last subcarrier: prefetch reads nothing
    // ---- A = H^H H + (N0/E_s) I and b = H^H y (Algorithm 1, initialization)
    GramAcc<W> acc;
    acc.clear();
    // ping-pong between two block buffers: blk holds the block at b0, alt
    // receives the next one (or the next subcarrier's first block).  With
    // kUncondMem the prefetch is issued on every path (an empty descriptor
    // after the last subcarrier), so the number of loads in flight is the
    // same everywhere and each wait covers exactly the block consumed.
    Blk alt;
    for (int b0 = 0;; b0 += 2 * Blk::ANT) {
      const bool more1 = b0 + Blk::ANT < B;
      if (kUncondMem<IN>)
        alt.template load<true>(more1 ? cur : nxt, more1 ? b0 + Blk::ANT : 0);
      else if (more1)
        alt.template load<true>(cur, b0 + Blk::ANT);
      else if (nn < prm.n_sc)
        alt.template load<true>(nxt, 0);
      blk.template mma<true, true>(acc);
      if (!more1) {                                // odd block count: hand over
        blk = alt;
        break;
      }
      const bool more2 = b0 + 2 * Blk::ANT < B;
      if (kUncondMem<IN>)
        blk.template load<true>(more2 ? cur : nxt, more2 ? b0 + 2 * Blk::ANT : 0);
      else if (more2)
        blk.template load<true>(cur, b0 + 2 * Blk::ANT);
      else if (nn < prm.n_sc)
        blk.template load<true>(nxt, 0);
      alt.template mma<true, true>(acc);
      if (!more2) break;                           // even block count: blk holds the next
    }
    finish_mf(IN{}, acc);
    AOperand<W> at;
    float d[W];
    gram_to_operands<W>(IN{}, acc, As, Gs, Ps, AST, prm.reg, U, c, g, at, d);
    cg_llr_epilogue<W, ST, M_BITS, kUncondMem<IN>, true>(prm, n, 0, acc, at, d, Gs, Ps, c, g,
                                                         W_s[wv]);
    n = nn;
    cur = nxt;
  }
}

// All right-hand sides of subcarrier n, in chunks of 16; the Gram is
// computed with the first chunk and kept in LDS.
template <int W, typename IN, typename ST, int M_BITS>
// With all right-hand sides in one chunk (S <= 16) the LLR tile is staged in
// `stg` (A and P of the wave, contiguous, at least 16 W x 16 x M_BITS floats).
__device__ __forceinline__ void detect_one(const DetectParams& prm, int64_t n, float2* As,
                                           float2* Ps, float* Gs, int c, int g, float* stg) {
  constexpr int AST = 16 * W + 2;
  const int B = prm.B, U = prm.U, S = prm.S;
  const void* Hn = offset_sc(IN{}, prm.H, n, B, U);
  const void* Yn = offset_sc(IN{}, prm.Y, n, B, S);
  AOperand<W> at;
  float d[W];
  for (int s0 = 0; s0 < S; s0 += 16) {
    GramAcc<W> acc;
    acc.clear();
    if (s0 == 0) {
      gram_mf<W, true, true>(IN{}, Hn, Yn, B, U, S, s0, c, g, acc);
      gram_to_operands<W>(IN{}, acc, As, Gs, Ps, AST, prm.reg, U, c, g, at, d);
    } else {
      gram_mf<W, false, true>(IN{}, Hn, Yn, B, U, S, s0, c, g, acc);
    }
    if (S <= 16)
      cg_llr_epilogue<W, ST, M_BITS, kUncondMem<IN>, true>(prm, n, s0, acc, at, d, Gs, Ps, c, g,
                                                           stg);
    else
      cg_llr_epilogue<W, ST, M_BITS, kUncondMem<IN>>(prm, n, s0, acc, at, d, Gs, Ps, c, g);
  }
}

// Generic kernel (any S).
template <int W, typename IN, typename ST, int M_BITS>
__global__ __launch_bounds__(256, 2) void detect_approx_kernel(DetectParams prm) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;   // LDS row stride (complex) of A
  // per wave: A then P (float2), reused as the LLR staging tile
  constexpr int AP = 2 * (NU * AST + NU * kPST);                     // floats
  constexpr int STG = NU * 16 * M_BITS;
  __shared__ __align__(16) float W_s[kWavesPerBlock][AP > STG ? AP : STG];
  __shared__ float G_s[kWavesPerBlock][NU];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  float2* As = (float2*)W_s[wv];
  float2* Ps = As + NU * AST;
  for (int64_t n = (int64_t)blockIdx.x * kWavesPerBlock + wv; n < prm.n_sc;
       n += (int64_t)gridDim.x * kWavesPerBlock)
    detect_one<W, IN, ST, M_BITS>(prm, n, As, Ps, G_s[wv], c, g, W_s[wv]);
}

// Batched kernel: frames of different shapes (same user class, QAM order,
// storage and scalar precision) in one launch.  Frame f covers global
// subcarriers [sc_begin_f, sc_begin_f + n_sc_f); each wave finds its frame
// by a binary search over the (wave-uniform) descriptor table.
template <int W, typename IN, typename ST, int M_BITS>
__global__ __launch_bounds__(256, 2) void detect_batch_kernel(BatchArgs args) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;
  // per wave: A then P (float2), reused as the LLR staging tile
  constexpr int AP = 2 * (NU * AST + NU * kPST);                     // floats
  constexpr int STG = NU * 16 * M_BITS;
  __shared__ __align__(16) float W_s[kWavesPerBlock][AP > STG ? AP : STG];
  __shared__ float G_s[kWavesPerBlock][NU];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  float2* As = (float2*)W_s[wv];
  float2* Ps = As + NU * AST;
  for (int64_t gsc = (int64_t)blockIdx.x * kWavesPerBlock + wv; gsc < args.total;
       gsc += (int64_t)gridDim.x * kWavesPerBlock) {
    const int f = find_frame(args, gsc);
    const FrameArgs& F = args.f[f];
    DetectParams prm{F.H, F.Y, F.B, F.U, F.S, F.K, F.n_sc, F.reg, F.n0, F.es, F.scale,
                     F.inv_scale, (float*)F.out, (float2*)F.out2, nullptr, nullptr};
    if constexpr (std::is_same<IN, InC32>::value) {
      if (F.U <= 8) {               // packed form, as a single call of this frame runs
        detect_one<1, InC32P, ST, M_BITS>(prm, gsc - F.sc_begin, As, Ps, G_s[wv], c, g,
                                          W_s[wv]);
        continue;
      }
    }
    detect_one<W, IN, ST, M_BITS>(prm, gsc - F.sc_begin, As, Ps, G_s[wv], c, g, W_s[wv]);
  }
}

template <int W, typename IN, typename ST, int M>
static void launch_one(const DetectParams& p, const Schedule& sch, hipStream_t stream) {
  const dim3 grid(sched_grid(p.n_sc, sch)), block(kWave * kWavesPerBlock);
  if (p.S > 16 || sch.variant == kDetectGeneric || sch.variant == kDetectPlain)
    hipLaunchKernelGGL((detect_approx_kernel<W, IN, ST, M>), grid, block, 0, stream, p);
  else if (sch.variant == kDetectStreamSmall)
    hipLaunchKernelGGL((detect_stream_kernel<W, IN, ST, M, true>), grid, block, 0, stream, p);
  else
    hipLaunchKernelGGL((detect_stream_kernel<W, IN, ST, M, false>), grid, block, 0, stream, p);
}

template <int W, typename IN, typename ST>
static hipError_t launch_m(const DetectParams& p, int m_bits, const Schedule& sch,
                           hipStream_t stream) {
  switch (m_bits) {
    case 2: launch_one<W, IN, ST, 2>(p, sch, stream); break;
    case 4: launch_one<W, IN, ST, 4>(p, sch, stream); break;
    case 6: launch_one<W, IN, ST, 6>(p, sch, stream); break;
    case 8: launch_one<W, IN, ST, 8>(p, sch, stream); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int W, typename IN>
static hipError_t launch_st(const DetectParams& p, int f64, int m_bits, const Schedule& sch,
                            hipStream_t stream) {
  return f64 ? launch_m<W, IN, double>(p, m_bits, sch, stream)
             : launch_m<W, IN, float>(p, m_bits, sch, stream);
}

template <int W>
static hipError_t launch_in(const DetectParams& p, int in_dtype, int f64, int m_bits,
                            const Schedule& sch, hipStream_t stream) {
  switch (in_dtype) {
    case 0:
      if constexpr (W == 1)
        if (p.U <= 8) return launch_st<1, InC32P>(p, f64, m_bits, sch, stream);
      return launch_st<W, InC32>(p, f64, m_bits, sch, stream);
    case 1: return launch_st<W, InF16>(p, f64, m_bits, sch, stream);
    case 2: return launch_st<W, InBF16>(p, f64, m_bits, sch, stream);
  }
  return hipErrorInvalidValue;
}

template <int W, typename IN, typename ST>
static hipError_t launch_batch_m(const BatchArgs& a, int m_bits, const Schedule& sch,
                                 hipStream_t stream) {
  const dim3 grid(sched_grid(a.total, sch)), block(kWave * kWavesPerBlock);
  switch (m_bits) {
    case 2: hipLaunchKernelGGL((detect_batch_kernel<W, IN, ST, 2>), grid, block, 0, stream, a); break;
    case 4: hipLaunchKernelGGL((detect_batch_kernel<W, IN, ST, 4>), grid, block, 0, stream, a); break;
    case 6: hipLaunchKernelGGL((detect_batch_kernel<W, IN, ST, 6>), grid, block, 0, stream, a); break;
    case 8: hipLaunchKernelGGL((detect_batch_kernel<W, IN, ST, 8>), grid, block, 0, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int W, typename IN>
static hipError_t launch_batch_st(const BatchArgs& a, int f64, int m_bits, const Schedule& sch,
                                  hipStream_t stream) {
  return f64 ? launch_batch_m<W, IN, double>(a, m_bits, sch, stream)
             : launch_batch_m<W, IN, float>(a, m_bits, sch, stream);
}

template <int W>
static hipError_t launch_batch_in(const BatchArgs& a, int in_dtype, int f64, int m_bits,
                                  const Schedule& sch, hipStream_t stream) {
  switch (in_dtype) {
    case 0: return launch_batch_st<W, InC32>(a, f64, m_bits, sch, stream);
    case 1: return launch_batch_st<W, InF16>(a, f64, m_bits, sch, stream);
    case 2: return launch_batch_st<W, InBF16>(a, f64, m_bits, sch, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_detect_batch(const BatchArgs& a, int max_u, int in_dtype, int scalar_f64,
                               int m_bits, const Schedule& sch, hipStream_t stream) {
  if (max_u <= 16) return launch_batch_in<1>(a, in_dtype, scalar_f64, m_bits, sch, stream);
  return launch_batch_in<2>(a, in_dtype, scalar_f64, m_bits, sch, stream);
}

hipError_t launch_detect_approx(const DetectParams& p, int in_dtype, int scalar_f64, int m_bits,
                                const Schedule& sch, hipStream_t stream) {
  if (sch.variant == kDetectPlain && in_dtype == 0)
    return launch_detect_plain(p, scalar_f64, m_bits, sch, stream);
  if (p.U <= 16) return launch_in<1>(p, in_dtype, scalar_f64, m_bits, sch, stream);
  return launch_in<2>(p, in_dtype, scalar_f64, m_bits, sch, stream);
}

}  // namespace mimo

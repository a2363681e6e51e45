// One uplink + downlink slot on a reciprocal channel, fused per subcarrier:
// CG-D detection (Sec. III-B/C, Algorithm 1, eqs. (4), (13)-(15)) of the
// uplink receive vectors and CG-P precoding (Sec. III-D, eq. (16)) of the
// downlink symbol vectors of the same subcarrier, in one wavefront.
//
// With H_d = H_u^H (reciprocity, Sec. II-B) both systems have the same Gram
// matrix, G = H_u^H H_u = H_d H_d^H; they differ only in the diagonal shift:
// A_u = G + (N0/E_s) I for detection and A_d = G + beta I for precoding.  G
// is therefore formed once per subcarrier, and the subcarrier's channel,
// held in registers from the Gram to the output contraction q = H_u v
// (resident.hpp), crosses HBM once for both directions.
//
// Per subcarrier:
//   1. G and the matched filter b = H^H y (MFMA; FP32 products, or the
//      bf16-split form of gram_phase.hpp with the "fused-x3" schedule), H
//      from registers, Y streamed through a ring of NY k-steps;
//   2. downlink: K_d CG iterations on A_d v = t, ||q||, q = H_u v (MFMA),
//      output tiles staged and stored; the freed H registers receive the
//      next subcarrier's channel;
//   3. uplink: K_u CG iterations on A_u x = b with the approximate SINR
//      tracker, mu, rho and max-log LLRs, while the next subcarrier's
//      channel (and, from the LLR stage on, the first NY k-steps of its Y)
//      are in flight.
// Every step runs the same arithmetic in the same order as the detection and
// precoding kernels, so LLRs (and xhat, mu, SINR), Q and qnorm are bitwise
// those of mimo_detect_cg and mimo_precode_cg on the same inputs.
#include <type_traits>

#include "detect_core.hpp"
#include "launch.hpp"
#include "resident.hpp"

namespace mimo {

// Y rows of k-step t (antennas 4 t .. 4 t + 3) for lane (c, g): Y[4 t + g][c]
template <typename Sub>
__device__ __forceinline__ float2 load_y_step(const Sub& sb, int t) {
  return bload2(sb.ry, sb.oy, (uint32_t)(4 * t) * sb.S * 8u);
}

// 16-bit storage: the Y parts (re, im) of the 32-antenna block q for lane
// (c, g), in the operand order of Block16 (as its load with the matched
// filter reads them).
template <typename V8>
__device__ __forceinline__ void load_y_block16(const Sub16<1>& sb, int q, V8& yr, V8& yi) {
  const uint32_t kb = (uint32_t)(4 * q);              // first 8-antenna block of the step
  yr = __builtin_bit_cast(V8, bload4(sb.ry, sb.oy, kb * 2u * sb.S * 16u));
  yi = __builtin_bit_cast(V8, bload4(sb.ry, sb.oy, (kb * 2u + 1u) * sb.S * 16u));
}

template <typename IN>
struct SlotY16 {                                      // complex64 forms: Y through the ring
  static constexpr bool on = false;
  using V8 = float;
};
template <>
struct SlotY16<InF16> {
  static constexpr bool on = true;
  using V8 = h8;
};
template <>
struct SlotY16<InBF16> {
  static constexpr bool on = true;
  using V8 = bf8;
};

// Register budget.  The channel (64 VGPRs at B = 128) is held from the Gram
// to the output stage and the next subcarrier's is in flight during the
// uplink stage: 174 VGPRs with FP32 CG scalars, 2 waves per SIMD.  A 3-wave
// budget (168) costs 0-24 bytes per lane of spills with FP32 scalars and was
// faster: 226-230 against 239-241 us per 19,200 subcarriers of 128x16 at
// K = 4, 64-QAM, each at its best grid (A/B on one device, kept busy
// before each timing; 242 against 246 us with 256-QAM).  With FP64 scalars
// (92-116 bytes), the packed U <= 8 form (52-84) and the bf16-split Gram
// (24-48) the 3-wave budget spills more, so those keep 2 waves (at B <= 64
// every form fits 3 waves anyway).
template <typename IN, typename ST>
constexpr int slot_min_blocks() { return std::is_same<IN, InC32>::value && sizeof(ST) == 4 ? 3 : 2; }

template <int BMAX, typename IN, typename ST, int M_BITS>
__global__ __launch_bounds__(256, (slot_min_blocks<IN, ST>())) void slot_resident_kernel(
    SlotParams sp) {
  constexpr int NU = 16, AST = NU + 2;
  using Sub = typename Storage<IN, 1>::Sub;
  using RB = typename ResidentBlock<IN>::type;
  constexpr int NK = BMAX / RB::ANT;            // blocks of H held in registers
  constexpr int KS = RB::ANT / 4;               // k-steps (4 antennas) per block
  constexpr int NKS = BMAX / 4;                 // k-steps of Y per subcarrier
  constexpr int NY = 8;                         // k-steps of Y in flight (16, 32: no faster)
  // 16-bit storage: the whole subcarrier's Y (NK blocks, 32 VGPRs at B = 128)
  // is held like its channel instead of the complex64 ring
  constexpr bool Y16 = SlotY16<IN>::on;
  using V8 = typename SlotY16<IN>::V8;
  // per wave: A, P, the second H tile buffer and the output tile (float2),
  // reused as the uplink LLR staging tile
  constexpr int APH = 2 * (NU * AST + 2 * NU * kPST + 16 * 16);       // floats
  constexpr int STG = NU * 16 * M_BITS;
  __shared__ __align__(16) float W_s[kWavesPerBlock][APH > STG ? APH : STG];
  __shared__ float G_s[kWavesPerBlock][NU];
  __shared__ float N_s[kWavesPerBlock][16];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  float2* As = (float2*)W_s[wv];
  float2* Ps = As + NU * AST;
  float2* H2 = Ps + NU * kPST;
  float2* Qs = H2 + NU * kPST;                        // output tile of the downlink
  float* Gs = G_s[wv];
  float* Ns = N_s[wv];
  const int64_t n_sc = sp.ul.n_sc;
  const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;

  int64_t n = (int64_t)blockIdx.x * kWavesPerBlock + wv;
  RB hb[NK];
  float2 yv[Y16 ? 1 : NY];
  V8 y16r[Y16 ? NK : 1], y16i[Y16 ? NK : 1];
  Sub cur;
  if (n < n_sc) {
    const int B = sp.ul.B, U = sp.ul.U, Su = sp.ul.S;
    cur.init(offset_sc(IN{}, sp.ul.H, n, B, U), offset_sc(IN{}, sp.ul.Y, n, B, Su), B, U, Su, 0,
             c, g);
#pragma unroll
    for (int t = 0; t < NK; ++t) hb[t].template load<false, kOnceCPol>(cur, t * RB::ANT);
    if constexpr (Y16) {
#pragma unroll
      for (int q = 0; q < NK; ++q) load_y_block16(cur, q, y16r[q], y16i[q]);
    } else {
#pragma unroll
      for (int t = 0; t < NY; ++t) yv[t] = load_y_step(cur, t);
    }
  }
  while (n < n_sc) {
    const DetectParams ul = opaque_sizes(sp.ul);
    const PrecodeParams dl = opaque_sizes(sp.dl);
    const int B = ul.B, U = ul.U, Su = ul.S, Sd = dl.S;
    const int64_t nn = n + stride;
    const int64_t nc = nn < n_sc ? nn : n;            // descriptors only used if nn < n_sc
    Sub nxt;
    nxt.init(offset_sc(IN{}, ul.H, nc, B, U), offset_sc(IN{}, ul.Y, nc, B, Su), B, U, Su, 0, c,
             g);
    if (nn >= n_sc) nxt.disable();                    // last subcarrier: prefetch reads nothing
    float2 bd[1][4];                                  // downlink right-hand sides b = t
    {
      const __amdgpu_buffer_rsrc_t rt = make_rsrc(dl.T + (size_t)n * U * Sd, (uint32_t)U * Sd * 8u);
#pragma unroll
      for (int j = 0; j < 4; ++j) {                   // T[c][4 g + j]
        const int s = 4 * g + j;
        bd[0][j] = bload2(rt, (c < U && s < Sd) ? (uint32_t)(c * Sd + s) * 8u : kOOB, 0u);
      }
    }
    // ---- G = H^H H and b = H^H y (Algorithm 1, initialization)
    GramAcc<1> acc;
    acc.clear();
#pragma unroll
    for (int q = 0; q < NK; ++q) {
      if constexpr (Y16) {
        if (q * RB::ANT < B) {
          hb[q].template mma<true, false>(acc);
          RB blk = hb[q];                             // with the block's held Y parts
          blk.yr[0] = y16r[q];
          blk.yi[0] = y16i[q];
          blk.template mma<false, true>(acc);
        }
      } else {
        if (q * RB::ANT < B) {
          hb[q].template mma<true, false>(acc);
          RB blk = hb[q];                             // with the block's Y k-steps from the ring
#pragma unroll
          for (int e = 0; e < KS; ++e) blk.y[e] = yv[(q * KS + e) % NY];
          blk.template mma<false, true>(acc);
        }
#pragma unroll
        for (int e = 0; e < KS; ++e) {
          const int t = q * KS + e;
          if (t + NY < NKS) yv[t % NY] = load_y_step(cur, t + NY);
        }
      }
    }
    finish_mf(IN{}, acc);
    // A_u = G + (N0/E_s) I: A^T operand and d = diag(A_u); Gs = diag(G)
    AOperand<1> at;
    float d[1];
    gram_to_operands<1>(IN{}, acc, As, Gs, Ps, AST, ul.reg, U, c, g, at, d);
    // A_d = G + beta I: the diagonal of A_u replaced
    AOperand<1> atd = at;
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (c == 4 * t + g) atd.a[0][t] = make_float2(Gs[c] + dl.beta, 0.f);

    // ---- downlink: K_d iterations on A_d v = t, then ||q||, q = H_u v; the
    // freed H registers receive the next subcarrier's channel
    {
      CGState<1, ST> sd;
      cg_init<1, ST>(sd, bd);
      for (int k = 0; k < dl.K; ++k) {
        ST al[4], be[4];
        cg_step<1, ST>(sd, atd, Ps, c, g, al, be);
      }
      resident_output<BMAX, IN, ST>(dl, n, hb, nxt, atd, Gs, sd.v, Qs, H2, Ps, Ns, c, g, lane);
    }
    wave_lds_sync();                                  // output tiles read before reuse of LDS

    // ---- uplink: K_u iterations on A_u x = b with the tracker, then mu,
    // rho and the LLRs; the next subcarrier's first Y k-steps join its
    // channel in flight before the LLR stage
    CGState<1, ST> su;
    {
      float2 bu[1][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) bu[0][j] = make_float2(acc.dr[0][j], acc.di[0][j]);
      cg_init<1, ST>(su, bu);
    }
    Tracker<1, ST> tk;
    tk.init();
    for (int k = 0; k < ul.K; ++k) {
      ST al[4], be[4];
      cg_step<1, ST>(su, at, Ps, c, g, al, be);
      tracker_step<1, ST>(tk, d, al, be);
    }
    if constexpr (Y16) {
#pragma unroll
      for (int q = 0; q < NK; ++q) load_y_block16(nxt, q, y16r[q], y16i[q]);
    } else {
#pragma unroll
      for (int t = 0; t < NY; ++t) yv[t] = load_y_step(nxt, t);
    }
    llr_stage<1, ST, M_BITS, true, true>(ul, n, 0, su.v, tk.tv, Gs, c, g, W_s[wv]);
    n = nn;
    cur = nxt;
  }
}

bool slot_eligible(const SlotParams& p, int in_dtype) {
  return in_dtype >= 0 && in_dtype <= 2 && p.ul.U <= 16 && p.ul.S <= 16 && p.dl.S <= 16 &&
         p.ul.B <= 128;
}

template <int BMAX, typename IN, typename ST>
static hipError_t launch_m(const SlotParams& p, int m_bits, const Schedule& sch,
                           hipStream_t stream) {
  const dim3 grid(sched_grid(p.ul.n_sc, sch)), block(kWave * kWavesPerBlock);
  switch (m_bits) {
    case 2: hipLaunchKernelGGL((slot_resident_kernel<BMAX, IN, ST, 2>), grid, block, 0, stream, p); break;
    case 4: hipLaunchKernelGGL((slot_resident_kernel<BMAX, IN, ST, 4>), grid, block, 0, stream, p); break;
    case 6: hipLaunchKernelGGL((slot_resident_kernel<BMAX, IN, ST, 6>), grid, block, 0, stream, p); break;
    case 8: hipLaunchKernelGGL((slot_resident_kernel<BMAX, IN, ST, 8>), grid, block, 0, stream, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename IN, typename ST>
static hipError_t launch_b(const SlotParams& p, int m_bits, const Schedule& sch,
                           hipStream_t stream) {
  return p.ul.B <= 64 ? launch_m<64, IN, ST>(p, m_bits, sch, stream)
                      : launch_m<128, IN, ST>(p, m_bits, sch, stream);
}

template <typename IN>
static hipError_t launch_st(const SlotParams& p, int f64, int m_bits, const Schedule& sch,
                            hipStream_t stream) {
  return f64 ? launch_b<IN, double>(p, m_bits, sch, stream)
             : launch_b<IN, float>(p, m_bits, sch, stream);
}

hipError_t launch_slot(const SlotParams& p, int in_dtype, int scalar_f64, int m_bits,
                       const Schedule& sch, hipStream_t stream) {
  if (in_dtype == 1) return launch_st<InF16>(p, scalar_f64, m_bits, sch, stream);
  if (in_dtype == 2) return launch_st<InBF16>(p, scalar_f64, m_bits, sch, stream);
  if (sch.variant == kSlotFusedX3) return launch_st<InC32X3>(p, scalar_f64, m_bits, sch, stream);
  if (p.ul.U <= 8) return launch_st<InC32P>(p, scalar_f64, m_bits, sch, stream);
  return launch_st<InC32>(p, scalar_f64, m_bits, sch, stream);
}

}  // namespace mimo

// Fused CG-P kernel (Sec. III-D): Gram on MFMA, K CG iterations on
// (H_d H_d^H + beta I) v = t, then q = H_d^H v = H_u v on MFMA, with the
// optional power normalization s = q / ||q|| (Sec. II-B).  One wavefront per
// subcarrier.
//
// ||q||^2 = v^H H^H H v = v^H G v is formed in the CG layout from one more
// mat-vec (with G), so each output tile is written once, already scaled.
#include <type_traits>

// H is read twice per launch here (or once per iteration): keep its lines in
// the caches (default policy for every buffer access).
#define MIMO_CACHE_STREAMING 0
#include "launch.hpp"
#include "precode_out.hpp"
#include "resident.hpp"

namespace mimo {

// All right-hand sides of subcarrier n (chunks of 16; the Gram with the
// first chunk).
template <int W, typename IN, typename ST>
__device__ __forceinline__ void precode_one(const PrecodeParams& prm, int64_t n, float2* As,
                                            float2* Ps, float* Gs, float* Ns, int c, int g) {
  constexpr int AST = 16 * W + 2;
  const int B = prm.B, U = prm.U, S = prm.S;
  const float beta = prm.beta;
  const void* Hn = offset_sc(IN{}, prm.H, n, B, U);
  AOperand<W> at;
  for (int s0 = 0; s0 < S; s0 += 16) {
    // ---- A = H_d H_d^H + beta I = G + beta I (Algorithm 1, initialization)
    if (s0 == 0) {
      if (prm.gram) {                 // cached G: H is read only for q = H v
        load_cached_gram<W>(prm.gram + (size_t)n * U * U, U, beta, As, Gs, AST, 16 * g + c);
      } else {
        GramAcc<W> acc;
        acc.clear();
        gram_mf<W, true, false>(IN{}, Hn, nullptr, B, U, S, 0, c, g, acc);
        store_gram(IN{}, acc, As, Gs, (float*)Ps, AST, beta, c, g);
      }
      wave_lds_sync();
      at.load(As, AST, c, g, U);
    }
    // b = t
    float2 b[W][4];
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int u = 16 * w + c, s = s0 + 4 * g + j;
        b[w][j] = (u < U && s < S) ? prm.T[((size_t)n * U + u) * S + s] : make_float2(0.f, 0.f);
      }

    CGState<W, ST> st;
    cg_init<W, ST>(st, b);
    for (int k = 0; k < prm.K; ++k) {
      ST al[4], be[4];
      cg_step<W, ST>(st, at, Ps, c, g, al, be);
    }

    precode_store<W, IN, ST>(prm, n, s0, Hn, st.v, at, Gs, Ps, Ns, c, g);
    wave_lds_sync();
  }
}

template <int W, typename IN, typename ST>
__global__ __launch_bounds__(256, 2) void precode_kernel(PrecodeParams prm) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;
  __shared__ __align__(16) float2 A_s[kWavesPerBlock][NU * AST];
  __shared__ __align__(16) float2 P_s[kWavesPerBlock][NU * kPST];
  __shared__ float G_s[kWavesPerBlock][NU];
  __shared__ float N_s[kWavesPerBlock][16];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  for (int64_t n = (int64_t)blockIdx.x * kWavesPerBlock + wv; n < prm.n_sc;
       n += (int64_t)gridDim.x * kWavesPerBlock)
    precode_one<W, IN, ST>(opaque_sizes(prm), n, A_s[wv], P_s[wv], G_s[wv], N_s[wv], c, g);
}

// Streaming kernel for S <= 16 (one right-hand-side chunk): the Gram's H
// blocks ping-pong between two register buffers with the next block's loads
// in flight during the current block's MFMAs, and the first block of the
// wave's next subcarrier is issued before the CG and output stages of the
// current one.  Loads are issued on every path (an empty descriptor after
// the last subcarrier), so the compiler's load-counter waits cover exactly
// the block consumed.  Same arithmetic in the same order as precode_one.
// CACHED: A from the cached Gram matrix prm.gram; no block loads at all (H is
// read only for q = H v), as precode_one's cached branch.
template <int W, typename IN, typename ST, bool SMALL, bool CACHED = false>
__global__ __launch_bounds__(256, 2) void precode_stream_kernel(PrecodeParams kprm) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;
  using Sub = typename Storage<IN, W>::Sub;
  using Blk = typename std::conditional<SMALL, typename Storage<IN, W>::SmallBlock,
                                        typename Storage<IN, W>::Block>::type;
  __shared__ __align__(16) float2 A_s[kWavesPerBlock][NU * AST];
  __shared__ __align__(16) float2 P_s[kWavesPerBlock][NU * kPST];
  __shared__ float G_s[kWavesPerBlock][NU];
  __shared__ float N_s[kWavesPerBlock][16];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  float2* As = A_s[wv];
  float2* Ps = P_s[wv];
  float* Gs = G_s[wv];
  float* Ns = N_s[wv];
  const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;

  int64_t n = (int64_t)blockIdx.x * kWavesPerBlock + wv;
  Sub cur;
  Blk blk;
  if (n < kprm.n_sc) {
    cur.init(offset_sc(IN{}, kprm.H, n, kprm.B, kprm.U), nullptr, kprm.B, kprm.U, kprm.S, 0, c, g);
    if constexpr (!CACHED) blk.template load<false>(cur, 0);
  }
  while (n < kprm.n_sc) {
    const PrecodeParams prm = opaque_sizes(kprm);
    const int B = prm.B, U = prm.U, S = prm.S;
    const int64_t nn = n + stride;
    const int64_t nc = nn < prm.n_sc ? nn : n;
    Sub nxt;
    nxt.init(offset_sc(IN{}, prm.H, nc, B, U), nullptr, B, U, S, 0, c, g);
    if (nn >= prm.n_sc) nxt.disable();
    const void* Hn = offset_sc(IN{}, prm.H, n, B, U);
    // ---- A = H_d H_d^H + beta I = G + beta I (Algorithm 1, initialization)
    if constexpr (CACHED) {
      load_cached_gram<W>(prm.gram + (size_t)n * U * U, U, prm.beta, As, Gs, AST, lane);
    } else {
      GramAcc<W> acc;
      acc.clear();
      Blk alt;
      // pairs of blocks; an odd count's last partner lies past B and reads
      // zero, adding exact zeros (one loop exit, so nothing after the Gram
      // waits for the next subcarrier's block in flight)
      for (int b0 = 0;; b0 += 2 * Blk::ANT) {
        alt.template load<false>(cur, b0 + Blk::ANT);
        blk.template mma<true, false>(acc);
        const bool more2 = b0 + 2 * Blk::ANT < B;
        blk.template load<false>(more2 ? cur : nxt, more2 ? b0 + 2 * Blk::ANT : 0);
        alt.template mma<true, false>(acc);
        if (!more2) break;
      }
      store_gram(IN{}, acc, As, Gs, (float*)Ps, AST, prm.beta, c, g);
    }
    wave_lds_sync();
    AOperand<W> at;
    at.load(As, AST, c, g, U);
    float2 b[W][4];                                   // b = t
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int u = 16 * w + c, s = 4 * g + j;
        b[w][j] = (u < U && s < S) ? prm.T[((size_t)n * U + u) * S + s] : make_float2(0.f, 0.f);
      }
    CGState<W, ST> st;
    cg_init<W, ST>(st, b);
    for (int k = 0; k < prm.K; ++k) {
      ST al[4], be[4];
      cg_step<W, ST>(st, at, Ps, c, g, al, be);
    }
    precode_store<W, IN, ST>(prm, n, 0, Hn, st.v, at, Gs, Ps, Ns, c, g, As);
    wave_lds_sync();
    n = nn;
    cur = nxt;
  }
}


// H-resident kernel (U <= 16, S <= 16, B <= BMAX; resident.hpp): a
// subcarrier's channel stays in registers from the Gram to the output
// contraction, so H crosses HBM once (the other kernels read it a second
// time for q = H v).  Same arithmetic in the same order as precode_one.
//
// Occupancy the register budget is sized for: 3 waves per SIMD (H takes 64
// VGPRs at B = 128 in complex64, 32 in 16-bit storage, where 4 waves would
// spill), 2 with FP64 scalars.
template <typename ST>
constexpr int resident_min_blocks() { return sizeof(ST) == 8 ? 2 : 3; }

// CACHED: A from the cached Gram matrix prm.gram; H is still held for q = H v.
template <int BMAX, typename IN, typename ST, bool CACHED = false>
__global__ __launch_bounds__(256, resident_min_blocks<ST>()) void precode_resident_kernel(
    PrecodeParams kprm) {
  constexpr int NU = 16, AST = NU + 2;
  using Sub = typename Storage<IN, 1>::Sub;
  using RB = typename ResidentBlock<IN>::type;
  constexpr int NK = BMAX / RB::ANT;            // k-steps held in registers
  __shared__ __align__(16) float2 A_s[kWavesPerBlock][NU * AST];
  __shared__ __align__(16) float2 P_s[kWavesPerBlock][NU * kPST];
  __shared__ __align__(16) float2 H2_s[kWavesPerBlock][NU * kPST];
  __shared__ float G_s[kWavesPerBlock][NU];
  __shared__ float N_s[kWavesPerBlock][16];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  float2* As = A_s[wv];
  float2* Ps = P_s[wv];
  float2* H2 = H2_s[wv];
  float* Gs = G_s[wv];
  float* Ns = N_s[wv];
  const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
  uint32_t ot[4];                                                      // T[c][4 g + j]
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int s = 4 * g + j;
    ot[j] = (c < kprm.U && s < kprm.S) ? (uint32_t)(c * kprm.S + s) * 8u : kOOB;
  }

  int64_t n = (int64_t)blockIdx.x * kWavesPerBlock + wv;
  RB hb[NK];
  if (n < kprm.n_sc) {
    Sub cur;
    cur.init(offset_sc(IN{}, kprm.H, n, kprm.B, kprm.U), nullptr, kprm.B, kprm.U, kprm.S, 0, c, g);
#pragma unroll
    for (int t = 0; t < NK; ++t) hb[t].template load<false, kOnceCPol>(cur, t * RB::ANT);
  }
  while (n < kprm.n_sc) {
    const PrecodeParams prm = opaque_sizes(kprm);
    const int B = prm.B, U = prm.U, S = prm.S;
    const int64_t nn = n + stride;
    float2 b[1][4];                                   // b = t
    {
      const __amdgpu_buffer_rsrc_t rt = make_rsrc(prm.T + (size_t)n * U * S, (uint32_t)U * S * 8u);
#pragma unroll
      for (int j = 0; j < 4; ++j) b[0][j] = bload2(rt, ot[j], 0u);
    }
    // ---- A = H_d H_d^H + beta I = G + beta I (Algorithm 1, initialization)
    if constexpr (CACHED) {
      load_cached_gram<1>(prm.gram + (size_t)n * U * U, U, prm.beta, As, Gs, AST, lane);
    } else {
      GramAcc<1> acc;
      acc.clear();
#pragma unroll
      for (int t = 0; t < NK; ++t)
        if (t * RB::ANT < B) hb[t].template mma<true, false>(acc);
      store_gram(IN{}, acc, As, Gs, (float*)Ps, AST, prm.beta, c, g);
    }
    wave_lds_sync();
    AOperand<1> at;
    at.load(As, AST, c, g, U);
    CGState<1, ST> st;
    cg_init<1, ST>(st, b);
    for (int k = 0; k < prm.K; ++k) {
      ST al[4], be[4];
      cg_step<1, ST>(st, at, Ps, c, g, al, be);
    }

    Sub nxt;                                          // empty past the last subcarrier
    nxt.init(offset_sc(IN{}, prm.H, nn < prm.n_sc ? nn : n, B, U), nullptr, B, U, S, 0, c, g);
    if (nn >= prm.n_sc) nxt.disable();
    resident_output<BMAX, IN, ST>(prm, n, hb, nxt, at, Gs, st.v, As, H2, Ps, Ns, c, g, lane);
    wave_lds_sync();
    n = nn;
  }
}

// Whether the H-resident kernel covers a launch.
template <int W>
static bool resident_fits(const PrecodeParams& p) {
  return W == 1 && p.S <= 16 && p.B <= 128;
}

// Batched kernel: frames of different shapes in one launch (see detect.hip).
template <int W, typename IN, typename ST>
__global__ __launch_bounds__(256, 2) void precode_batch_kernel(BatchArgs args) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;
  __shared__ __align__(16) float2 A_s[kWavesPerBlock][NU * AST];
  __shared__ __align__(16) float2 P_s[kWavesPerBlock][NU * kPST];
  __shared__ float G_s[kWavesPerBlock][NU];
  __shared__ float N_s[kWavesPerBlock][16];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  for (int64_t gsc = (int64_t)blockIdx.x * kWavesPerBlock + wv; gsc < args.total;
       gsc += (int64_t)gridDim.x * kWavesPerBlock) {
    const int f = find_frame(args, gsc);
    const FrameArgs& F = args.f[f];
    PrecodeParams prm{F.H, (const float2*)F.Y, F.B, F.U, F.S, F.K, F.n_sc, F.beta,
                      F.normalize, (float2*)F.out, (float*)F.out2, (const float2*)F.gram};
    if constexpr (std::is_same<IN, InC32>::value) {
      if (F.U <= 8) {               // packed form, as a single call of this frame runs
        precode_one<1, InC32P, ST>(prm, gsc - F.sc_begin, A_s[wv], P_s[wv], G_s[wv], N_s[wv], c,
                                   g);
        continue;
      }
    }
    precode_one<W, IN, ST>(prm, gsc - F.sc_begin, A_s[wv], P_s[wv], G_s[wv], N_s[wv], c, g);
  }
}

template <int W, typename IN, typename ST>
static void launch_one(const PrecodeParams& p, const Schedule& sch, hipStream_t stream) {
  const dim3 grid(sched_grid(p.n_sc, sch)), block(kWave * kWavesPerBlock);
  if (p.gram && p.S <= 16 && sch.variant != kPrecodeGeneric) {   // cached Gram
    if (sch.variant == kPrecodeResident && resident_fits<W>(p)) {
      if (p.B <= 64)
        hipLaunchKernelGGL((precode_resident_kernel<64, IN, ST, true>), grid, block, 0, stream, p);
      else
        hipLaunchKernelGGL((precode_resident_kernel<128, IN, ST, true>), grid, block, 0, stream,
                           p);
    } else if (sch.variant == kPrecodeStream) {
      hipLaunchKernelGGL((precode_stream_kernel<W, IN, ST, false, true>), grid, block, 0, stream,
                         p);
    } else {
      hipLaunchKernelGGL((precode_stream_kernel<W, IN, ST, true, true>), grid, block, 0, stream,
                         p);
    }
  } else if (sch.variant == kPrecodeResident && resident_fits<W>(p)) {
    if (p.B <= 64)
      hipLaunchKernelGGL((precode_resident_kernel<64, IN, ST>), grid, block, 0, stream, p);
    else
      hipLaunchKernelGGL((precode_resident_kernel<128, IN, ST>), grid, block, 0, stream, p);
  } else if (p.S > 16 || sch.variant == kPrecodeGeneric)
    hipLaunchKernelGGL((precode_kernel<W, IN, ST>), grid, block, 0, stream, p);
  else if (sch.variant == kPrecodeStreamSmall)
    hipLaunchKernelGGL((precode_stream_kernel<W, IN, ST, true>), grid, block, 0, stream, p);
  else
    hipLaunchKernelGGL((precode_stream_kernel<W, IN, ST, false>), grid, block, 0, stream, p);
}

template <int W, typename IN>
static hipError_t launch_st(const PrecodeParams& p, int f64, const Schedule& sch,
                            hipStream_t stream) {
  if (f64)
    launch_one<W, IN, double>(p, sch, stream);
  else
    launch_one<W, IN, float>(p, sch, stream);
  return hipGetLastError();
}

template <int W>
static hipError_t launch_in(const PrecodeParams& p, int in_dtype, int f64, const Schedule& sch,
                            hipStream_t stream) {
  switch (in_dtype) {
    case 0:
      if (sch.variant == kPrecodeX3)   // bf16-split Gram: resident kernel where it fits
        return launch_st<W, InC32X3>(p, f64, Schedule{kPrecodeResident, sch.blocks_per_cu},
                                     stream);
      if constexpr (W == 1)
        if (p.U <= 8) return launch_st<1, InC32P>(p, f64, sch, stream);
      return launch_st<W, InC32>(p, f64, sch, stream);
    case 1: return launch_st<W, InF16>(p, f64, sch, stream);
    case 2: return launch_st<W, InBF16>(p, f64, sch, stream);
  }
  return hipErrorInvalidValue;
}

template <int W, typename IN>
static hipError_t launch_batch_st(const BatchArgs& a, int f64, const Schedule& sch,
                                  hipStream_t stream) {
  const dim3 grid(sched_grid(a.total, sch)), block(kWave * kWavesPerBlock);
  if (f64)
    hipLaunchKernelGGL((precode_batch_kernel<W, IN, double>), grid, block, 0, stream, a);
  else
    hipLaunchKernelGGL((precode_batch_kernel<W, IN, float>), grid, block, 0, stream, a);
  return hipGetLastError();
}

template <int W>
static hipError_t launch_batch_in(const BatchArgs& a, int in_dtype, int f64, const Schedule& sch,
                                  hipStream_t stream) {
  switch (in_dtype) {
    case 0: return launch_batch_st<W, InC32>(a, f64, sch, stream);
    case 1: return launch_batch_st<W, InF16>(a, f64, sch, stream);
    case 2: return launch_batch_st<W, InBF16>(a, f64, sch, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_precode_batch(const BatchArgs& a, int max_u, int in_dtype, int scalar_f64,
                                const Schedule& sch, hipStream_t stream) {
  if (max_u <= 16) return launch_batch_in<1>(a, in_dtype, scalar_f64, sch, stream);
  return launch_batch_in<2>(a, in_dtype, scalar_f64, sch, stream);
}

hipError_t launch_precode(const PrecodeParams& p, int in_dtype, int scalar_f64,
                          const Schedule& sch, hipStream_t stream) {
  // a cached Gram runs the generic, streaming or resident kernels (the bf16-split
  // form has no Gram to split: resident; split: stream-small)
  if (p.gram && (sch.variant == kPrecodeSplit || sch.variant == kPrecodeX3))
    return launch_precode(p, in_dtype, scalar_f64,
                          Schedule{sch.variant == kPrecodeX3 ? kPrecodeResident
                                                             : kPrecodeStreamSmall,
                                   sch.blocks_per_cu},
                          stream);
  if (sch.variant == kPrecodeSplit) {
    if (split_eligible(in_dtype, p.U, p.S, p.B, true))
      return launch_precode_split(p, scalar_f64, sch, stream);
    return launch_precode(p, in_dtype, scalar_f64,
                          Schedule{kPrecodeStreamSmall, sch.blocks_per_cu}, stream);
  }
  if (p.U <= 16) return launch_in<1>(p, in_dtype, scalar_f64, sch, stream);
  return launch_in<2>(p, in_dtype, scalar_f64, sch, stream);
}

}  // namespace mimo

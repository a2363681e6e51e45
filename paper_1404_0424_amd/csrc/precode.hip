// Fused CG-P kernel (Sec. III-D): Gram on MFMA, K CG iterations on
// (H_d H_d^H + beta I) v = t, then q = H_d^H v = H_u v on MFMA, with the
// optional power normalization s = q / ||q|| (Sec. II-B).  One wavefront per
// subcarrier.
//
// ||q||^2 = v^H H^H H v = v^H G v is formed in the CG layout from one more
// mat-vec with A (v^H A v - beta ||v||^2), so each output tile is written
// once, already scaled.
#include <type_traits>

#include "launch.hpp"
#include "precode_out.hpp"

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
      GramAcc<W> acc;
      acc.clear();
      gram_mf<W, true, false>(IN{}, Hn, nullptr, B, U, S, 0, c, g, acc);
      store_gram_lds<W>(acc, As, Gs, (float*)Ps, AST, beta, c, g);
      wave_lds_sync();
      at.load(As, AST, c, g);
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

    precode_store<W, IN, ST>(prm, n, s0, Hn, st.v, at, Ps, Ns, c, g);
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
    precode_one<W, IN, ST>(prm, n, A_s[wv], P_s[wv], G_s[wv], N_s[wv], c, g);
}

// Streaming kernel for S <= 16 (one right-hand-side chunk): the Gram's H
// blocks ping-pong between two register buffers with the next block's loads
// in flight during the current block's MFMAs, and the first block of the
// wave's next subcarrier is issued before the CG and output stages of the
// current one.  Loads are issued on every path (an empty descriptor after
// the last subcarrier), so the compiler's load-counter waits cover exactly
// the block consumed.  Same arithmetic in the same order as precode_one.
template <int W, typename IN, typename ST, bool SMALL>
__global__ __launch_bounds__(256, 2) void precode_stream_kernel(PrecodeParams prm) {
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
  const int B = prm.B, U = prm.U, S = prm.S;
  const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;

  int64_t n = (int64_t)blockIdx.x * kWavesPerBlock + wv;
  Sub cur;
  Blk blk;
  if (n < prm.n_sc) {
    cur.init(offset_sc(IN{}, prm.H, n, B, U), nullptr, B, U, S, 0, c, g);
    blk.template load<false>(cur, 0);
  }
  while (n < prm.n_sc) {
    const int64_t nn = n + stride;
    const int64_t nc = nn < prm.n_sc ? nn : n;
    Sub nxt;
    nxt.init(offset_sc(IN{}, prm.H, nc, B, U), nullptr, B, U, S, 0, c, g);
    if (nn >= prm.n_sc) nxt.disable();
    const void* Hn = offset_sc(IN{}, prm.H, n, B, U);
    // ---- A = H_d H_d^H + beta I = G + beta I (Algorithm 1, initialization)
    GramAcc<W> acc;
    acc.clear();
    Blk alt;
    for (int b0 = 0;; b0 += 2 * Blk::ANT) {
      const bool more1 = b0 + Blk::ANT < B;
      alt.template load<false>(more1 ? cur : nxt, more1 ? b0 + Blk::ANT : 0);
      blk.template mma<true, false>(acc);
      if (!more1) {
        blk = alt;
        break;
      }
      const bool more2 = b0 + 2 * Blk::ANT < B;
      blk.template load<false>(more2 ? cur : nxt, more2 ? b0 + 2 * Blk::ANT : 0);
      alt.template mma<true, false>(acc);
      if (!more2) break;
    }
    store_gram_lds<W>(acc, As, Gs, (float*)Ps, AST, prm.beta, c, g);
    wave_lds_sync();
    AOperand<W> at;
    at.load(As, AST, c, g);
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
    precode_store<W, IN, ST>(prm, n, 0, Hn, st.v, at, Ps, Ns, c, g);
    wave_lds_sync();
    n = nn;
    cur = nxt;
  }
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
                      F.normalize, (float2*)F.out, (float*)F.out2};
    precode_one<W, IN, ST>(prm, gsc - F.sc_begin, A_s[wv], P_s[wv], G_s[wv], N_s[wv], c, g);
  }
}

template <int W, typename IN, typename ST>
static void launch_one(const PrecodeParams& p, const Schedule& sch, hipStream_t stream) {
  const dim3 grid(sched_grid(p.n_sc, sch)), block(kWave * kWavesPerBlock);
  if (p.S > 16 || sch.variant == kPrecodeGeneric)
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
    case 0: return launch_st<W, InC32>(p, f64, sch, stream);
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
  if (p.U <= 16) return launch_in<1>(p, in_dtype, scalar_f64, sch, stream);
  return launch_in<2>(p, in_dtype, scalar_f64, sch, stream);
}

}  // namespace mimo

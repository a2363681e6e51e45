// Comparison detectors and precoders of Sec. III-F: the exact soft-output
// MMSE detector and MMSE / ZF precoder through the Cholesky factorization
// (Sec. III-F-1), and the truncated Neumann-series approximation of the
// inverse (Sec. III-F-2).  One wavefront (one block) per subcarrier: Gram
// and matched filter on MFMA as in CG-D, the explicit (approximate) inverse
// X of A in LDS, then xhat = X b on MFMA with the soft output of the linear
// detector W = X H^H (eqs. (2)-(4)), or v = X t and q = H_u v (eq. (5)).
// H is read twice per launch here (or once per iteration): keep its lines in
// the caches (default policy for every buffer access).
#define MIMO_CACHE_STREAMING 0
#include "gram_stream.hpp"
#include "inverse.hpp"
#include "launch.hpp"
#include "llr.hpp"
#include "precode_out.hpp"

namespace mimo {

template <int W>
struct InverseLds {
  static constexpr int NU = 16 * W, AST = NU + 2;
  __align__(16) float2 A[NU * AST];    // A = G + reg I (padding block: identity)
  __align__(16) float2 X[NU * AST];    // explicit (approximate) inverse
  __align__(16) float2 P[NU * kPST];   // mat-vec staging / Gram scratch
  __align__(16) float2 xch[4 * NU];    // Cholesky exchange buffers
  float G[NU];                         // raw diagonal G_ii
  float Dinv[NU];                      // (A^{-1})_ii (Cholesky)
  float MU[NU], RHO[NU];               // per-user gain and SINR (detection)
  float N[16];                         // ||q||^2 of the chunk (precoding)
};

template <int W, int METHOD>
__device__ __forceinline__ void build_inverse(InverseLds<W>& sm, int U, int K, int lane, int c,
                                              int g) {
  constexpr int AST = InverseLds<W>::AST;
  pad_unit_diagonal<W>(sm.A, AST, U, lane);
  wave_lds_sync();
  if (METHOD == kInvCholesky)
    cholesky_full_inverse<W>(sm.A, sm.X, sm.Dinv, (float*)sm.P, sm.xch, AST, U, c, g);
  else
    neumann_series<W>(sm.A, sm.X, AST, K, lane, c, g);
}

// e = X x for x in the CG lane layout (user 16 w + c, rhs 4 g + j).
template <int W>
__device__ __forceinline__ void apply_inverse(InverseLds<W>& sm, const float2 (&x)[W][4], int c,
                                              int g, float2 (&e)[W][4]) {
  stage_vec<W>(sm.P, c, g, x);
  wave_lds_sync();
  AOperand<W> xo;
  xo.load(sm.X, InverseLds<W>::AST, c, g, 16 * W);
  matvec_mfma<W>(xo, sm.P, c, g, e);
  wave_lds_sync();
}

// After the Gram phase of chunk s0 (acc: Gram tiles on the first chunk, the
// matched filter b of rhs s0 .. s0 + 15): on the first chunk build X and the
// per-user gain and SINR, then xhat = X b and the LLRs of the chunk.
// STAGE (streaming form, one chunk): the subcarrier's LLR tile is assembled in
// A, X and P (contiguous, dead once xhat is formed) and written in contiguous
// pieces, as the CG detectors do, when it fits there.
template <int W, int M_BITS, int METHOD, bool STAGE = false>
__device__ __forceinline__ void detect_inverse_chunk(const DetectParams& prm, InverseLds<W>& sm,
                                                     int64_t n, int s0, const GramAcc<W>& acc,
                                                     int lane, int c, int g) {
  constexpr int AST = InverseLds<W>::AST;
  constexpr int kStageFloats = 2 * (2 * InverseLds<W>::NU * AST + InverseLds<W>::NU * kPST);
  const int U = prm.U, S = prm.S;
  const int total = U * S * M_BITS;                  // floats of the subcarrier's LLR tile
  const bool stage = STAGE && total <= kStageFloats;
  float* stg = (float*)sm.A;
  if (s0 == 0) {
    store_gram_lds<W>(acc, sm.A, sm.G, (float*)sm.P, AST, prm.reg, c, g);
    wave_lds_sync();
    build_inverse<W, METHOD>(sm, U, prm.K, lane, c, g);
    if (METHOD == kInvCholesky) {
      // unbiased MMSE: mu_i = (A^{-1} G)_ii = 1 - (N0/E_s)(A^{-1})_ii and
      // rho_i = mu_i^2 / nu_i^2 = mu_i / (N0 (A^{-1})_ii)
      if (lane < U) {
        const float d = sm.Dinv[lane];
        const float mu = 1.f - prm.reg * d;
        sm.MU[lane] = mu;
        sm.RHO[lane] = mu / (prm.n0 * d);
      }
    } else {
      linear_sinr<W>(sm.A, sm.G, sm.X, AST, prm.es, prm.n0, c, g, sm.MU, sm.RHO);
    }
    wave_lds_sync();
  }
  float2 b[W][4], x[W][4];
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int j = 0; j < 4; ++j) b[w][j] = make_float2(acc.dr[w][j], acc.di[w][j]);
  apply_inverse<W>(sm, b, c, g, x);                      // xhat = X H^H y
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int u = 16 * w + c;
    const int uu = u < U ? u : 0;
    const float mu = sm.MU[uu];
    // mu = 0 (a zero channel column): z = 0 and rho = G_ii / N0
    const bool live = fabsf(mu) >= __FLT_MIN__;
    const float rho = live ? sm.RHO[uu] : sm.G[uu] / prm.n0;
    const float imu = live ? __builtin_amdgcn_rcpf(mu) : 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int s = s0 + 4 * g + j;
      const float2 xx = x[w][j];
      float out[M_BITS];
      llr_maxlog<M_BITS>(make_float2(xx.x * imu, xx.y * imu), rho, prm.scale, prm.inv_scale,
                         out);
      if (u < U && s < S) {
        const size_t idx = ((size_t)n * U + u) * S + s;
        float* lp = stage ? stg + (u * S + s) * M_BITS : prm.llr + idx * M_BITS;
#pragma unroll
        for (int q = 0; q < M_BITS; ++q) lp[q] = out[q];
        if (prm.xhat) prm.xhat[idx] = xx;
        if (prm.mu) prm.mu[idx] = mu;
        if (prm.sinr) prm.sinr[idx] = rho;
      }
    }
  }
  if (stage) {
    wave_lds_sync();
    const __amdgpu_buffer_rsrc_t rl = make_rsrc(prm.llr + (size_t)n * total, (uint32_t)total * 4u);
    if ((total & 3) == 0) {
      const float4* src = (const float4*)stg;
      for (int o = lane; o < total / 4; o += kWave) {
        const float4 v = src[o];
        bstore4(rl, (uint32_t)o * 16u, v.x, v.y, v.z, v.w);
      }
    } else {
      const float2* src = (const float2*)stg;
      for (int o = lane; o < total / 2; o += kWave) {
        const float2 v = src[o];
        bstore2(rl, (uint32_t)o * 8u, v.x, v.y);
      }
    }
    wave_lds_sync();
  }
}

// Generic form (any S): one subcarrier per block in turn, rhs in chunks of 16.
template <int W, typename IN, int M_BITS, int METHOD>
__global__ __launch_bounds__(64) void detect_inverse_kernel(DetectParams prm) {
  __shared__ InverseLds<W> sm;
  const int lane = threadIdx.x;
  const int c = lane & 15, g = lane >> 4;
  const int B = prm.B, U = prm.U, S = prm.S;
  for (int64_t n = blockIdx.x; n < prm.n_sc; n += gridDim.x) {
    const void* Hn = offset_sc(IN{}, prm.H, n, B, U);
    const void* Yn = offset_sc(IN{}, prm.Y, n, B, S);
    for (int s0 = 0; s0 < S; s0 += 16) {
      GramAcc<W> acc;
      acc.clear();
      if (s0 == 0)
        gram_mf<W, true, true>(IN{}, Hn, Yn, B, U, S, 0, c, g, acc);
      else
        gram_mf<W, false, true>(IN{}, Hn, Yn, B, U, S, s0, c, g, acc);
      detect_inverse_chunk<W, M_BITS, METHOD>(prm, sm, n, s0, acc, lane, c, g);
    }
  }
}

// Streaming form for S <= 16: a persistent grid in which each wavefront
// walks several subcarriers with the Gram's loads streamed (gram_stream).
// Same arithmetic in the same order as detect_inverse_kernel.
template <int W, typename IN, int M_BITS, int METHOD>
__global__ __launch_bounds__(64, W == 2 ? 1 : (METHOD == kInvCholesky ? 4 : 3)) void detect_inverse_stream_kernel(DetectParams kprm) {
  using Sub = typename Storage<IN, W>::Sub;
  using Blk = typename Storage<IN, W>::SmallBlock;
  __shared__ InverseLds<W> sm;
  const int lane = threadIdx.x;
  const int c = lane & 15, g = lane >> 4;
  int64_t n = blockIdx.x;
  Sub cur;
  Blk blk;
  if (n < kprm.n_sc) {
    const int B = kprm.B, U = kprm.U, S = kprm.S;
    cur.init(offset_sc(IN{}, kprm.H, n, B, U), offset_sc(IN{}, kprm.Y, n, B, S), B, U, S, 0, c,
             g);
    blk.template load<true>(cur, 0);
  }
  while (n < kprm.n_sc) {
    const DetectParams prm = opaque_sizes(kprm);
    const int B = prm.B, U = prm.U, S = prm.S;
    const int64_t nn = n + gridDim.x;
    const int64_t nc = nn < prm.n_sc ? nn : n;
    Sub nxt;
    nxt.init(offset_sc(IN{}, prm.H, nc, B, U), offset_sc(IN{}, prm.Y, nc, B, S), B, U, S, 0, c, g);
    if (nn >= prm.n_sc) nxt.disable();
    GramAcc<W> acc;
    acc.clear();
    gram_stream<W, true>(IN{}, blk, cur, nxt, B, acc);
    // staged LLR stores where they measured faster (Neumann); at 4 waves per
    // SIMD they make the Cholesky kernel spill
    detect_inverse_chunk<W, M_BITS, METHOD, METHOD == kInvNeumann>(prm, sm, n, 0, acc, lane, c,
                                                                    g);
    n = nn;
    cur = nxt;
  }
}

// Precoding after the Gram phase: X on the first chunk, then v = X t and the
// shared output stage for rhs s0 .. s0 + 15.
template <int W, typename IN, int METHOD>
__device__ __forceinline__ void precode_inverse_chunk(const PrecodeParams& prm,
                                                      InverseLds<W>& sm, int64_t n, int s0,
                                                      const GramAcc<W>* acc, AOperand<W>& at,
                                                      int lane, int c, int g) {
  constexpr int AST = InverseLds<W>::AST;
  const int B = prm.B, U = prm.U, S = prm.S;
  if (s0 == 0) {
    store_gram_lds<W>(*acc, sm.A, sm.G, (float*)sm.P, AST, prm.beta, c, g);
    wave_lds_sync();
    build_inverse<W, METHOD>(sm, U, prm.K, lane, c, g);
    // A operand for ||q||^2 = v^H G v (the output stage puts the raw
    // diagonal sm.G in place of A's)
    at.load(sm.A, AST, c, g, 16 * W);
  }
  float2 t[W][4], v[W][4];
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int u = 16 * w + c, s = s0 + 4 * g + j;
      t[w][j] = (u < U && s < S) ? prm.T[((size_t)n * U + u) * S + s] : make_float2(0.f, 0.f);
    }
  apply_inverse<W>(sm, t, c, g, v);                      // v = X t
  precode_store<W, IN, float>(prm, n, s0, offset_sc(IN{}, prm.H, n, B, U), v, at, sm.G, sm.P,
                              sm.N, c, g);
  wave_lds_sync();
}

template <int W, typename IN, int METHOD>
__global__ __launch_bounds__(64) void precode_inverse_kernel(PrecodeParams prm) {
  __shared__ InverseLds<W> sm;
  const int lane = threadIdx.x;
  const int c = lane & 15, g = lane >> 4;
  const int B = prm.B, U = prm.U, S = prm.S;
  for (int64_t n = blockIdx.x; n < prm.n_sc; n += gridDim.x) {
    const void* Hn = offset_sc(IN{}, prm.H, n, B, U);
    AOperand<W> at;
    for (int s0 = 0; s0 < S; s0 += 16) {
      GramAcc<W> acc;
      if (s0 == 0) {
        acc.clear();
        gram_mf<W, true, false>(IN{}, Hn, nullptr, B, U, S, 0, c, g, acc);
      }
      precode_inverse_chunk<W, IN, METHOD>(prm, sm, n, s0, &acc, at, lane, c, g);
    }
  }
}

// Streaming form for S <= 16 (see detect_inverse_stream_kernel).
template <int W, typename IN, int METHOD>
__global__ __launch_bounds__(64, W == 1 ? 4 : 1) void precode_inverse_stream_kernel(PrecodeParams kprm) {
  using Sub = typename Storage<IN, W>::Sub;
  using Blk = typename Storage<IN, W>::SmallBlock;
  __shared__ InverseLds<W> sm;
  const int lane = threadIdx.x;
  const int c = lane & 15, g = lane >> 4;
  int64_t n = blockIdx.x;
  Sub cur;
  Blk blk;
  if (n < kprm.n_sc) {
    cur.init(offset_sc(IN{}, kprm.H, n, kprm.B, kprm.U), nullptr, kprm.B, kprm.U, kprm.S, 0, c,
             g);
    blk.template load<false>(cur, 0);
  }
  while (n < kprm.n_sc) {
    const PrecodeParams prm = opaque_sizes(kprm);
    const int B = prm.B, U = prm.U, S = prm.S;
    const int64_t nn = n + gridDim.x;
    const int64_t nc = nn < prm.n_sc ? nn : n;
    Sub nxt;
    nxt.init(offset_sc(IN{}, prm.H, nc, B, U), nullptr, B, U, S, 0, c, g);
    if (nn >= prm.n_sc) nxt.disable();
    GramAcc<W> acc;
    acc.clear();
    gram_stream<W, false>(IN{}, blk, cur, nxt, B, acc);
    AOperand<W> at;
    precode_inverse_chunk<W, IN, METHOD>(prm, sm, n, 0, &acc, at, lane, c, g);
    n = nn;
    cur = nxt;
  }
}

static dim3 sc_grid(int64_t n_sc) {
  int64_t blocks = n_sc < (1 << 20) ? n_sc : (1 << 20);
  return dim3((unsigned)(blocks < 1 ? 1 : blocks));
}

// Persistent grid of the streaming forms: as many one-wave blocks per CU as
// the LDS allows, up to 16.
template <int W>
static dim3 stream_grid(int64_t n_sc) {
  constexpr int64_t kLdsPerCu = 160 * 1024;
  constexpr int64_t fit = kLdsPerCu / (int64_t)sizeof(InverseLds<W>);
  const int64_t cap = (int64_t)num_compute_units() * (fit < 16 ? fit : 16);
  const int64_t blocks = n_sc < cap ? n_sc : cap;
  return dim3((unsigned)(blocks < 1 ? 1 : blocks));
}

template <int W, typename IN, int M, int METHOD>
static void launch_detect_form(const DetectParams& p, hipStream_t stream) {
  if (p.S <= 16)
    hipLaunchKernelGGL((detect_inverse_stream_kernel<W, IN, M, METHOD>), stream_grid<W>(p.n_sc),
                       dim3(kWave), 0, stream, p);
  else
    hipLaunchKernelGGL((detect_inverse_kernel<W, IN, M, METHOD>), sc_grid(p.n_sc), dim3(kWave),
                       0, stream, p);
}

template <int W, typename IN, int METHOD>
static hipError_t launch_detect_m(const DetectParams& p, int m_bits, hipStream_t stream) {
  switch (m_bits) {
    case 2: launch_detect_form<W, IN, 2, METHOD>(p, stream); break;
    case 4: launch_detect_form<W, IN, 4, METHOD>(p, stream); break;
    case 6: launch_detect_form<W, IN, 6, METHOD>(p, stream); break;
    case 8: launch_detect_form<W, IN, 8, METHOD>(p, stream); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int W, int METHOD>
static hipError_t launch_detect_in(const DetectParams& p, int in_dtype, int m_bits,
                                   hipStream_t stream) {
  switch (in_dtype) {
    case 0: return launch_detect_m<W, InC32, METHOD>(p, m_bits, stream);
    case 1: return launch_detect_m<W, InF16, METHOD>(p, m_bits, stream);
    case 2: return launch_detect_m<W, InBF16, METHOD>(p, m_bits, stream);
  }
  return hipErrorInvalidValue;
}

template <int W, typename IN, int METHOD>
static void launch_precode_form(const PrecodeParams& p, hipStream_t stream) {
  if (p.S <= 16)
    hipLaunchKernelGGL((precode_inverse_stream_kernel<W, IN, METHOD>), stream_grid<W>(p.n_sc),
                       dim3(kWave), 0, stream, p);
  else
    hipLaunchKernelGGL((precode_inverse_kernel<W, IN, METHOD>), sc_grid(p.n_sc), dim3(kWave), 0,
                       stream, p);
}

template <int W, int METHOD>
static hipError_t launch_precode_in(const PrecodeParams& p, int in_dtype, hipStream_t stream) {
  switch (in_dtype) {
    case 0: launch_precode_form<W, InC32, METHOD>(p, stream); break;
    case 1: launch_precode_form<W, InF16, METHOD>(p, stream); break;
    case 2: launch_precode_form<W, InBF16, METHOD>(p, stream); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_detect_inverse(const DetectParams& p, int method, int in_dtype, int m_bits,
                                 hipStream_t stream) {
  if (method == kInvCholesky)
    return p.U <= 16 ? launch_detect_in<1, kInvCholesky>(p, in_dtype, m_bits, stream)
                     : launch_detect_in<2, kInvCholesky>(p, in_dtype, m_bits, stream);
  if (method == kInvNeumann)
    return p.U <= 16 ? launch_detect_in<1, kInvNeumann>(p, in_dtype, m_bits, stream)
                     : launch_detect_in<2, kInvNeumann>(p, in_dtype, m_bits, stream);
  return hipErrorInvalidValue;
}

hipError_t launch_precode_inverse(const PrecodeParams& p, int method, int in_dtype,
                                  hipStream_t stream) {
  if (method == kInvCholesky)
    return p.U <= 16 ? launch_precode_in<1, kInvCholesky>(p, in_dtype, stream)
                     : launch_precode_in<2, kInvCholesky>(p, in_dtype, stream);
  if (method == kInvNeumann)
    return p.U <= 16 ? launch_precode_in<1, kInvNeumann>(p, in_dtype, stream)
                     : launch_precode_in<2, kInvNeumann>(p, in_dtype, stream);
  return hipErrorInvalidValue;
}

}  // namespace mimo

// Fused CG-P kernel (Sec. III-D): Gram on MFMA, K CG iterations on
// (H_d H_d^H + beta I) v = t, then q = H_d^H v = H_u v on MFMA, with the
// optional power normalization s = q / ||q|| (Sec. II-B).  One wavefront per
// subcarrier.
//
// ||q||^2 = v^H H^H H v = v^H G v is formed in the CG layout from one more
// mat-vec with A (v^H A v - beta ||v||^2), so each output tile is written
// once, already scaled.
#include "cg_core.hpp"
#include "gram_phase.hpp"
#include "kernels.hpp"

namespace mimo {

// One element H[b][u] of a subcarrier's channel as complex FP32.
__device__ __forceinline__ float2 load_h(InC32, const void* Hn, int b, int u, int U) {
  return ((const float2*)Hn)[(size_t)b * U + u];
}
__device__ __forceinline__ float2 load_h(InF16, const void* Hn, int b, int u, int U) {
  const _Float16* p = (const _Float16*)Hn + ((size_t)(2 * (b >> 3)) * U + u) * 8 + (b & 7);
  return make_float2((float)p[0], (float)p[(size_t)U * 8]);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t x) {
  return __builtin_bit_cast(float, (uint32_t)x << 16);
}
__device__ __forceinline__ float2 load_h(InBF16, const void* Hn, int b, int u, int U) {
  const uint16_t* p = (const uint16_t*)Hn + ((size_t)(2 * (b >> 3)) * U + u) * 8 + (b & 7);
  return make_float2(bf16_to_f32(p[0]), bf16_to_f32(p[(size_t)U * 8]));
}

// A-operand rows of the output contraction: H[b][u] for u = 16 w + 4 g + t.
// Row b0 + c of H (users 16 w + 4 g + t); rows past B read zero.
template <int W>
__device__ __forceinline__ void load_h_row(InC32, const void* Hn, int B, int U, int b0, int c,
                                           int w, int g, float2 (&hv)[4]) {
  const __amdgpu_buffer_rsrc_t rh = make_rsrc(Hn, (uint32_t)B * U * 8u);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int u = 16 * w + 4 * g + t;
    hv[t] = bload2(rh, u < U ? (uint32_t)(c * U + u) * 8u : kOOB, (uint32_t)b0 * U * 8u);
  }
}
template <int W, typename IN>
__device__ __forceinline__ void load_h_row(IN tag, const void* Hn, int B, int U, int b0, int c,
                                           int w, int g, float2 (&hv)[4]) {
  const int brow = b0 + c;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int u = 16 * w + 4 * g + t;
    hv[t] = (brow < B && u < U) ? load_h(tag, Hn, brow, u, U) : make_float2(0.f, 0.f);
  }
}

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

    // ---- ||q||^2 = v^H G v ; V stays staged in Ps for the output contraction
    stage_vec<W>(Ps, c, g, st.v);
    wave_lds_sync();
    float2 e[W][4];
    matvec_mfma<W>(at, Ps, c, g, e);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      ST part = ST(0);
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const float2 v = st.v[w][j];
        part += (ST)v.x * (ST)e[w][j].x + (ST)v.y * (ST)e[w][j].y -
                (ST)beta * ((ST)v.x * (ST)v.x + (ST)v.y * (ST)v.y);
      }
      const ST qq = row_sum16(part);
      if (c == 0) Ns[4 * g + j] = (float)(qq > ST(0) ? qq : ST(0));
    }
    wave_lds_sync();

    // ---- q = H_u v (Algorithm 1 output) on MFMA: rows = antennas,
    // columns = right-hand sides, k = users (k-group g takes users
    // 16 w + 4 g + t, t = 0..3, so a lane reads 4 adjacent users of a row).
    const int s = s0 + c;
    const float nrm2 = Ns[c];
    const float scl = prm.normalize ? (nrm2 > 0.f ? __builtin_amdgcn_rsqf(nrm2) : 0.f) : 1.0f;
    float2 vv[W][4];
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int t = 0; t < 4; ++t) vv[w][t] = Ps[(16 * w + 4 * g + t) * kPST + c];
    float2 hn[W][4];                                 // next row tile, loaded ahead
#pragma unroll
    for (int w = 0; w < W; ++w) load_h_row<W>(IN{}, Hn, B, U, 0, c, w, g, hn[w]);
    // three real products per complex one: P1 = Hr Vr, P2 = Hi Vi,
    // P3 = (Hr + Hi)(Vr + Vi); Re q = P1 - P2, Im q = P3 - P1 - P2
    float vs[W][4];
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int t = 0; t < 4; ++t) vs[w][t] = vv[w][t].x + vv[w][t].y;
    for (int b0 = 0; b0 < B; b0 += 16) {
      f4 p1 = zero4(), p2 = zero4(), p3 = zero4();
      float2 hc[W][4];
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int t = 0; t < 4; ++t) hc[w][t] = hn[w][t];
#pragma unroll
      for (int w = 0; w < W; ++w) load_h_row<W>(IN{}, Hn, B, U, b0 + 16, c, w, g, hn[w]);
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const float2(&hv)[4] = hc[w];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          p1 = mfma4(hv[t].x, vv[w][t].x, p1);
          p2 = mfma4(hv[t].y, vv[w][t].y, p2);
          p3 = mfma4(hv[t].x + hv[t].y, vs[w][t], p3);
        }
      }
      const f4 qr = p1 - p2;
      const f4 qi = p3 - p1 - p2;
      if (s < S) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int bb = b0 + 4 * g + j;
          if (bb < B) prm.Q[((size_t)n * B + bb) * S + s] = make_float2(qr[j] * scl, qi[j] * scl);
        }
      }
    }
    if (prm.qnorm && c == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int ss = s0 + 4 * g + j;
        if (ss < S) prm.qnorm[(size_t)n * S + ss] = sqrtf(Ns[4 * g + j]);
      }
    }
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

template <int W, typename IN>
static hipError_t launch_st(const PrecodeParams& p, int f64, const Schedule& sch,
                            hipStream_t stream) {
  const dim3 grid(sched_grid(p.n_sc, sch)), block(kWave * kWavesPerBlock);
  if (f64)
    hipLaunchKernelGGL((precode_kernel<W, IN, double>), grid, block, 0, stream, p);
  else
    hipLaunchKernelGGL((precode_kernel<W, IN, float>), grid, block, 0, stream, p);
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

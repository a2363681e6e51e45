// Fused CG-D kernel: Gram + matched filter (MFMA) -> K CG iterations with the
// approximate in-loop SINR tracker -> max-log LLR epilogue, one wavefront per
// subcarrier (Sec. III-B, III-C-2, Algorithm 1, eqs. (4), (13)-(15)).
#include "cg_core.hpp"
#include "gram_phase.hpp"
#include "kernels.hpp"
#include "llr.hpp"

namespace mimo {

template <int W, typename IN, typename ST, int M_BITS>
__global__ __launch_bounds__(256, 2) void detect_approx_kernel(DetectParams prm) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;   // LDS row stride (complex) of A
  __shared__ __align__(16) float2 A_s[kWavesPerBlock][NU * AST];
  __shared__ __align__(16) float2 P_s[kWavesPerBlock][NU * kPST];
  __shared__ float G_s[kWavesPerBlock][NU];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  float2* As = A_s[wv];
  float2* Ps = P_s[wv];
  float* Gs = G_s[wv];
  const int B = prm.B, U = prm.U, S = prm.S;

  for (int64_t n = (int64_t)blockIdx.x * kWavesPerBlock + wv; n < prm.n_sc;
       n += (int64_t)gridDim.x * kWavesPerBlock) {
    const void* Hn = offset_sc(IN{}, prm.H, n, B, U);
    const void* Yn = offset_sc(IN{}, prm.Y, n, B, S);
    AOperand<W> at;
    float d[W];
    for (int s0 = 0; s0 < S; s0 += 16) {
      // ---- A = H^H H + (N0/E_s) I and b = H^H y (Algorithm 1, initialization)
      GramAcc<W> acc;
      acc.clear();
      if (s0 == 0) {
        gram_mf<W, true, true>(IN{}, Hn, Yn, B, U, S, s0, c, g, acc);
        store_gram_lds<W>(acc, As, Gs, (float*)Ps, AST, prm.reg, c, g);
        wave_lds_sync();
        at.load(As, AST, c, g);
#pragma unroll
        for (int w = 0; w < W; ++w) d[w] = As[(16 * w + c) * AST + 16 * w + c].x;
      } else {
        gram_mf<W, false, true>(IN{}, Hn, Yn, B, U, S, s0, c, g, acc);
      }

      // ---- K iterations of Algorithm 1 with the tracker of eq. (13)
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

      // ---- mu (eq. (14)), rho (eq. (15)), z = xhat / mu, LLRs (eq. (4))
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const int u = 16 * w + c;
        if (u >= U) continue;
        const float Guu = Gs[u];
        const float rho = Guu / prm.n0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int s = s0 + 4 * g + j;
          if (s >= S) continue;
          const float mu = (float)(tk.tv[w][j] * (ST)Guu);
          const float2 x = st.v[w][j];
          // |mu| < FLT_MIN only when the right-hand side froze at (near) zero:
          // z = 0 as for b = 0.
          const float imu = fabsf(mu) >= __FLT_MIN__ ? __builtin_amdgcn_rcpf(mu) : 0.f;
          const float2 z = make_float2(x.x * imu, x.y * imu);
          float out[M_BITS];
          llr_maxlog<M_BITS>(z, rho, prm.scale, prm.inv_scale, out);
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
  }
}

template <int W, typename IN, typename ST>
static hipError_t launch_m(const DetectParams& p, int m_bits, hipStream_t stream) {
  const dim3 grid(wave_grid(p.n_sc)), block(kWave * kWavesPerBlock);
  switch (m_bits) {
    case 2: hipLaunchKernelGGL((detect_approx_kernel<W, IN, ST, 2>), grid, block, 0, stream, p); break;
    case 4: hipLaunchKernelGGL((detect_approx_kernel<W, IN, ST, 4>), grid, block, 0, stream, p); break;
    case 6: hipLaunchKernelGGL((detect_approx_kernel<W, IN, ST, 6>), grid, block, 0, stream, p); break;
    case 8: hipLaunchKernelGGL((detect_approx_kernel<W, IN, ST, 8>), grid, block, 0, stream, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int W, typename IN>
static hipError_t launch_st(const DetectParams& p, int f64, int m_bits, hipStream_t stream) {
  return f64 ? launch_m<W, IN, double>(p, m_bits, stream) : launch_m<W, IN, float>(p, m_bits, stream);
}

template <int W>
static hipError_t launch_in(const DetectParams& p, int in_dtype, int f64, int m_bits,
                            hipStream_t stream) {
  switch (in_dtype) {
    case 0: return launch_st<W, InC32>(p, f64, m_bits, stream);
    case 1: return launch_st<W, InF16>(p, f64, m_bits, stream);
    case 2: return launch_st<W, InBF16>(p, f64, m_bits, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_detect_approx(const DetectParams& p, int in_dtype, int scalar_f64, int m_bits,
                                hipStream_t stream) {
  if (p.U <= 16) return launch_in<1>(p, in_dtype, scalar_f64, m_bits, stream);
  return launch_in<2>(p, in_dtype, scalar_f64, m_bits, stream);
}

}  // namespace mimo

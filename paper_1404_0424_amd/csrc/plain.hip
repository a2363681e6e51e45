// Plain FP32 per-system detection: the straightforward mapping used as the
// baseline the optimized kernels are measured against.  One wavefront per
// subcarrier; the Gram matrix, the matched filter and the CG mat-vec are
// plain FP32 FMAs on the vector ALUs (no MFMA); the right-hand sides are
// solved one after another with one lane per user.  Same method and
// outputs as detect.hip (Algorithm 1, eqs. (4), (13)-(15)).
#include "cg_core.hpp"
#include "gram_phase.hpp"
#include "launch.hpp"
#include "llr.hpp"

namespace mimo {

template <typename ST, int M_BITS>
__global__ __launch_bounds__(256) void detect_plain_kernel(DetectParams prm) {
  constexpr int UM = 32, AST = UM + 1;
  __shared__ float2 A_s[kWavesPerBlock][UM * AST];
  __shared__ float G_s[kWavesPerBlock][UM];
  __shared__ float2 X_s[kWavesPerBlock][UM];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  float2* As = A_s[wv];
  float* Gs = G_s[wv];
  float2* Xs = X_s[wv];
  const int B = prm.B, U = prm.U, S = prm.S;
  for (int64_t n = (int64_t)blockIdx.x * kWavesPerBlock + wv; n < prm.n_sc;
       n += (int64_t)gridDim.x * kWavesPerBlock) {
    const float2* Hn = (const float2*)prm.H + (size_t)n * B * U;
    const float2* Yn = (const float2*)prm.Y + (size_t)n * B * S;
    // A = H^H H + reg I: upper triangle over the lanes, mirrored
    for (int idx = lane; idx < U * U; idx += kWave) {
      const int i = idx / U, j = idx % U;
      if (i > j) continue;
      float2 acc = make_float2(0.f, 0.f);
      for (int b = 0; b < B; ++b) {
        const float2 hi = Hn[(size_t)b * U + i], hj = Hn[(size_t)b * U + j];
        cfma(acc, make_float2(hi.x, -hi.y), hj);
      }
      if (i == j) {
        As[i * AST + i] = make_float2(acc.x + prm.reg, 0.f);
        Gs[i] = acc.x;
      } else {
        As[i * AST + j] = acc;
        As[j * AST + i] = make_float2(acc.x, -acc.y);
      }
    }
    wave_lds_sync();
    const bool own = lane < U;
    const float d = own ? As[lane * AST + lane].x : 1.f;
    const float Guu = own ? Gs[lane] : 0.f;
    for (int s = 0; s < S; ++s) {
      // b = H^H y_s, lane u
      float2 bu = make_float2(0.f, 0.f);
      if (own)
        for (int b = 0; b < B; ++b) {
          const float2 h = Hn[(size_t)b * U + lane];
          cfma(bu, make_float2(h.x, -h.y), Yn[(size_t)b * S + s]);
        }
      float2 v = make_float2(0.f, 0.f), r = bu, p = bu;
      ST rr = wave_sum<ST>((ST)bu.x * (ST)bu.x + (ST)bu.y * (ST)bu.y);
      ST tv = ST(0), tr = ST(1), tp = ST(1);
      for (int k = 0; k < prm.K; ++k) {
        if (own) Xs[lane] = p;
        wave_lds_sync();
        float2 e = make_float2(0.f, 0.f);
        if (own)
          for (int l = 0; l < U; ++l) cfma(e, As[lane * AST + l], Xs[l]);
        wave_lds_sync();
        const ST pe = wave_sum<ST>((ST)p.x * (ST)e.x + (ST)p.y * (ST)e.y);
        const bool live = live_floor<ST>(rr, pe);
        const ST alpha = live ? div_fast<ST>(rr, pe) : ST(0);
        const float af = (float)alpha;
        v.x = __builtin_fmaf(af, p.x, v.x);
        v.y = __builtin_fmaf(af, p.y, v.y);
        r.x = __builtin_fmaf(-af, e.x, r.x);
        r.y = __builtin_fmaf(-af, e.y, r.y);
        const ST rr_new = wave_sum<ST>((ST)r.x * (ST)r.x + (ST)r.y * (ST)r.y);
        const ST beta = live ? div_fast<ST>(rr_new, rr) : ST(0);
        const float bf = (float)beta;
        if (live) {
          p.x = __builtin_fmaf(bf, p.x, r.x);
          p.y = __builtin_fmaf(bf, p.y, r.y);
          rr = rr_new;
        }
        tv = tv + alpha * tp;                     // tracker of eq. (13)
        tr = tr - alpha * (ST)d * tp;
        tp = tr + beta * tp;
      }
      if (own) {
        const float mu = (float)(tv * (ST)Guu);
        const float rho = Guu / prm.n0;
        const float imu = fabsf(mu) >= __FLT_MIN__ ? __builtin_amdgcn_rcpf(mu) : 0.f;
        float out[M_BITS];
        llr_maxlog<M_BITS>(make_float2(v.x * imu, v.y * imu), rho, prm.scale, prm.inv_scale, out);
        const size_t idx = ((size_t)n * U + lane) * S + s;
#pragma unroll
        for (int q = 0; q < M_BITS; ++q) prm.llr[idx * M_BITS + q] = out[q];
        if (prm.xhat) prm.xhat[idx] = v;
        if (prm.mu) prm.mu[idx] = mu;
        if (prm.sinr) prm.sinr[idx] = rho;
      }
    }
    wave_lds_sync();
  }
}

template <typename ST>
static hipError_t launch_m(const DetectParams& p, int m_bits, const Schedule& sch,
                           hipStream_t stream) {
  const dim3 grid(sched_grid(p.n_sc, sch)), block(kWave * kWavesPerBlock);
  switch (m_bits) {
    case 2: hipLaunchKernelGGL((detect_plain_kernel<ST, 2>), grid, block, 0, stream, p); break;
    case 4: hipLaunchKernelGGL((detect_plain_kernel<ST, 4>), grid, block, 0, stream, p); break;
    case 6: hipLaunchKernelGGL((detect_plain_kernel<ST, 6>), grid, block, 0, stream, p); break;
    case 8: hipLaunchKernelGGL((detect_plain_kernel<ST, 8>), grid, block, 0, stream, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_detect_plain(const DetectParams& p, int scalar_f64, int m_bits,
                               const Schedule& sch, hipStream_t stream) {
  return scalar_f64 ? launch_m<double>(p, m_bits, sch, stream)
                    : launch_m<float>(p, m_bits, sch, stream);
}

}  // namespace mimo

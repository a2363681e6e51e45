// CG-D with the exact in-loop SINR of Sec. III-C-1 (parity mode).
//
// The CG-equivalent matrix L_k of eq. (9) obeys the matrix form of
// Algorithm 1 with the CG's own alpha_k, beta_k (V_0 = 0, R_0 = P_0 = I,
// V_k = V_{k-1} + alpha_k P_{k-1}, R_k = R_{k-1} - alpha_k A P_{k-1},
// P_k = R_k + beta_k P_{k-1}); eliminating R and P gives recursion (12), and
// V_k b = v_k.  After K iterations B = L_K G, mu_i = B_ii, C = B L_K^H and
// nu_i^2 = sum_{j != i} |B_ij|^2 E_s + C_ii N0, rho_i = mu_i^2 / nu_i^2.
//
// This costs a U x U x U complex product per iteration and right-hand side
// (the paper notes its high complexity); one wavefront handles one subcarrier
// and walks its right-hand sides in turn.  With one user tile (U <= 16) the
// products run on MFMA with V, R, P in registers; two tiles use VALU FMAs
// over LDS.
#include "cg_core.hpp"
#include "gram_phase.hpp"
#include "launch.hpp"
#include "llr.hpp"

namespace mimo {

template <int W, typename IN, typename ST, int M_BITS>
__global__ __launch_bounds__(64) void detect_exact_kernel(DetectParams prm) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;
  constexpr int MST = NU + 1;   // matrix row stride for the scalar-indexed loops
  __shared__ __align__(16) float2 As[NU * AST];
  __shared__ float Gs[NU];
  __shared__ __align__(16) float2 Bs[16 * AST];   // matched filter of the current chunk [rhs][user]
  // (one tile keeps R in registers and needs 16 entries of Em for the row terms)
  __shared__ __align__(16) float2 Vm[NU * MST], Pm[NU * MST];
  __shared__ __align__(16) float2 Rm[W == 1 ? 1 : NU * MST], Em[W == 1 ? 16 : NU * MST];
  __shared__ __align__(16) float2 pv[NU];
  const int t = threadIdx.x;
  const int c = t & 15, g = t >> 4;
  const int B = prm.B, U = prm.U, S = prm.S;
  const int UU = U * U;

  for (int64_t n = blockIdx.x; n < prm.n_sc; n += gridDim.x) {
    const void* Hn = offset_sc(IN{}, prm.H, n, B, U);
    const void* Yn = offset_sc(IN{}, prm.Y, n, B, S);
    for (int s0 = 0; s0 < S; s0 += 16) {
      GramAcc<W> acc;
      acc.clear();
      if (s0 == 0) {
        gram_mf<W, true, true>(IN{}, Hn, Yn, B, U, S, s0, c, g, acc);
        store_gram_lds<W>(acc, As, Gs, (float*)Bs, AST, prm.reg, c, g);
        wave_lds_sync();
      } else {
        gram_mf<W, false, true>(IN{}, Hn, Yn, B, U, S, s0, c, g, acc);
      }
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          Bs[(4 * g + j) * AST + 16 * w + c] = make_float2(acc.dr[w][j], acc.di[w][j]);
      __syncthreads();

      const int nrhs = (S - s0) < 16 ? (S - s0) : 16;
      for (int sl = 0; sl < nrhs; ++sl) {
        const int s = s0 + sl;
        // ---- vector CG state: thread t < U owns entry t
        const bool own = t < U;
        const float2 bu = own ? Bs[sl * AST + t] : make_float2(0.f, 0.f);
        float2 v = make_float2(0.f, 0.f), r = bu, p = bu;
        ST rr = wave_sum<ST>((ST)bu.x * (ST)bu.x + (ST)bu.y * (ST)bu.y);
        float mu = 0.f, nu2 = 0.f;     // mu_t = Re B_tt and nu_t^2 of the own user t
        if constexpr (W == 1) {
          // Matrices on MFMA (16x16x4, four real products per complex one),
          // held in the D layout: lane (c, g) keeps entries (4 g + jj, c).
          float2 Vr[4], Rr[4], Pr[4];
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const int i = 4 * g + jj;
            const float2 id = make_float2(i == c && i < U ? 1.f : 0.f, 0.f);
            Vr[jj] = make_float2(0.f, 0.f);
            Rr[jj] = id;
            Pr[jj] = id;
          }
          for (int k = 0; k < prm.K; ++k) {
            if (own) pv[t] = p;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) Pm[(4 * g + jj) * MST + c] = Pr[jj];
            __syncthreads();
            float2 e = make_float2(0.f, 0.f);
            if (own)
              for (int l = 0; l < U; ++l) cfma(e, As[t * AST + l], pv[l]);
            f4 er = zero4(), ei = zero4();                    // E = A P
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
              const float2 a = As[c * AST + 4 * tt + g];      // A[c][4 tt + g]
              const float2 b = Pm[(4 * tt + g) * MST + c];    // P[4 tt + g][c]
              er = mfma4(a.x, b.x, er);
              er = mfma4(-a.y, b.y, er);
              ei = mfma4(a.x, b.y, ei);
              ei = mfma4(a.y, b.x, ei);
            }
            const ST pe = wave_sum<ST>((ST)p.x * (ST)e.x + (ST)p.y * (ST)e.y);
            const bool live = rr > ST(0) && pe > ST(0);
            const ST alpha = live ? rr / pe : ST(0);
            const float af = (float)alpha;
            v.x = __builtin_fmaf(af, p.x, v.x);
            v.y = __builtin_fmaf(af, p.y, v.y);
            r.x = __builtin_fmaf(-af, e.x, r.x);
            r.y = __builtin_fmaf(-af, e.y, r.y);
            const ST rr_new = wave_sum<ST>((ST)r.x * (ST)r.x + (ST)r.y * (ST)r.y);
            const ST beta = live ? rr_new / rr : ST(0);
            const float bf = (float)beta;
            if (live) {
              p.x = __builtin_fmaf(bf, p.x, r.x);
              p.y = __builtin_fmaf(bf, p.y, r.y);
              rr = rr_new;
            }
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              const float2 P0 = Pr[jj];
              Vr[jj].x = __builtin_fmaf(af, P0.x, Vr[jj].x);
              Vr[jj].y = __builtin_fmaf(af, P0.y, Vr[jj].y);
              Rr[jj].x = __builtin_fmaf(-af, er[jj], Rr[jj].x);
              Rr[jj].y = __builtin_fmaf(-af, ei[jj], Rr[jj].y);
              Pr[jj] = make_float2(__builtin_fmaf(bf, P0.x, Rr[jj].x),
                                   __builtin_fmaf(bf, P0.y, Rr[jj].y));
            }
            __syncthreads();
          }
          // B = L_K G (G = A - reg I off the diagonal; diagonal G_ii)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) Vm[(4 * g + jj) * MST + c] = Vr[jj];
          __syncthreads();
          f4 br = zero4(), bi = zero4();
#pragma unroll
          for (int tt = 0; tt < 4; ++tt) {
            const int l = 4 * tt + g;
            const float2 a = Vm[c * MST + l];                  // V[c][l]
            const float2 b = l == c ? make_float2(Gs[c], 0.f) : As[l * AST + c];   // G[l][c]
            br = mfma4(a.x, b.x, br);
            br = mfma4(-a.y, b.y, br);
            bi = mfma4(a.x, b.y, bi);
            bi = mfma4(a.y, b.x, bi);
          }
          // row i = 4 g + jj: mu_i = Re B_ii, sum_{j != i} |B_ij|^2 and
          // C_ii = sum_j Re(B_ij conj(L_ij)), reduced over the row's 16 lanes
          float2* X = (float2*)Em;
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const int i = 4 * g + jj;
            const float2 b = make_float2(br[jj], bi[jj]);
            float off = (c != i && c < U) ? cabs2(b) : 0.f;
            float cii = b.x * Vr[jj].x + b.y * Vr[jj].y;
            float mui = c == i ? b.x : 0.f;
            off = row_sum16(off);
            cii = row_sum16(cii);
            mui = row_sum16(mui);
            if (c == 0) X[i] = make_float2(mui, off * prm.es + cii * prm.n0);
          }
          __syncthreads();
          if (own) {
            mu = X[t].x;
            nu2 = X[t].y;
          }
        } else {
          for (int idx = t; idx < UU; idx += kWave) {
            const int i = idx / U, j = idx % U;
            const float2 id = make_float2(i == j ? 1.f : 0.f, 0.f);
            Vm[i * MST + j] = make_float2(0.f, 0.f);
            Rm[i * MST + j] = id;
            Pm[i * MST + j] = id;
          }
          __syncthreads();
          for (int k = 0; k < prm.K; ++k) {
            if (own) pv[t] = p;
            __syncthreads();
            float2 e = make_float2(0.f, 0.f);
            if (own)
              for (int l = 0; l < U; ++l) cfma(e, As[t * AST + l], pv[l]);
            for (int idx = t; idx < UU; idx += kWave) {          // E = A P
              const int i = idx / U, j = idx % U;
              float2 x = make_float2(0.f, 0.f);
              for (int l = 0; l < U; ++l) cfma(x, As[i * AST + l], Pm[l * MST + j]);
              Em[i * MST + j] = x;
            }
            const ST pe = wave_sum<ST>((ST)p.x * (ST)e.x + (ST)p.y * (ST)e.y);
            const bool live = rr > ST(0) && pe > ST(0);
            const ST alpha = live ? rr / pe : ST(0);
            const float af = (float)alpha;
            v.x = __builtin_fmaf(af, p.x, v.x);
            v.y = __builtin_fmaf(af, p.y, v.y);
            r.x = __builtin_fmaf(-af, e.x, r.x);
            r.y = __builtin_fmaf(-af, e.y, r.y);
            const ST rr_new = wave_sum<ST>((ST)r.x * (ST)r.x + (ST)r.y * (ST)r.y);
            const ST beta = live ? rr_new / rr : ST(0);
            const float bf = (float)beta;
            if (live) {
              p.x = __builtin_fmaf(bf, p.x, r.x);
              p.y = __builtin_fmaf(bf, p.y, r.y);
              rr = rr_new;
            }
            __syncthreads();
            for (int idx = t; idx < UU; idx += kWave) {
              const int i = idx / U, j = idx % U, o = i * MST + j;
              const float2 P0 = Pm[o], E0 = Em[o];
              float2 Vn = Vm[o], Rn = Rm[o];
              Vn.x = __builtin_fmaf(af, P0.x, Vn.x);
              Vn.y = __builtin_fmaf(af, P0.y, Vn.y);
              Rn.x = __builtin_fmaf(-af, E0.x, Rn.x);
              Rn.y = __builtin_fmaf(-af, E0.y, Rn.y);
              Vm[o] = Vn;
              Rm[o] = Rn;
              Pm[o] = make_float2(__builtin_fmaf(bf, P0.x, Rn.x), __builtin_fmaf(bf, P0.y, Rn.y));
            }
            __syncthreads();
          }
          // ---- B = L_K G (G = A - reg I off the diagonal; diagonal G_ii)
          for (int idx = t; idx < UU; idx += kWave) {
            const int i = idx / U, j = idx % U;
            float2 x = make_float2(0.f, 0.f);
            for (int l = 0; l < U; ++l) {
              const float2 gl = (l == j) ? make_float2(Gs[j], 0.f) : As[l * AST + j];
              cfma(x, Vm[i * MST + l], gl);
            }
            Em[i * MST + j] = x;
          }
          __syncthreads();
          if (own) {
            const int i = t;
            mu = Em[i * MST + i].x;
            float off = 0.f, cii = 0.f;
            for (int j = 0; j < U; ++j) {
              const float2 bij = Em[i * MST + j], lij = Vm[i * MST + j];
              if (j != i) off += cabs2(bij);
              cii += bij.x * lij.x + bij.y * lij.y;       // Re(B_ij conj(L_ij))
            }
            nu2 = off * prm.es + cii * prm.n0;
          }
        }
        if (own) {
          const int i = t;
          float rho = (mu * mu) / nu2;
          float2 z;
          if (mu != 0.f) {
            z = make_float2(v.x / mu, v.y / mu);
          } else {
            z = make_float2(0.f, 0.f);
            rho = Gs[i] / prm.n0;
          }
          float out[M_BITS];
          llr_maxlog<M_BITS>(z, rho, prm.scale, prm.inv_scale, out);
          const size_t o = ((size_t)n * U + i) * S + s;
          float* lp = prm.llr + o * M_BITS;
#pragma unroll
          for (int q = 0; q < M_BITS; ++q) lp[q] = out[q];
          if (prm.xhat) prm.xhat[o] = v;
          if (prm.mu) prm.mu[o] = mu;
          if (prm.sinr) prm.sinr[o] = rho;
        }
        __syncthreads();
      }
    }
  }
}

template <int W, typename IN, typename ST>
static hipError_t launch_m(const DetectParams& p, int m_bits, hipStream_t stream) {
  int64_t blocks = p.n_sc < (1 << 20) ? p.n_sc : (1 << 20);
  if (blocks < 1) blocks = 1;
  const dim3 grid((unsigned)blocks), block(kWave);
  switch (m_bits) {
    case 2: hipLaunchKernelGGL((detect_exact_kernel<W, IN, ST, 2>), grid, block, 0, stream, p); break;
    case 4: hipLaunchKernelGGL((detect_exact_kernel<W, IN, ST, 4>), grid, block, 0, stream, p); break;
    case 6: hipLaunchKernelGGL((detect_exact_kernel<W, IN, ST, 6>), grid, block, 0, stream, p); break;
    case 8: hipLaunchKernelGGL((detect_exact_kernel<W, IN, ST, 8>), grid, block, 0, stream, p); break;
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

hipError_t launch_detect_exact(const DetectParams& p, int in_dtype, int scalar_f64, int m_bits,
                               hipStream_t stream) {
  if (p.U <= 16) return launch_in<1>(p, in_dtype, scalar_f64, m_bits, stream);
  return launch_in<2>(p, in_dtype, scalar_f64, m_bits, stream);
}

}  // namespace mimo

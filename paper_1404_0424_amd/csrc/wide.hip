// CG-D detection and CG-P precoding for 32 < U <= 64 (the paper's U <= B
// allows any U; Sec. II-A), complex64 storage: one workgroup of four
// wavefronts per subcarrier, wavefront w owning users 16 w .. 16 w + 15.
//
// Each wavefront accumulates its 16 rows of G = H^H H (all 64 columns: the
// four tiles (w, j) on MFMA, the channel streamed from HBM; the other
// wavefronts' loads of the same rows hit the CU's caches) and, for
// detection, the matched filter of its users; its rows of A = G + reg I go
// to LDS and come back as the A^T operand of its part of the mat-vec.  Per
// CG iteration (Algorithm 1 loop body) the wavefronts exchange P through a
// shared LDS array and the partial inner products Re(p^H e) and ||r||^2 of
// their users through a small LDS table, summed over the four wavefronts in
// a fixed order, so every wavefront computes the same step sizes.  The
// approximate SINR tracker of eq. (13), mu, rho and the LLRs (eq. (4)) are
// per user and stay in the owning wavefront.  Precoding forms ||q||^2 =
// v^H G v the same way and then q = H_u v (Algorithm 1 output) with V from
// LDS, each wavefront taking every fourth 16-antenna tile.
#include <type_traits>

#include "detect_core.hpp"
#include "launch.hpp"
#include "precode_out.hpp"

namespace mimo {

constexpr int kWideTiles = 4;
constexpr int kWideUsers = 16 * kWideTiles;
constexpr int kWideAst = kWideUsers + 2;   // LDS row stride (complex) of a wavefront's rows of A

template <typename ST>
struct WideLds {
  float2 A[kWideTiles][16 * kWideAst];       // rows 16 w .. 16 w + 15 of A, per wavefront
  float2 P[kWideUsers * kPST];               // P[user][rhs] of all users
  ST red[2][kWideTiles][16];                 // partial sums per wavefront and rhs
  float G[kWideUsers];                       // raw diagonal G_uu
  float N[16];                               // ||q||^2 per rhs (precoding)
};

// Lane (c, g) of wavefront w: user 16 w + c, right-hand sides s0 + 4 g + j.
struct WideLane {
  int w, c, g, lane;
};

// Rows 16 w .. of G (all four column tiles) and, with Y, b = H^H y of the
// wavefront's users for right-hand sides s0 ..; four antennas per MFMA step.
// gr/gi: Re and Im of tile (w, j); p1, p2, p3: the three-product matched
// filter (Re b = p1 + p2, Im b = p3 - p1 + p2).
struct WideAcc {
  f4 gr[kWideTiles], gi[kWideTiles];
  f4 p1, p2, p3;
};

template <bool DO_GRAM, bool DO_MF>
__device__ __forceinline__ void wide_gram_mf(const void* Hn, const void* Yn, int B, int U, int S,
                                             int s0, const WideLane& L, WideAcc& acc) {
  const __amdgpu_buffer_rsrc_t rh = make_rsrc(Hn, (uint32_t)B * U * 8u);
  const __amdgpu_buffer_rsrc_t ry =
      make_rsrc(DO_MF ? Yn : Hn, DO_MF ? (uint32_t)B * S * 8u : 0u);
  uint32_t oh[kWideTiles];
#pragma unroll
  for (int j = 0; j < kWideTiles; ++j) {
    const int u = 16 * j + L.c;
    oh[j] = u < U ? (uint32_t)(L.g * U + u) * 8u : kOOB;
  }
  const int uw = 16 * L.w + L.c;
  const uint32_t ow = uw < U ? (uint32_t)(L.g * U + uw) * 8u : kOOB;
  const int s = s0 + L.c;
  const uint32_t oy = s < S ? (uint32_t)(L.g * S + s) * 8u : kOOB;
#pragma unroll
  for (int j = 0; j < kWideTiles; ++j) { acc.gr[j] = zero4(); acc.gi[j] = zero4(); }
  acc.p1 = acc.p2 = acc.p3 = zero4();
  constexpr int UNR = 4;                         // k-steps loaded together
  for (int b0 = 0; b0 < B; b0 += 4 * UNR) {
    float2 h[UNR][kWideTiles], hw[UNR], y[UNR];
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      const int b = b0 + 4 * t;
      hw[t] = bload2(rh, ow, (uint32_t)b * U * 8u);
      if (DO_GRAM) {
#pragma unroll
        for (int j = 0; j < kWideTiles; ++j) h[t][j] = bload2(rh, oh[j], (uint32_t)b * U * 8u);
      }
      if (DO_MF) y[t] = bload2(ry, oy, (uint32_t)b * S * 8u);
    }
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      if (DO_GRAM) {
#pragma unroll
        for (int j = 0; j < kWideTiles; ++j) {
          acc.gr[j] = mfma4(hw[t].x, h[t][j].x, acc.gr[j]);
          acc.gr[j] = mfma4(hw[t].y, h[t][j].y, acc.gr[j]);
          acc.gi[j] = mfma4(hw[t].x, h[t][j].y, acc.gi[j]);
          acc.gi[j] = mfma4(-hw[t].y, h[t][j].x, acc.gi[j]);
        }
      }
      if (DO_MF) {
        acc.p1 = mfma4(y[t].x, hw[t].x, acc.p1);
        acc.p2 = mfma4(y[t].y, hw[t].y, acc.p2);
        acc.p3 = mfma4(y[t].x + y[t].y, hw[t].x - hw[t].y, acc.p3);
      }
    }
  }
}

// The wavefront's rows of A = G + reg I to LDS (the diagonal real, G_uu to
// lds.G), then its A^T operand a[t] = A[16 w + c][4 t + g] and d = A_uu.
template <typename ST>
__device__ __forceinline__ void wide_store_a(const WideAcc& acc, WideLds<ST>& lds, float reg,
                                             int U, const WideLane& L, float2 (&a)[16],
                                             float& d) {
  float2* Aw = lds.A[L.w];
#pragma unroll
  for (int j = 0; j < kWideTiles; ++j)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int rl = 4 * L.g + jj;                 // local row
      const int col = 16 * j + L.c;
      if (16 * L.w + rl == col) {
        Aw[rl * kWideAst + col] = make_float2(acc.gr[j][jj] + reg, 0.f);
        lds.G[col] = acc.gr[j][jj];
      } else {
        Aw[rl * kWideAst + col] = make_float2(acc.gr[j][jj], acc.gi[j][jj]);
      }
    }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 16; ++t) a[t] = Aw[L.c * kWideAst + 4 * t + L.g];
  d = Aw[L.c * kWideAst + 16 * L.w + L.c].x;
  (void)U;
}

// Sum of the four wavefronts' partial sums x[j] (rhs 4 g + j, the row sum
// of the wavefront's users already taken) through lds.red[slot]: the same
// value, in the same order, in every wavefront.
template <typename ST>
__device__ __forceinline__ void wide_sum(ST (&x)[4], WideLds<ST>& lds, int slot,
                                         const WideLane& L) {
  if (L.c == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) lds.red[slot][L.w][4 * L.g + j] = x[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int s = 4 * L.g + j;
    x[j] = ((lds.red[slot][0][s] + lds.red[slot][1][s]) + lds.red[slot][2][s]) +
           lds.red[slot][3][s];
  }
}

// e = A p for the wavefront's users from P of all users in LDS (E^T = P^T
// A^T on MFMA, k over users; k-steps past U are zero and skipped).
__device__ __forceinline__ void wide_matvec(const float2 (&a)[16], const float2* Ps, int nk,
                                            const WideLane& L, float2 (&e)[4]) {
  f4 er = zero4(), ei = zero4();
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    if (t < nk) {                                    // wave-uniform
      const float2 pk = Ps[(4 * t + L.g) * kPST + L.c];
      er = mfma4(pk.x, a[t].x, er);
      ei = mfma4(pk.x, a[t].y, ei);
      er = mfma4(-pk.y, a[t].y, er);
      ei = mfma4(pk.y, a[t].x, ei);
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) e[j] = make_float2(er[j], ei[j]);
}

template <typename ST>
__device__ __forceinline__ void wide_stage(const float2 (&x)[4], float2* Ps, const WideLane& L) {
  float4* d = (float4*)&Ps[(16 * L.w + L.c) * kPST + 4 * L.g];
  d[0] = make_float4(x[0].x, x[0].y, x[1].x, x[1].y);
  d[1] = make_float4(x[2].x, x[2].y, x[3].x, x[3].y);
}

template <typename ST>
__device__ __forceinline__ void wide_cg_init(CGState<1, ST>& st, const float2 (&b)[4],
                                             WideLds<ST>& lds, const WideLane& L) {
  __syncthreads();                                   // last readers of lds.red are done
  ST part[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    part[j] = (ST)b[j].x * (ST)b[j].x + (ST)b[j].y * (ST)b[j].y;
    st.v[0][j] = make_float2(0.f, 0.f);
    st.r[0][j] = b[j];
    st.p[0][j] = b[j];
  }
  row_sum16_x4(part);
  wide_sum(part, lds, 1, L);
#pragma unroll
  for (int j = 0; j < 4; ++j) st.rr[j] = part[j];
}

// One iteration of Algorithm 1 over the four wavefronts of the subcarrier:
// the arithmetic of cg_update with the inner products summed over users of
// all wavefronts.
template <typename ST>
__device__ __forceinline__ void wide_cg_step(CGState<1, ST>& st, const float2 (&a)[16], int nk,
                                             WideLds<ST>& lds, const WideLane& L,
                                             ST (&alpha)[4], ST (&beta)[4]) {
  __syncthreads();                                   // previous readers of P are done
  wide_stage<ST>(st.p[0], lds.P, L);
  __syncthreads();
  float2 e[4];
  wide_matvec(a, lds.P, nk, L, e);
  ST pe[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
    pe[j] = (ST)st.p[0][j].x * (ST)e[j].x + (ST)st.p[0][j].y * (ST)e[j].y;
  row_sum16_x4(pe);
  wide_sum(pe, lds, 0, L);                           // Re(p^H e)
  bool live[4];
  ST rr_new[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    live[j] = live_floor<ST>(st.rr[j], pe[j]);
    alpha[j] = live[j] ? div_fast<ST>(st.rr[j], pe[j]) : ST(0);
    const float af = (float)alpha[j];
    st.v[0][j].x = __builtin_fmaf(af, st.p[0][j].x, st.v[0][j].x);
    st.v[0][j].y = __builtin_fmaf(af, st.p[0][j].y, st.v[0][j].y);
    st.r[0][j].x = __builtin_fmaf(-af, e[j].x, st.r[0][j].x);
    st.r[0][j].y = __builtin_fmaf(-af, e[j].y, st.r[0][j].y);
    rr_new[j] = (ST)st.r[0][j].x * (ST)st.r[0][j].x + (ST)st.r[0][j].y * (ST)st.r[0][j].y;
  }
  row_sum16_x4(rr_new);
  wide_sum(rr_new, lds, 1, L);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    beta[j] = live[j] ? div_fast<ST>(rr_new[j], st.rr[j]) : ST(0);
    const float bf = (float)beta[j];
    const float px = __builtin_fmaf(bf, st.p[0][j].x, st.r[0][j].x);
    const float py = __builtin_fmaf(bf, st.p[0][j].y, st.r[0][j].y);
    st.p[0][j].x = live[j] ? px : st.p[0][j].x;
    st.p[0][j].y = live[j] ? py : st.p[0][j].y;
    // (a conditional store rather than a select: the select of the two
    // array elements becomes a select of their addresses with FP64 scalars,
    // which keeps both arrays in scratch memory)
    if (live[j]) st.rr[j] = rr_new[j];
  }
}

// mu (eq. (14)), rho (eq. (15)), z = xhat / mu and the max-log LLRs (eq. (4))
// of the wavefront's users for right-hand sides s0 + 4 g + j, and their
// stores (masked entries dropped by the descriptors' range check).
template <typename ST, int M_BITS>
__device__ __forceinline__ void wide_llr(const DetectParams& prm, int64_t n, int s0,
                                         const float2 (&v)[4], const ST (&tv)[4], const float* Gs,
                                         const WideLane& L) {
  DetectStore<M_BITS> os;
  os.init(prm, n);
  const int u = 16 * L.w + L.c;
  const bool uok = u < prm.U;
  const float Guu = Gs[uok ? u : 0];
  const float rho = Guu / prm.n0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int s = s0 + 4 * L.g + j;
    const float mu = (float)(tv[j] * (ST)Guu);
    // |mu| < FLT_MIN only when the right-hand side froze at (near) zero
    const float imu = fabsf(mu) >= __FLT_MIN__ ? __builtin_amdgcn_rcpf(mu) : 0.f;
    const float2 z = make_float2(v[j].x * imu, v[j].y * imu);
    float out[M_BITS];
    llr_maxlog<M_BITS>(z, rho, prm.scale, prm.inv_scale, out);
    os.store((uok && s < prm.S) ? u * prm.S + s : -1, out, v[j], mu, rho);
  }
}

template <typename ST, int M_BITS>
__global__ __launch_bounds__(256) void detect_wide_kernel(DetectParams prm) {
  __shared__ __align__(16) WideLds<ST> lds;
  const int lane = threadIdx.x & 63;
  const WideLane L{__builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane & 15, lane >> 4, lane};
  const int B = prm.B, U = prm.U, S = prm.S;
  const int nk = __builtin_amdgcn_readfirstlane((U + 3) >> 2);
  for (int64_t n = blockIdx.x; n < prm.n_sc; n += gridDim.x) {
    const void* Hn = offset_sc(InC32{}, prm.H, n, B, U);
    const void* Yn = offset_sc(InC32{}, prm.Y, n, B, S);
    float2 a[16];
    float d[1];
    for (int s0 = 0; s0 < S; s0 += 16) {
      WideAcc acc;
      if (s0 == 0) {
        wide_gram_mf<true, true>(Hn, Yn, B, U, S, s0, L, acc);
        wide_store_a<ST>(acc, lds, prm.reg, U, L, a, d[0]);
      } else {
        wide_gram_mf<false, true>(Hn, Yn, B, U, S, s0, L, acc);
      }
      float2 b[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float p1 = acc.p1[j], p2 = acc.p2[j];
        b[j] = make_float2(p1 + p2, acc.p3[j] - p1 + p2);
      }
      CGState<1, ST> st;
      wide_cg_init<ST>(st, b, lds, L);
      Tracker<1, ST> tk;
      tk.init();
      for (int k = 0; k < prm.K; ++k) {
        ST al[4], be[4];
        wide_cg_step<ST>(st, a, nk, lds, L, al, be);
        tracker_step<1, ST>(tk, d, al, be);
      }
      wide_llr<ST, M_BITS>(prm, n, s0, st.v[0], tk.tv[0], lds.G, L);
    }
    __syncthreads();                                 // LDS of this subcarrier read by all
  }
}

template <typename ST>
__global__ __launch_bounds__(256) void precode_wide_kernel(PrecodeParams prm) {
  __shared__ __align__(16) WideLds<ST> lds;
  const int lane = threadIdx.x & 63;
  const WideLane L{__builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane & 15, lane >> 4, lane};
  const int B = prm.B, U = prm.U, S = prm.S;
  const int nk = __builtin_amdgcn_readfirstlane((U + 3) >> 2);
  const int u = 16 * L.w + L.c;
  for (int64_t n = blockIdx.x; n < prm.n_sc; n += gridDim.x) {
    const void* Hn = offset_sc(InC32{}, prm.H, n, B, U);
    float2 a[16];
    float d;
    {
      WideAcc acc;
      wide_gram_mf<true, false>(Hn, nullptr, B, U, S, 0, L, acc);
      wide_store_a<ST>(acc, lds, prm.beta, U, L, a, d);
    }
    // G operand for ||q||^2 = v^H G v: A's diagonal entries replaced by G_uu
    float2 ga[16];
#pragma unroll
    for (int t = 0; t < 16; ++t)
      ga[t] = (u == 4 * t + L.g) ? make_float2(lds.G[u], 0.f) : a[t];
    const __amdgpu_buffer_rsrc_t rt =
        make_rsrc(prm.T + (size_t)n * U * S, (uint32_t)U * S * 8u);
    const __amdgpu_buffer_rsrc_t rq = make_rsrc(prm.Q + (size_t)n * B * S, (uint32_t)B * S * 8u);
    for (int s0 = 0; s0 < S; s0 += 16) {
      float2 b[4];                                   // b = t
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int s = s0 + 4 * L.g + j;
        b[j] = bload2(rt, (u < U && s < S) ? (uint32_t)(u * S + s) * 8u : kOOB, 0u);
      }
      CGState<1, ST> st;
      wide_cg_init<ST>(st, b, lds, L);
      for (int k = 0; k < prm.K; ++k) {
        ST al[4], be[4];
        wide_cg_step<ST>(st, a, nk, lds, L, al, be);
      }
      // ---- ||q||^2 = v^H G v over all users; V stays in LDS for q = H v
      __syncthreads();
      wide_stage<ST>(st.v[0], lds.P, L);
      __syncthreads();
      float2 e[4];
      wide_matvec(ga, lds.P, nk, L, e);
      ST qq[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        qq[j] = (ST)st.v[0][j].x * (ST)e[j].x + (ST)st.v[0][j].y * (ST)e[j].y;
      row_sum16_x4(qq);
      wide_sum(qq, lds, 0, L);
      float nrm2[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) nrm2[j] = (float)(qq[j] > ST(0) ? qq[j] : ST(0));
      if (L.w == 0 && L.c == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) lds.N[4 * L.g + j] = nrm2[j];
      }
      __syncthreads();
      const float nc = lds.N[L.c];
      const float scl = prm.normalize ? (nc > 0.f ? __builtin_amdgcn_rsqf(nc) : 0.f) : 1.0f;
      // ---- q = H_u v (Algorithm 1 output): 16-antenna tiles w, w + 4, ...;
      // P1 = Hr Vr, P2 = Hi Vi, P3 = (Hr + Hi)(Vr + Vi)
      float2 vv[16];
      float vs[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        vv[t] = lds.P[(4 * t + L.g) * kPST + L.c];
        vs[t] = vv[t].x + vv[t].y;
      }
      const int s = s0 + L.c;
      for (int b0 = 16 * L.w; b0 < B; b0 += 16 * kWideTiles) {
        f4 p1 = zero4(), p2 = zero4(), p3 = zero4();
#pragma unroll
        for (int q = 0; q < 4; ++q) {               // users 16 q .. 16 q + 15
          if (16 * q < U) {
            float2 hv[4];
            load_h_row<4>(InC32{}, Hn, B, U, b0, L.c, q, L.g, hv);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              if (16 * q + 4 * t < U) {
                p1 = mfma4(hv[t].x, vv[4 * q + t].x, p1);
                p2 = mfma4(hv[t].y, vv[4 * q + t].y, p2);
                p3 = mfma4(hv[t].x + hv[t].y, vs[4 * q + t], p3);
              }
            }
          }
        }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int bb = b0 + 4 * L.g + jj;
          const float qr = p1[jj] - p2[jj], qi = p3[jj] - p1[jj] - p2[jj];
          bstore2(rq, (bb < B && s < S) ? (uint32_t)(bb * S + s) * 8u : kOOB, qr * scl, qi * scl);
        }
      }
      if (prm.qnorm && L.w == 0 && L.c == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int ss = s0 + 4 * L.g + j;
          if (ss < S) prm.qnorm[(size_t)n * S + ss] = sqrtf(nrm2[j]);
        }
      }
    }
    __syncthreads();
  }
}

// One workgroup per subcarrier, up to 2^20 workgroups walking the rest.
static unsigned int wide_grid(int64_t n_sc) {
  return (unsigned int)(n_sc < (1 << 20) ? (n_sc > 0 ? n_sc : 1) : (1 << 20));
}

template <typename ST>
static hipError_t launch_detect_wide_st(const DetectParams& p, int m_bits, hipStream_t stream) {
  const dim3 grid(wide_grid(p.n_sc)), block(kWave * kWideTiles);
  switch (m_bits) {
    case 2: hipLaunchKernelGGL((detect_wide_kernel<ST, 2>), grid, block, 0, stream, p); break;
    case 4: hipLaunchKernelGGL((detect_wide_kernel<ST, 4>), grid, block, 0, stream, p); break;
    case 6: hipLaunchKernelGGL((detect_wide_kernel<ST, 6>), grid, block, 0, stream, p); break;
    case 8: hipLaunchKernelGGL((detect_wide_kernel<ST, 8>), grid, block, 0, stream, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_detect_wide(const DetectParams& p, int scalar_f64, int m_bits,
                              hipStream_t stream) {
  return scalar_f64 ? launch_detect_wide_st<double>(p, m_bits, stream)
                    : launch_detect_wide_st<float>(p, m_bits, stream);
}

hipError_t launch_precode_wide(const PrecodeParams& p, int scalar_f64, hipStream_t stream) {
  const dim3 grid(wide_grid(p.n_sc)), block(kWave * kWideTiles);
  if (scalar_f64)
    hipLaunchKernelGGL((precode_wide_kernel<double>), grid, block, 0, stream, p);
  else
    hipLaunchKernelGGL((precode_wide_kernel<float>), grid, block, 0, stream, p);
  return hipGetLastError();
}

}  // namespace mimo

// CGLS on the augmented systems of Sec. III-E: detection solves
// min ||[y; 0] - [H; sqrt(N0/E_s) I] x|| (eq. (17)) and precoding
// min ||t - [H^H, sqrt(beta) I] qbar|| (eq. (18)), by the conjugate-gradient
// least-squares recursion (residual r of the augmented system kept,
// s = Hbar^H r recomputed from it):
//   q = Hbar p;  alpha = gamma / ||q||^2;  x += alpha p;  r -= alpha q;
//   s = Hbar^H r;  gamma' = ||s||^2;  beta = gamma' / gamma;  p = s + beta p.
// No Gram matrix is formed: every iteration runs the two contractions with
// H on MFMA, one 16-antenna tile at a time.  One wavefront per subcarrier
// and 16 right-hand sides per pass.  Two lane layouts meet here:
//   user layout     lane (c, g) holds users 16 w + c, rhs 4 g + j (as CG)
//   antenna layout  lane (c, g) holds antennas b0 + 4 g + j, rhs c
// H v lands in the antenna layout (rows = antennas) and H^H r in the user
// layout, taking the lane's own antenna-layout entries as its A-operand (the
// k-steps of a tile run over j), so antenna-length vectors never move
// between lanes; they live in lane-private LDS slots.  Per-rhs step sizes
// cross between the layouts through a 16-entry LDS array.
// H is read twice per launch here (or once per iteration): keep its lines in
// the caches (default policy for every buffer access).
#define MIMO_CACHE_STREAMING 0
#include "cg_core.hpp"
#include "gram_phase.hpp"
#include "launch.hpp"
#include "llr.hpp"
#include "precode_out.hpp"

namespace mimo {

// H v for the 16 antennas b0 .. b0 + 15 (element j: antenna b0 + 4 g + j,
// rhs c); vv / vs are the staged v[16 w + 4 t + g][c] and Re + Im of it.
template <int W, typename IN>
__device__ __forceinline__ void h_times(IN tag, const void* Hn, int B, int U, int b0, int c,
                                        int g, const float2 (&vv)[W][4], const float (&vs)[W][4],
                                        f4& qr, f4& qi) {
  f4 p1 = zero4(), p2 = zero4(), p3 = zero4();
#pragma unroll
  for (int w = 0; w < W; ++w) {
    float2 hv[4];
    load_h_row<W>(tag, Hn, B, U, b0, c, w, g, hv);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      p1 = mfma4(hv[t].x, vv[w][t].x, p1);
      p2 = mfma4(hv[t].y, vv[w][t].y, p2);
      p3 = mfma4(hv[t].x + hv[t].y, vs[w][t], p3);
    }
  }
  qr = p1 - p2;
  qi = p3 - p1 - p2;
}

// H entries (antenna b0 + 4 g + j, user 16 w + c), zero outside the matrix.
template <int W, typename IN>
__device__ __forceinline__ void h_gather(IN tag, const void* Hn, int B, int U, int b0, int c,
                                         int g, float2 (&h)[W][4]) {
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int b = b0 + 4 * g + j, u = 16 * w + c;
      h[w][j] = (b < B && u < U) ? load_h(tag, Hn, b, u, U) : make_float2(0.f, 0.f);
    }
}

// s += H^H r for one tile: s^T = r^T conj(H), k-step j takes antenna
// b0 + 4 g + j in k-group g (the lane's own r[j]).
template <int W>
__device__ __forceinline__ void hh_times(const float2 (&r)[4], const float2 (&h)[W][4],
                                         f4 (&sr)[W], f4 (&si)[W]) {
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      sr[w] = mfma4(r[j].x, h[w][j].x, sr[w]);
      sr[w] = mfma4(r[j].y, h[w][j].y, sr[w]);
      si[w] = mfma4(r[j].y, h[w][j].x, si[w]);
      si[w] = mfma4(-r[j].x, h[w][j].y, si[w]);
    }
}

// Staged v in the operand order of h_times.
template <int W>
__device__ __forceinline__ void load_staged(const float2* Ps, int c, int g, float2 (&vv)[W][4],
                                            float (&vs)[W][4]) {
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      vv[w][t] = Ps[(16 * w + 4 * t + g) * kPST + c];
      vs[w][t] = vv[w][t].x + vv[w][t].y;
    }
}

// Sum over the four k-groups (lanes c, c + 16, c + 32, c + 48).
template <typename T>
__device__ __forceinline__ T group_sum(T x) {
  x += __shfl_xor(x, 16, 64);
  x += __shfl_xor(x, 32, 64);
  return x;
}

// Per-rhs sums of |x|^2 in the user layout (rhs 4 g + j).
template <int W, typename ST>
__device__ __forceinline__ void user_norms(const float2 (&x)[W][4], ST (&out)[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    out[j] = ST(0);
#pragma unroll
    for (int w = 0; w < W; ++w) out[j] += (ST)x[w][j].x * (ST)x[w][j].x + (ST)x[w][j].y * (ST)x[w][j].y;
  }
  row_sum16_x4(out);
}

__device__ __forceinline__ float2* slot(float2* base, int tile, int lane) {
  return base + ((size_t)tile * kWave + lane) * 4;
}

template <int W, typename IN, typename ST, int M_BITS>
__global__ __launch_bounds__(64) void detect_cgls_kernel(DetectParams prm) {
  constexpr int NU = 16 * W;
  extern __shared__ float4 dyn_lds[];                 // residual: [B/16][64 lanes][4]
  __shared__ __align__(16) float2 Ps[NU * kPST];
  __shared__ ST QQ[16];
  __shared__ float AL[16];
  float2* Rs = (float2*)dyn_lds;
  const int lane = threadIdx.x;
  const int c = lane & 15, g = lane >> 4;
  const int B = prm.B, U = prm.U, S = prm.S;
  const int nt = (B + 15) >> 4;
  const float sreg = sqrtf(prm.reg);
  for (int64_t n = blockIdx.x; n < prm.n_sc; n += gridDim.x) {
    const void* Hn = offset_sc(IN{}, prm.H, n, B, U);
    const void* Yn = offset_sc(IN{}, prm.Y, n, B, S);
    for (int s0 = 0; s0 < S; s0 += 16) {
      // ---- r_0 = [y; 0], s_0 = Hbar^H r_0 = H^H y, column norms G_ii
      f4 sr[W], si[W];
      float gacc[W];
#pragma unroll
      for (int w = 0; w < W; ++w) { sr[w] = zero4(); si[w] = zero4(); gacc[w] = 0.f; }
      for (int bt = 0; bt < nt; ++bt) {
        const int b0 = 16 * bt;
        float2 r[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int b = b0 + 4 * g + j, s = s0 + c;
          r[j] = (b < B && s < S) ? load_h(IN{}, Yn, b, s, S) : make_float2(0.f, 0.f);
        }
        float2* rp = slot(Rs, bt, lane);
#pragma unroll
        for (int j = 0; j < 4; ++j) rp[j] = r[j];
        float2 h[W][4];
        h_gather<W>(IN{}, Hn, B, U, b0, c, g, h);
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int j = 0; j < 4; ++j) gacc[w] += h[w][j].x * h[w][j].x + h[w][j].y * h[w][j].y;
        hh_times<W>(r, h, sr, si);
      }
      float Gii[W], d[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        Gii[w] = group_sum(gacc[w]);
        d[w] = Gii[w] + prm.reg;
      }
      float2 x[W][4], p[W][4], rb[W][4];
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          p[w][j] = make_float2(sr[w][j], si[w][j]);
          x[w][j] = make_float2(0.f, 0.f);
          rb[w][j] = make_float2(0.f, 0.f);        // lower block of the residual
        }
      ST gam[4];
      user_norms<W, ST>(p, gam);
      Tracker<W, ST> tk;
      tk.init();
      for (int k = 0; k < prm.K; ++k) {
        // ---- q = Hbar p: ||H p||^2 (antenna layout) + reg ||p||^2
        stage_vec<W>(Ps, c, g, p);
        wave_lds_sync();
        float2 vv[W][4];
        float vs[W][4];
        load_staged<W>(Ps, c, g, vv, vs);
        ST qq = ST(0);
        for (int bt = 0; bt < nt; ++bt) {
          f4 qr, qi;
          h_times<W>(IN{}, Hn, B, U, 16 * bt, c, g, vv, vs, qr, qi);
#pragma unroll
          for (int j = 0; j < 4; ++j) qq += (ST)qr[j] * (ST)qr[j] + (ST)qi[j] * (ST)qi[j];
        }
        qq = group_sum(qq);
        if (g == 0) QQ[c] = qq;
        ST pp[4];
        user_norms<W, ST>(p, pp);
        wave_lds_sync();
        ST al[4], be[4];
        bool live[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const ST qn = QQ[4 * g + j] + (ST)prm.reg * pp[j];
          live[j] = live_floor<ST>(gam[j], qn);
          al[j] = live[j] ? div_fast<ST>(gam[j], qn) : ST(0);
          const float af = (float)al[j];
#pragma unroll
          for (int w = 0; w < W; ++w) {
            x[w][j].x = __builtin_fmaf(af, p[w][j].x, x[w][j].x);
            x[w][j].y = __builtin_fmaf(af, p[w][j].y, x[w][j].y);
            const float aq = af * sreg;              // q lower block = sqrt(reg) p
            rb[w][j].x = __builtin_fmaf(-aq, p[w][j].x, rb[w][j].x);
            rb[w][j].y = __builtin_fmaf(-aq, p[w][j].y, rb[w][j].y);
          }
        }
        if (c == 0) {
#pragma unroll
          for (int j = 0; j < 4; ++j) AL[4 * g + j] = (float)al[j];
        }
        wave_lds_sync();
        const float ac = AL[c];
        // ---- r_top -= alpha H p, s = H^H r_top + sqrt(reg) r_bot
#pragma unroll
        for (int w = 0; w < W; ++w) { sr[w] = zero4(); si[w] = zero4(); }
        for (int bt = 0; bt < nt; ++bt) {
          const int b0 = 16 * bt;
          f4 qr, qi;
          h_times<W>(IN{}, Hn, B, U, b0, c, g, vv, vs, qr, qi);
          float2* rp = slot(Rs, bt, lane);
          float2 r[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            r[j] = rp[j];
            r[j].x = __builtin_fmaf(-ac, qr[j], r[j].x);
            r[j].y = __builtin_fmaf(-ac, qi[j], r[j].y);
            rp[j] = r[j];
          }
          float2 h[W][4];
          h_gather<W>(IN{}, Hn, B, U, b0, c, g, h);
          hh_times<W>(r, h, sr, si);
        }
        float2 s[W][4];
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            s[w][j] = make_float2(__builtin_fmaf(sreg, rb[w][j].x, sr[w][j]),
                                  __builtin_fmaf(sreg, rb[w][j].y, si[w][j]));
        ST gn[4];
        user_norms<W, ST>(s, gn);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          be[j] = live[j] ? div_fast<ST>(gn[j], gam[j]) : ST(0);
          const float bf = (float)be[j];
#pragma unroll
          for (int w = 0; w < W; ++w) {
            const float px = __builtin_fmaf(bf, p[w][j].x, s[w][j].x);
            const float py = __builtin_fmaf(bf, p[w][j].y, s[w][j].y);
            p[w][j].x = live[j] ? px : p[w][j].x;
            p[w][j].y = live[j] ? py : p[w][j].y;
          }
          gam[j] = live[j] ? gn[j] : gam[j];
        }
        tracker_step<W, ST>(tk, d, al, be);          // eq. (13) on the CGLS steps
      }
      // ---- mu (eq. (14)), rho (eq. (15)), LLRs (eq. (4))
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const int u = 16 * w + c;
        const float rho = Gii[w] / prm.n0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int s = s0 + 4 * g + j;
          const float mu = (float)(tk.tv[w][j] * (ST)Gii[w]);
          const float imu = fabsf(mu) >= __FLT_MIN__ ? __builtin_amdgcn_rcpf(mu) : 0.f;
          const float2 xx = x[w][j];
          float out[M_BITS];
          llr_maxlog<M_BITS>(make_float2(xx.x * imu, xx.y * imu), rho, prm.scale,
                             prm.inv_scale, out);
          if (u < U && s < S) {
            const size_t idx = ((size_t)n * U + u) * S + s;
            float* lp = prm.llr + idx * M_BITS;
#pragma unroll
            for (int q = 0; q < M_BITS; ++q) lp[q] = out[q];
            if (prm.xhat) prm.xhat[idx] = xx;
            if (prm.mu) prm.mu[idx] = mu;
            if (prm.sinr) prm.sinr[idx] = rho;
          }
        }
      }
      wave_lds_sync();
    }
  }
}

template <int W, typename IN, typename ST>
__global__ __launch_bounds__(64) void precode_cgls_kernel(PrecodeParams prm) {
  constexpr int NU = 16 * W;
  extern __shared__ float4 dyn_lds[];   // x_top, p_top, s_top: 3 x [B/16][64 lanes][4]
  __shared__ __align__(16) float2 Ps[NU * kPST];
  __shared__ ST QQ[16];
  __shared__ float AL[16], BE[16];
  const int lane = threadIdx.x;
  const int c = lane & 15, g = lane >> 4;
  const int B = prm.B, U = prm.U, S = prm.S;
  const int nt = (B + 15) >> 4;
  float2* Xt = (float2*)dyn_lds;
  float2* Pt = Xt + (size_t)nt * kWave * 4;
  float2* St = Pt + (size_t)nt * kWave * 4;
  const float sb = sqrtf(prm.beta);
  for (int64_t n = blockIdx.x; n < prm.n_sc; n += gridDim.x) {
    const void* Hn = offset_sc(IN{}, prm.H, n, B, U);
    for (int s0 = 0; s0 < S; s0 += 16) {
      // ---- r_0 = t, s_0 = Hbar_d^H t = [H t; sqrt(beta) t], p_0 = s_0, x_0 = 0
      float2 r[W][4], xb[W][4], pb[W][4];
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int u = 16 * w + c, s = s0 + 4 * g + j;
          r[w][j] = (u < U && s < S) ? prm.T[((size_t)n * U + u) * S + s] : make_float2(0.f, 0.f);
          xb[w][j] = make_float2(0.f, 0.f);
          pb[w][j] = make_float2(sb * r[w][j].x, sb * r[w][j].y);
        }
      stage_vec<W>(Ps, c, g, r);
      wave_lds_sync();
      float2 vv[W][4];
      float vs[W][4];
      load_staged<W>(Ps, c, g, vv, vs);
      ST st2 = ST(0);
      for (int bt = 0; bt < nt; ++bt) {
        f4 qr, qi;
        h_times<W>(IN{}, Hn, B, U, 16 * bt, c, g, vv, vs, qr, qi);
        float2* xp = slot(Xt, bt, lane);
        float2* pp = slot(Pt, bt, lane);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          xp[j] = make_float2(0.f, 0.f);
          pp[j] = make_float2(qr[j], qi[j]);
          st2 += (ST)qr[j] * (ST)qr[j] + (ST)qi[j] * (ST)qi[j];
        }
      }
      st2 = group_sum(st2);
      if (g == 0) QQ[c] = st2;
      ST gam[4];
      user_norms<W, ST>(pb, gam);                    // ||sqrt(beta) t||^2
      wave_lds_sync();
#pragma unroll
      for (int j = 0; j < 4; ++j) gam[j] += QQ[4 * g + j];
      for (int k = 0; k < prm.K; ++k) {
        // ---- q = Hbar_d p = H^H p_top + sqrt(beta) p_bot (user layout)
        f4 sr[W], si[W];
#pragma unroll
        for (int w = 0; w < W; ++w) { sr[w] = zero4(); si[w] = zero4(); }
        for (int bt = 0; bt < nt; ++bt) {
          const float2* pp = slot(Pt, bt, lane);
          float2 pt[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) pt[j] = pp[j];
          float2 h[W][4];
          h_gather<W>(IN{}, Hn, B, U, 16 * bt, c, g, h);
          hh_times<W>(pt, h, sr, si);
        }
        float2 q[W][4];
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            q[w][j] = make_float2(__builtin_fmaf(sb, pb[w][j].x, sr[w][j]),
                                  __builtin_fmaf(sb, pb[w][j].y, si[w][j]));
        ST qq[4];
        user_norms<W, ST>(q, qq);
        ST al[4];
        bool live[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          live[j] = live_floor<ST>(gam[j], qq[j]);
          al[j] = live[j] ? div_fast<ST>(gam[j], qq[j]) : ST(0);
          const float af = (float)al[j];
#pragma unroll
          for (int w = 0; w < W; ++w) {
            xb[w][j].x = __builtin_fmaf(af, pb[w][j].x, xb[w][j].x);
            xb[w][j].y = __builtin_fmaf(af, pb[w][j].y, xb[w][j].y);
            r[w][j].x = __builtin_fmaf(-af, q[w][j].x, r[w][j].x);
            r[w][j].y = __builtin_fmaf(-af, q[w][j].y, r[w][j].y);
          }
        }
        if (c == 0) {
#pragma unroll
          for (int j = 0; j < 4; ++j) AL[4 * g + j] = (float)al[j];
        }
        // ---- s = Hbar_d^H r = [H r; sqrt(beta) r]; x_top += alpha p_top
        stage_vec<W>(Ps, c, g, r);
        wave_lds_sync();
        const float ac = AL[c];
        load_staged<W>(Ps, c, g, vv, vs);
        ST sn = ST(0);
        for (int bt = 0; bt < nt; ++bt) {
          f4 qr, qi;
          h_times<W>(IN{}, Hn, B, U, 16 * bt, c, g, vv, vs, qr, qi);
          float2* xp = slot(Xt, bt, lane);
          const float2* pp = slot(Pt, bt, lane);
          float2* sp = slot(St, bt, lane);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float2 pt = pp[j];
            float2 xt = xp[j];
            xt.x = __builtin_fmaf(ac, pt.x, xt.x);
            xt.y = __builtin_fmaf(ac, pt.y, xt.y);
            xp[j] = xt;
            sp[j] = make_float2(qr[j], qi[j]);
            sn += (ST)qr[j] * (ST)qr[j] + (ST)qi[j] * (ST)qi[j];
          }
        }
        sn = group_sum(sn);
        if (g == 0) QQ[c] = sn;
        float2 sbv[W][4];
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int j = 0; j < 4; ++j) sbv[w][j] = make_float2(sb * r[w][j].x, sb * r[w][j].y);
        ST gl[4];
        user_norms<W, ST>(sbv, gl);
        wave_lds_sync();
        ST be[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const ST gn = gl[j] + QQ[4 * g + j];
          be[j] = live[j] ? div_fast<ST>(gn, gam[j]) : ST(0);
          const float bf = (float)be[j];
#pragma unroll
          for (int w = 0; w < W; ++w) {
            const float px = __builtin_fmaf(bf, pb[w][j].x, sbv[w][j].x);
            const float py = __builtin_fmaf(bf, pb[w][j].y, sbv[w][j].y);
            pb[w][j].x = live[j] ? px : pb[w][j].x;
            pb[w][j].y = live[j] ? py : pb[w][j].y;
          }
          gam[j] = live[j] ? gn : gam[j];
        }
        // ---- p_top = s_top + beta p_top (frozen rhs keep p)
        if (c == 0) {
#pragma unroll
          for (int j = 0; j < 4; ++j) BE[4 * g + j] = live[j] ? (float)be[j] : -1.f;
        }
        wave_lds_sync();
        const float bc = BE[c];
        const bool lc = bc >= 0.f;
        for (int bt = 0; bt < nt; ++bt) {
          float2* pp = slot(Pt, bt, lane);
          const float2* sp = slot(St, bt, lane);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const float2 pt = pp[j], sv = sp[j];
            if (lc) pp[j] = make_float2(__builtin_fmaf(bc, pt.x, sv.x), __builtin_fmaf(bc, pt.y, sv.y));
          }
        }
      }
      // ---- q = qbar[0 .. B): ||q|| per rhs, optional normalization (Sec. II-B)
      ST qn2 = ST(0);
      for (int bt = 0; bt < nt; ++bt) {
        const float2* xp = slot(Xt, bt, lane);
#pragma unroll
        for (int j = 0; j < 4; ++j) qn2 += (ST)xp[j].x * (ST)xp[j].x + (ST)xp[j].y * (ST)xp[j].y;
      }
      qn2 = group_sum(qn2);
      const float nrm2 = (float)qn2;
      const float scl = prm.normalize ? (nrm2 > 0.f ? __builtin_amdgcn_rsqf(nrm2) : 0.f) : 1.f;
      const int s = s0 + c;
      if (s < S) {
        for (int bt = 0; bt < nt; ++bt) {
          const float2* xp = slot(Xt, bt, lane);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int b = 16 * bt + 4 * g + j;
            if (b < B) prm.Q[((size_t)n * B + b) * S + s] = make_float2(xp[j].x * scl, xp[j].y * scl);
          }
        }
        if (prm.qnorm && g == 0) prm.qnorm[(size_t)n * S + s] = sqrtf(nrm2);
      }
      wave_lds_sync();
    }
  }
}

static dim3 sc_grid1(int64_t n_sc) {
  int64_t blocks = n_sc < (1 << 20) ? n_sc : (1 << 20);
  return dim3((unsigned)(blocks < 1 ? 1 : blocks));
}

size_t cgls_lds_bytes(int B, bool precode) {
  const size_t tiles = (size_t)(B + 15) / 16;
  return tiles * kWave * 4 * sizeof(float2) * (precode ? 3 : 1);
}

template <int W, typename IN, typename ST>
static hipError_t launch_detect_cgls_m(const DetectParams& p, int m_bits, hipStream_t stream) {
  const dim3 grid = sc_grid1(p.n_sc), block(kWave);
  const size_t lds = cgls_lds_bytes(p.B, false);
  switch (m_bits) {
    case 2: hipLaunchKernelGGL((detect_cgls_kernel<W, IN, ST, 2>), grid, block, lds, stream, p); break;
    case 4: hipLaunchKernelGGL((detect_cgls_kernel<W, IN, ST, 4>), grid, block, lds, stream, p); break;
    case 6: hipLaunchKernelGGL((detect_cgls_kernel<W, IN, ST, 6>), grid, block, lds, stream, p); break;
    case 8: hipLaunchKernelGGL((detect_cgls_kernel<W, IN, ST, 8>), grid, block, lds, stream, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int W, typename IN>
static hipError_t launch_detect_cgls_st(const DetectParams& p, int f64, int m_bits,
                                        hipStream_t stream) {
  return f64 ? launch_detect_cgls_m<W, IN, double>(p, m_bits, stream)
             : launch_detect_cgls_m<W, IN, float>(p, m_bits, stream);
}

template <int W>
static hipError_t launch_detect_cgls_in(const DetectParams& p, int in_dtype, int f64, int m_bits,
                                        hipStream_t stream) {
  switch (in_dtype) {
    case 0: return launch_detect_cgls_st<W, InC32>(p, f64, m_bits, stream);
    case 1: return launch_detect_cgls_st<W, InF16>(p, f64, m_bits, stream);
    case 2: return launch_detect_cgls_st<W, InBF16>(p, f64, m_bits, stream);
  }
  return hipErrorInvalidValue;
}

template <int W, typename IN>
static hipError_t launch_precode_cgls_st(const PrecodeParams& p, int f64, hipStream_t stream) {
  const dim3 grid = sc_grid1(p.n_sc), block(kWave);
  const size_t lds = cgls_lds_bytes(p.B, true);
  if (f64)
    hipLaunchKernelGGL((precode_cgls_kernel<W, IN, double>), grid, block, lds, stream, p);
  else
    hipLaunchKernelGGL((precode_cgls_kernel<W, IN, float>), grid, block, lds, stream, p);
  return hipGetLastError();
}

template <int W>
static hipError_t launch_precode_cgls_in(const PrecodeParams& p, int in_dtype, int f64,
                                         hipStream_t stream) {
  switch (in_dtype) {
    case 0: return launch_precode_cgls_st<W, InC32>(p, f64, stream);
    case 1: return launch_precode_cgls_st<W, InF16>(p, f64, stream);
    case 2: return launch_precode_cgls_st<W, InBF16>(p, f64, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_detect_cgls(const DetectParams& p, int in_dtype, int scalar_f64, int m_bits,
                              hipStream_t stream) {
  return p.U <= 16 ? launch_detect_cgls_in<1>(p, in_dtype, scalar_f64, m_bits, stream)
                   : launch_detect_cgls_in<2>(p, in_dtype, scalar_f64, m_bits, stream);
}

hipError_t launch_precode_cgls(const PrecodeParams& p, int in_dtype, int scalar_f64,
                               hipStream_t stream) {
  return p.U <= 16 ? launch_precode_cgls_in<1>(p, in_dtype, scalar_f64, stream)
                   : launch_precode_cgls_in<2>(p, in_dtype, scalar_f64, stream);
}

}  // namespace mimo

// Conjugate gradient (Algorithm 1) for one subcarrier per wavefront.
//
// Lane (c, g) = lane % 16, lane / 16 owns users u = 16 w + c (w < W) and
// right-hand sides s = s0 + 4 g + j (j < 4): the 16 lanes of a DPP row hold
// one right-hand side's vector, so inner products over users are a row sum
// (four DPP steps) plus a sum over w inside the lane.  A is in the wave's
// LDS region; the search direction p is exchanged through LDS for the
// mat-vec e = A p.  Vectors are FP32; the scalar recurrences (||r||^2,
// p^H e, alpha, beta) use ST (float or double).
#pragma once

#include "common.hpp"

namespace mimo {

template <int W, typename ST>
struct CGState {
  float2 v[W][4], r[W][4], p[W][4];
  ST rr[4];                  // ||r_{k-1}||^2 of each right-hand side
};

// Approximate SINR tracker of eq. (13): with A replaced by D = diag(A) the
// matrices stay diagonal and each entry follows Algorithm 1 on the scalar
// d_i with the CG's own alpha_k, beta_k (v~_0 = 0, r~_0 = p~_0 = 1).
template <int W, typename ST>
struct Tracker {
  ST tv[W][4], tr[W][4], tp[W][4];
  __device__ void init() {
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int j = 0; j < 4; ++j) { tv[w][j] = ST(0); tr[w][j] = ST(1); tp[w][j] = ST(1); }
  }
};

template <typename ST>
__device__ __forceinline__ ST to_st(float x) { return (ST)x; }

template <int W, typename ST>
__device__ __forceinline__ void cg_init(CGState<W, ST>& st, const float2 (&b)[W][4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ST part = ST(0);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      st.v[w][j] = make_float2(0.f, 0.f);
      st.r[w][j] = b[w][j];
      st.p[w][j] = b[w][j];
      part += (ST)b[w][j].x * (ST)b[w][j].x + (ST)b[w][j].y * (ST)b[w][j].y;
    }
    st.rr[j] = row_sum16(part);
  }
}

// e[w][j] = (A x)_{16 w + c} for the 4 right-hand sides of this lane, with x
// staged in Ps (row = rhs within the chunk, column = user).
template <int W>
__device__ __forceinline__ void matvec(const float2* __restrict__ As, const float2* __restrict__ Ps,
                                       int ast, int c, int g, float2 (&e)[W][4]) {
  constexpr int NU = 16 * W;
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int j = 0; j < 4; ++j) e[w][j] = make_float2(0.f, 0.f);
#pragma unroll 2
  for (int k = 0; k < NU; k += 2) {
    float4 a[W], x[4];
#pragma unroll
    for (int w = 0; w < W; ++w) a[w] = *(const float4*)&As[(16 * w + c) * ast + k];
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = *(const float4*)&Ps[(4 * g + j) * ast + k];
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        cfma(e[w][j], make_float2(a[w].x, a[w].y), make_float2(x[j].x, x[j].y));
        cfma(e[w][j], make_float2(a[w].z, a[w].w), make_float2(x[j].z, x[j].w));
      }
  }
}

template <int W>
__device__ __forceinline__ void stage_vec(float2* __restrict__ Ps, int ast, int c, int g,
                                          const float2 (&x)[W][4]) {
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int j = 0; j < 4; ++j) Ps[(4 * g + j) * ast + 16 * w + c] = x[w][j];
}

// One iteration of Algorithm 1 (loop body) for the lane's 4 right-hand
// sides.  alpha/beta are returned for the trackers.  A right-hand side whose
// residual norm is zero (converged or b = 0) freezes: alpha = beta = 0.
template <int W, typename ST>
__device__ __forceinline__ void cg_step(CGState<W, ST>& st, const float2* __restrict__ As,
                                        float2* __restrict__ Ps, int ast, int c, int g,
                                        ST (&alpha)[4], ST (&beta)[4]) {
  stage_vec<W>(Ps, ast, c, g, st.p);
  wave_lds_sync();
  float2 e[W][4];
  matvec<W>(As, Ps, ast, c, g, e);                 // e_{k-1} = A p_{k-1}
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ST part = ST(0);
#pragma unroll
    for (int w = 0; w < W; ++w)
      part += (ST)st.p[w][j].x * (ST)e[w][j].x + (ST)st.p[w][j].y * (ST)e[w][j].y;
    const ST pe = row_sum16(part);                 // Re(p^H e)
    const bool live = st.rr[j] > ST(0) && pe > ST(0);
    alpha[j] = live ? st.rr[j] / pe : ST(0);
    const float af = (float)alpha[j];
    ST part2 = ST(0);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      st.v[w][j].x = __builtin_fmaf(af, st.p[w][j].x, st.v[w][j].x);
      st.v[w][j].y = __builtin_fmaf(af, st.p[w][j].y, st.v[w][j].y);
      st.r[w][j].x = __builtin_fmaf(-af, e[w][j].x, st.r[w][j].x);
      st.r[w][j].y = __builtin_fmaf(-af, e[w][j].y, st.r[w][j].y);
      part2 += (ST)st.r[w][j].x * (ST)st.r[w][j].x + (ST)st.r[w][j].y * (ST)st.r[w][j].y;
    }
    const ST rr_new = row_sum16(part2);
    beta[j] = live ? rr_new / st.rr[j] : ST(0);
    const float bf = (float)beta[j];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      if (live) {
        st.p[w][j].x = __builtin_fmaf(bf, st.p[w][j].x, st.r[w][j].x);
        st.p[w][j].y = __builtin_fmaf(bf, st.p[w][j].y, st.r[w][j].y);
      }
    }
    if (live) st.rr[j] = rr_new;
  }
}

template <int W, typename ST>
__device__ __forceinline__ void tracker_step(Tracker<W, ST>& tk, const float (&d)[W],
                                             const ST (&alpha)[4], const ST (&beta)[4]) {
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      tk.tv[w][j] = tk.tv[w][j] + alpha[j] * tk.tp[w][j];
      tk.tr[w][j] = tk.tr[w][j] - alpha[j] * (ST)d[w] * tk.tp[w][j];
      tk.tp[w][j] = tk.tr[w][j] + beta[j] * tk.tp[w][j];
    }
}

}  // namespace mimo

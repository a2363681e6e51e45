// Conjugate gradient (Algorithm 1) for one subcarrier per wavefront.
//
// Lane (c, g) = lane % 16, lane / 16 owns users u = 16 w + c (w < W) and
// right-hand sides s = s0 + 4 g + j (j < 4): the 16 lanes of a DPP row hold
// one right-hand side's vector, so inner products over users are a row sum
// (four DPP steps) plus a sum over w inside the lane.  Vectors are FP32; the
// scalar recurrences (||r||^2, p^H e, alpha, beta) use ST (float or double).
//
// The mat-vec e = A p of all right-hand sides at once is the product
// E = A P, computed on MFMA in transposed form E^T = P^T A^T (rows =
// right-hand sides, columns = users) so that the result lands in the lane
// layout above.  P is exchanged through LDS as P[user][rhs]; the A^T operand
// (A[16 w + c][k] for the lane's k-group) stays in registers.
#pragma once

#include "common.hpp"

namespace mimo {

constexpr int kPST = 18;   // LDS row stride (complex) of P[user][rhs]

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

// A^T operand of the mat-vec: a[wc][t] = A[16 wc + c][4 t + g].  nk = the
// k-steps (4 users each) that reach a real user, ceil(U / 4): the vectors the
// CG multiplies are zero on padding users (b is zero there and A keeps them
// decoupled), so later k-steps would add exact zeros and are skipped.  A
// caller whose vectors are not zero on padding users passes U = 16 W.
template <int W>
struct AOperand {
  float2 a[W][4 * W];
  int nk;
  const float2* rows;   // the wave's LDS copy of A (row stride ast), for matvec_valu
  int ast, U;
  __device__ void load(const float2* __restrict__ As, int ast_, int c, int g, int U_) {
    rows = As;
    ast = ast_;
    U = U_;
    const int k = (U + 3) >> 2;
    nk = __builtin_amdgcn_readfirstlane(k < 4 * W ? k : 4 * W);
#pragma unroll
    for (int wc = 0; wc < W; ++wc)
#pragma unroll
      for (int t = 0; t < 4 * W; ++t) a[wc][t] = As[(16 * wc + c) * ast + 4 * t + g];
  }
};

// Scalar division of the recurrences.  FP32 uses the hardware reciprocal; it
// is only reached for operands >= FLT_MIN (see live_floor), where the
// reciprocal is finite and within 1 ulp.  FP64 divides exactly.
template <typename ST>
__device__ __forceinline__ ST div_fast(ST a, ST b) { return a / b; }
template <>
__device__ __forceinline__ float div_fast<float>(float a, float b) {
  return a * __builtin_amdgcn_rcpf(b);
}

// A right-hand side is live while ||r||^2 and p^H e are at least this value.
// FP64: any positive value (freeze only on an exact zero, as Algorithm 1
// leaves beta undefined there).  FP32: the smallest normal float -- past
// convergence the recursive residual keeps shrinking geometrically into
// denormals, where 1/x overflows; freezing there changes v by less than
// FP32 round-off.
template <typename ST>
__device__ __forceinline__ bool live_floor(ST rr, ST pe);
template <>
__device__ __forceinline__ bool live_floor<double>(double rr, double pe) {
  return rr > 0.0 && pe > 0.0;
}
template <>
__device__ __forceinline__ bool live_floor<float>(float rr, float pe) {
  return rr >= __FLT_MIN__ && pe >= __FLT_MIN__;
}

template <int W, typename ST>
__device__ __forceinline__ void cg_init(CGState<W, ST>& st, const float2 (&b)[W][4]) {
  ST part[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    part[j] = (ST)b[0][j].x * (ST)b[0][j].x + (ST)b[0][j].y * (ST)b[0][j].y;
#pragma unroll
    for (int w = 1; w < W; ++w)
      part[j] += (ST)b[w][j].x * (ST)b[w][j].x + (ST)b[w][j].y * (ST)b[w][j].y;
#pragma unroll
    for (int w = 0; w < W; ++w) {
      st.v[w][j] = make_float2(0.f, 0.f);
      st.r[w][j] = b[w][j];
      st.p[w][j] = b[w][j];
    }
  }
  row_sum16_x4(part);
#pragma unroll
  for (int j = 0; j < 4; ++j) st.rr[j] = part[j];
}

// Stage x (lane layout) to LDS as X[user][rhs].
template <int W>
__device__ __forceinline__ void stage_vec(float2* __restrict__ Ps, int c, int g,
                                          const float2 (&x)[W][4]) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    float4* d = (float4*)&Ps[(16 * w + c) * kPST + 4 * g];
    d[0] = make_float4(x[w][0].x, x[w][0].y, x[w][1].x, x[w][1].y);
    d[1] = make_float4(x[w][2].x, x[w][2].y, x[w][3].x, x[w][3].y);
  }
}

// e = A x for the staged X: E^T = X^T A^T on 16x16x4 MFMA, k over users.
template <int W>
__device__ __forceinline__ void matvec_mfma(const AOperand<W>& at, const float2* __restrict__ Ps,
                                            int c, int g, float2 (&e)[W][4]) {
  f4 er[W], ei[W];
#pragma unroll
  for (int w = 0; w < W; ++w) { er[w] = zero4(); ei[w] = zero4(); }
#pragma unroll
  for (int t = 0; t < 4 * W; ++t) {
    if (t >= at.nk) break;                            // users >= 4 t are padding
    const float2 pk = Ps[(4 * t + g) * kPST + c];     // X[k = 4 t + g][rhs c]
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const float2 a = at.a[w][t];
      er[w] = mfma4(pk.x, a.x, er[w]);
      ei[w] = mfma4(pk.x, a.y, ei[w]);
      er[w] = mfma4(-pk.y, a.y, er[w]);
      ei[w] = mfma4(pk.y, a.x, ei[w]);
    }
  }
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int j = 0; j < 4; ++j) e[w][j] = make_float2(er[w][j], ei[w][j]);
}

// e = A x with VALU FMAs instead of MFMA (a measured alternative, schedule
// variant "stream-valu"): lane (c, g) forms e[16 w + c][4 g + j] as
// sum_k A[16 w + c][k] X[k][4 g + j] over the users k < U, with A from the
// wave's LDS copy and X[k][.] from the staged vectors (the 16 lanes of a DPP
// row read the same address: a broadcast).  Terms k >= U are exact zeros
// and are skipped.  Sums in another order than the MFMA form.
template <int W>
__device__ __forceinline__ void matvec_valu(const AOperand<W>& at, const float2* __restrict__ Ps,
                                            int c, int g, float2 (&e)[W][4]) {
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int j = 0; j < 4; ++j) e[w][j] = make_float2(0.f, 0.f);
  for (int k = 0; k < at.U; ++k) {
    const float4 x01 = *(const float4*)&Ps[k * kPST + 4 * g];
    const float4 x23 = *(const float4*)&Ps[k * kPST + 4 * g + 2];
    const float2 x[4] = {make_float2(x01.x, x01.y), make_float2(x01.z, x01.w),
                         make_float2(x23.x, x23.y), make_float2(x23.z, x23.w)};
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const float2 a = at.rows[(16 * w + c) * at.ast + k];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        e[w][j].x = __builtin_fmaf(a.x, x[j].x, e[w][j].x);
        e[w][j].x = __builtin_fmaf(-a.y, x[j].y, e[w][j].x);
        e[w][j].y = __builtin_fmaf(a.x, x[j].y, e[w][j].y);
        e[w][j].y = __builtin_fmaf(a.y, x[j].x, e[w][j].y);
      }
    }
  }
}

// The part of one iteration of Algorithm 1 (loop body) after the mat-vec
// e = A p, for the lane's 4 right-hand sides: step size, v, r, residual
// norm, beta, p.  alpha/beta are returned for the trackers.  A right-hand
// side whose residual norm is zero (converged or b = 0) freezes: alpha =
// beta = 0.  Branch-free (selects), with the four right-hand sides'
// reductions interleaved.
template <int W, typename ST>
__device__ __forceinline__ void cg_update(CGState<W, ST>& st, const float2 (&e)[W][4],
                                          ST (&alpha)[4], ST (&beta)[4]) {
  ST pe[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    pe[j] = (ST)st.p[0][j].x * (ST)e[0][j].x + (ST)st.p[0][j].y * (ST)e[0][j].y;
#pragma unroll
    for (int w = 1; w < W; ++w)
      pe[j] += (ST)st.p[w][j].x * (ST)e[w][j].x + (ST)st.p[w][j].y * (ST)e[w][j].y;
  }
  row_sum16_x4(pe);                                // Re(p^H e)
  bool live[4];
  ST rr_new[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    live[j] = live_floor<ST>(st.rr[j], pe[j]);
    alpha[j] = live[j] ? div_fast<ST>(st.rr[j], pe[j]) : ST(0);
    const float af = (float)alpha[j];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      st.v[w][j].x = __builtin_fmaf(af, st.p[w][j].x, st.v[w][j].x);
      st.v[w][j].y = __builtin_fmaf(af, st.p[w][j].y, st.v[w][j].y);
      st.r[w][j].x = __builtin_fmaf(-af, e[w][j].x, st.r[w][j].x);
      st.r[w][j].y = __builtin_fmaf(-af, e[w][j].y, st.r[w][j].y);
    }
    rr_new[j] = (ST)st.r[0][j].x * (ST)st.r[0][j].x + (ST)st.r[0][j].y * (ST)st.r[0][j].y;
#pragma unroll
    for (int w = 1; w < W; ++w)
      rr_new[j] += (ST)st.r[w][j].x * (ST)st.r[w][j].x + (ST)st.r[w][j].y * (ST)st.r[w][j].y;
  }
  row_sum16_x4(rr_new);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    beta[j] = live[j] ? div_fast<ST>(rr_new[j], st.rr[j]) : ST(0);
    const float bf = (float)beta[j];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const float px = __builtin_fmaf(bf, st.p[w][j].x, st.r[w][j].x);
      const float py = __builtin_fmaf(bf, st.p[w][j].y, st.r[w][j].y);
      st.p[w][j].x = live[j] ? px : st.p[w][j].x;
      st.p[w][j].y = live[j] ? py : st.p[w][j].y;
    }
    st.rr[j] = live[j] ? rr_new[j] : st.rr[j];
  }
}

// One iteration of Algorithm 1 (loop body): P through LDS, e = A p, then
// cg_update.
// VALU: the mat-vec on VALU FMAs (matvec_valu) instead of MFMA.
template <int W, typename ST, bool VALU = false>
__device__ __forceinline__ void cg_step(CGState<W, ST>& st, const AOperand<W>& at,
                                        float2* __restrict__ Ps, int c, int g, ST (&alpha)[4],
                                        ST (&beta)[4]) {
  stage_vec<W>(Ps, c, g, st.p);
  wave_lds_sync();
  float2 e[W][4];
  if constexpr (VALU) matvec_valu<W>(at, Ps, c, g, e);   // e_{k-1} = A p_{k-1}
  else matvec_mfma<W>(at, Ps, c, g, e);
  wave_lds_sync();
  cg_update<W, ST>(st, e, alpha, beta);
}

// One iteration each of two independent systems of the same subcarrier (the
// uplink and downlink systems of a slot): their P go through LDS together
// (Pa, Pb), both mat-vecs follow one exchange, and the two updates, which
// do not depend on each other, can overlap.  Per system the operations are
// those of cg_step, in the same order.
template <int W, typename ST>
__device__ __forceinline__ void cg_step2(CGState<W, ST>& sa, const AOperand<W>& ata,
                                         float2* __restrict__ Pa, ST (&aa)[4], ST (&ba)[4],
                                         CGState<W, ST>& sb, const AOperand<W>& atb,
                                         float2* __restrict__ Pb, ST (&ab)[4], ST (&bb)[4],
                                         int c, int g) {
  stage_vec<W>(Pa, c, g, sa.p);
  stage_vec<W>(Pb, c, g, sb.p);
  wave_lds_sync();
  float2 ea[W][4], eb[W][4];
  matvec_mfma<W>(ata, Pa, c, g, ea);
  matvec_mfma<W>(atb, Pb, c, g, eb);
  wave_lds_sync();
  cg_update<W, ST>(sa, ea, aa, ba);
  cg_update<W, ST>(sb, eb, ab, bb);
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

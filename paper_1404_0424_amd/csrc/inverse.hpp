// Explicit inverses of the regularized Gram matrix A for the comparison
// methods of Sec. III-F: the exact inverse through the Cholesky factor and
// the truncated Neumann series.  One wavefront per subcarrier; matrices are
// complex64 in the wave's LDS with row stride `ast` (NU = 16 W rows).
// Padding users (>= U) carry a unit diagonal, so the padded matrix is
// block diagonal with an identity block and stays invertible.
#pragma once

#include "cg_core.hpp"
#include "gram_phase.hpp"

namespace mimo {

// Unit diagonal for the padding users (their rows and columns of A are zero
// apart from the diagonal, which the Gram phase set to the regularizer).
template <int W>
__device__ __forceinline__ void pad_unit_diagonal(float2* As, int ast, int U, int lane) {
  if (lane >= U && lane < 16 * W) As[lane * ast + lane] = make_float2(1.f, 0.f);
}

// Entries of an NU x NU matrix owned by lane (c, g):
// e[wr][wc][t] = (16 wr + c, 16 wc + 4 g + t).
template <int W>
using Owned = float2[W][W][4];

// A = M M^H and X = M^{-1} (Sec. III-F-1), one column per step: step j takes
// the pivot of the trailing matrix, forms column j of M, updates the
// trailing matrix by -M(:,j) M(:,j)^H (right-looking) and finishes row j of
// X by forward substitution of M X = I (row j scaled by 1/M_jj, then
// subtracted from the rows below with weights M(i,j)).  The current column of
// the trailing matrix and row j of X pass through LDS (`xch`: two ping-pong
// buffers of 2 x NU entries, one wave-level sync per step).  Steps stop at U:
// the padding block is already the identity in both matrices.  A must be
// positive definite; a non-positive pivot gives non-finite output.
template <int W>
__device__ __forceinline__ void cholesky_inverse(const float2* As, int ast, int U, float2* xch,
                                                 int c, int g, Owned<W>& X) {
  constexpr int NU = 16 * W;
  Owned<W> T;   // trailing matrix
#pragma unroll
  for (int wr = 0; wr < W; ++wr)
#pragma unroll
    for (int wc = 0; wc < W; ++wc)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = 16 * wr + c, k = 16 * wc + 4 * g + t;
        T[wr][wc][t] = As[i * ast + k];
        X[wr][wc][t] = make_float2(i == k ? 1.f : 0.f, 0.f);
      }
  for (int j = 0; j < U; ++j) {
    float2* col = xch + (j & 1) * 2 * NU;
    float2* row = col + NU;
    const int jw = j >> 4, jg = (j & 15) >> 2, jt = j & 3;
    if (g == jg) {                           // column j of the trailing matrix
#pragma unroll
      for (int wr = 0; wr < W; ++wr) {
        float2 v = make_float2(0.f, 0.f);
#pragma unroll
        for (int wc = 0; wc < W; ++wc)
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (wc == jw && t == jt) v = T[wr][wc][t];
        col[16 * wr + c] = v;
      }
    }
    if (c == (j & 15)) {                     // row j of X (before scaling)
#pragma unroll
      for (int wr = 0; wr < W; ++wr)
        if (wr == jw)
#pragma unroll
          for (int wc = 0; wc < W; ++wc)
#pragma unroll
            for (int t = 0; t < 4; ++t) row[16 * wc + 4 * g + t] = X[wr][wc][t];
    }
    wave_lds_sync();
    const float inv_d = __builtin_amdgcn_rsqf(col[j].x);     // 1 / M_jj
    float2 li[W];                                             // M(i, j), 0 for i <= j
#pragma unroll
    for (int wr = 0; wr < W; ++wr) {
      const int i = 16 * wr + c;
      const float2 a = col[i];
      li[wr] = i > j ? make_float2(a.x * inv_d, a.y * inv_d) : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int wc = 0; wc < W; ++wc)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = 16 * wc + 4 * g + t;
        const float2 a = col[k];
        const float2 lk = k > j ? make_float2(a.x * inv_d, a.y * inv_d) : make_float2(0.f, 0.f);
        const float2 r = row[k];
        const float2 xj = make_float2(r.x * inv_d, r.y * inv_d);   // X(j, k)
#pragma unroll
        for (int wr = 0; wr < W; ++wr) {
          const int i = 16 * wr + c;
          float2& tt = T[wr][wc][t];
          // T(i, k) -= M(i, j) conj(M(k, j))
          tt.x = __builtin_fmaf(-li[wr].x, lk.x, tt.x);
          tt.x = __builtin_fmaf(-li[wr].y, lk.y, tt.x);
          tt.y = __builtin_fmaf(-li[wr].y, lk.x, tt.y);
          tt.y = __builtin_fmaf(li[wr].x, lk.y, tt.y);
          // X(i, k) -= M(i, j) X(j, k) below row j; row j takes its final value
          float2& xx = X[wr][wc][t];
          float2 xn;
          xn.x = __builtin_fmaf(-li[wr].x, xj.x, xx.x);
          xn.x = __builtin_fmaf(li[wr].y, xj.y, xn.x);
          xn.y = __builtin_fmaf(-li[wr].x, xj.y, xx.y);
          xn.y = __builtin_fmaf(-li[wr].y, xj.x, xn.y);
          xx = i == j ? xj : xn;
        }
      }
  }
}

template <int W>
__device__ __forceinline__ void store_owned(float2* Xs, int ast, int c, int g, const Owned<W>& X) {
#pragma unroll
  for (int wr = 0; wr < W; ++wr)
#pragma unroll
    for (int wc = 0; wc < W; ++wc)
#pragma unroll
      for (int t = 0; t < 4; ++t) Xs[(16 * wr + c) * ast + 16 * wc + 4 * g + t] = X[wr][wc][t];
}

// G = X^H X for X in LDS: the Gram phase's MFMA tiles with the rows of X in
// place of antennas (k-step t takes rows 4 t + g).
template <int W>
__device__ __forceinline__ void lds_gram(const float2* Xs, int ast, int c, int g,
                                         GramAcc<W>& acc) {
  BlockC32<W, 4 * W> blk;
#pragma unroll
  for (int t = 0; t < 4 * W; ++t)
#pragma unroll
    for (int w = 0; w < W; ++w) blk.h[t][w] = Xs[(4 * t + g) * ast + 16 * w + c];
  blk.template mma<true, false>(acc);
}

// A^{-1} = M^{-H} M^{-1} into Xs, its real diagonal into Dinv.  `scratch`
// needs gram_scratch_floats<W>() floats.
template <int W>
__device__ __forceinline__ void cholesky_full_inverse(const float2* As, float2* Xs, float* Dinv,
                                                      float* scratch, float2* xch, int ast,
                                                      int U, int c, int g) {
  Owned<W> X;
  cholesky_inverse<W>(As, ast, U, xch, c, g, X);
  store_owned<W>(Xs, ast, c, g, X);
  wave_lds_sync();
  GramAcc<W> acc;
  acc.clear();
  lds_gram<W>(Xs, ast, c, g, acc);
  wave_lds_sync();
  store_gram_lds<W>(acc, Xs, Dinv, scratch, ast, 0.f, c, g);
  wave_lds_sync();
}

// X_K = sum_{k<K} (-D^{-1} E)^k D^{-1} (Sec. III-F-2, A = D + E) in Horner
// form: X_1 = D^{-1}, X_{k+1} = D^{-1} (I - E X_k).  Each step is one
// NU x NU complex product on 16x16x4 MFMA: A-operand E (A with its diagonal
// zeroed) from registers, B-operand X_k from LDS; output rows
// 16 wr + 4 g + j, columns 16 wc + c.
template <int W>
__device__ __forceinline__ void neumann_series(const float2* As, float2* Xs, int ast, int K,
                                               int lane, int c, int g) {
  constexpr int NU = 16 * W;
  AOperand<W> e;                       // e.a[wr][kt] = A(16 wr + c, 4 kt + g)
  e.load(As, ast, c, g, 16 * W);
#pragma unroll
  for (int wr = 0; wr < W; ++wr)
#pragma unroll
    for (int kt = 0; kt < 4 * W; ++kt)
      if (16 * wr + c == 4 * kt + g) e.a[wr][kt] = make_float2(0.f, 0.f);
  float dinv[W][4];
#pragma unroll
  for (int wr = 0; wr < W; ++wr)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 16 * wr + 4 * g + j;
      dinv[wr][j] = 1.0f / As[i * ast + i].x;
    }
  for (int idx = lane; idx < NU * NU; idx += kWave) {
    const int i = idx / NU, k = idx % NU;
    Xs[i * ast + k] = make_float2(i == k ? 1.0f / As[i * ast + i].x : 0.f, 0.f);
  }
  wave_lds_sync();
  for (int it = 1; it < K; ++it) {
    f4 pr[W][W], pi[W][W];
#pragma unroll
    for (int wr = 0; wr < W; ++wr)
#pragma unroll
      for (int wc = 0; wc < W; ++wc) { pr[wr][wc] = zero4(); pi[wr][wc] = zero4(); }
#pragma unroll
    for (int kt = 0; kt < 4 * W; ++kt) {
      float2 xb[W];
#pragma unroll
      for (int wc = 0; wc < W; ++wc) xb[wc] = Xs[(4 * kt + g) * ast + 16 * wc + c];
#pragma unroll
      for (int wr = 0; wr < W; ++wr) {
        const float2 a = e.a[wr][kt];
#pragma unroll
        for (int wc = 0; wc < W; ++wc) {
          pr[wr][wc] = mfma4(a.x, xb[wc].x, pr[wr][wc]);
          pr[wr][wc] = mfma4(-a.y, xb[wc].y, pr[wr][wc]);
          pi[wr][wc] = mfma4(a.x, xb[wc].y, pi[wr][wc]);
          pi[wr][wc] = mfma4(a.y, xb[wc].x, pi[wr][wc]);
        }
      }
    }
    wave_lds_sync();
#pragma unroll
    for (int wr = 0; wr < W; ++wr)
#pragma unroll
      for (int wc = 0; wc < W; ++wc)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int i = 16 * wr + 4 * g + j, k = 16 * wc + c;
          const float re = (i == k ? 1.f : 0.f) - pr[wr][wc][j];
          Xs[i * ast + k] = make_float2(re * dinv[wr][j], -pi[wr][wc][j] * dinv[wr][j]);
        }
    wave_lds_sync();
  }
}

// Soft-output statistics of the linear detector W = X H^H (Sec. II-A):
// with B = X G, mu_i = B_ii, nu_i^2 = E_s sum_{j != i} |B_ij|^2 + N0 C_ii,
// C_ii = (B X^H)_ii = sum_j Re(B_ij conj(X_ij)), rho_i = mu_i^2 / nu_i^2.
// B on MFMA (A-operand X from LDS, B-operand G = A - reg I from LDS with the
// raw diagonal Gd); row sums over the 16 lanes of a DPP row.
template <int W>
__device__ __forceinline__ void linear_sinr(const float2* As, const float* Gd, const float2* Xs,
                                            int ast, float es, float n0, int c, int g,
                                            float* MUs, float* RHOs) {
  f4 br[W][W], bi[W][W];
#pragma unroll
  for (int wr = 0; wr < W; ++wr)
#pragma unroll
    for (int wc = 0; wc < W; ++wc) { br[wr][wc] = zero4(); bi[wr][wc] = zero4(); }
#pragma unroll
  for (int kt = 0; kt < 4 * W; ++kt) {
    const int k = 4 * kt + g;
    float2 xa[W], gb[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      xa[w] = Xs[(16 * w + c) * ast + k];
      const int col = 16 * w + c;
      gb[w] = k == col ? make_float2(Gd[k], 0.f) : As[k * ast + col];
    }
#pragma unroll
    for (int wr = 0; wr < W; ++wr)
#pragma unroll
      for (int wc = 0; wc < W; ++wc) {
        br[wr][wc] = mfma4(xa[wr].x, gb[wc].x, br[wr][wc]);
        br[wr][wc] = mfma4(-xa[wr].y, gb[wc].y, br[wr][wc]);
        bi[wr][wc] = mfma4(xa[wr].x, gb[wc].y, bi[wr][wc]);
        bi[wr][wc] = mfma4(xa[wr].y, gb[wc].x, bi[wr][wc]);
      }
  }
#pragma unroll
  for (int wr = 0; wr < W; ++wr) {
    float mu[4], off[4], cii[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = 16 * wr + 4 * g + j;
      mu[j] = 0.f;
      off[j] = 0.f;
      cii[j] = 0.f;
#pragma unroll
      for (int wc = 0; wc < W; ++wc) {
        const int col = 16 * wc + c;
        const float bx = br[wr][wc][j], by = bi[wr][wc][j];
        const float2 x = Xs[i * ast + col];
        const bool diag = col == i;
        mu[j] += diag ? bx : 0.f;
        off[j] += diag ? 0.f : bx * bx + by * by;
        cii[j] += bx * x.x + by * x.y;
      }
    }
    row_sum16_x4(mu);
    row_sum16_x4(off);
    row_sum16_x4(cii);
    if (c == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = 16 * wr + 4 * g + j;
        MUs[i] = mu[j];
        RHOs[i] = mu[j] * mu[j] / (es * off[j] + n0 * cii[j]);
      }
    }
  }
}

}  // namespace mimo

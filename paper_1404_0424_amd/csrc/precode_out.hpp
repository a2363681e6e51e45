// Output stage of the precoders (Sec. III-D, Algorithm 1 output): given
// the solution v of (H_d H_d^H + beta I) v = t in the CG lane layout, form
// ||q||^2 = v^H G v from one mat-vec with G, then q = H_d^H v = H_u v on
// MFMA with the optional power normalization s = q / ||q|| (Sec. II-B), each
// output tile written once, already scaled.
#pragma once

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

// A-operand rows of the output contraction: H[b][u] for u = 16 w + 4 t + g
// (k-step t covers users 16 w + 4 t .. 16 w + 4 t + 3, so k-steps past the
// last user can be skipped).  Row b0 + c of H; rows past B read zero.
template <int W>
__device__ __forceinline__ void load_h_row(InC32, const void* Hn, int B, int U, int b0, int c,
                                           int w, int g, float2 (&hv)[4]) {
  const __amdgpu_buffer_rsrc_t rh = make_rsrc(Hn, (uint32_t)B * U * 8u);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int u = 16 * w + 4 * t + g;
    hv[t] = bload2(rh, u < U ? (uint32_t)(c * U + u) * 8u : kOOB, (uint32_t)b0 * U * 8u);
  }
}
template <int W>
__device__ __forceinline__ void load_h_row(InC32P, const void* Hn, int B, int U, int b0, int c,
                                           int w, int g, float2 (&hv)[4]) {
  load_h_row<W>(InC32{}, Hn, B, U, b0, c, w, g, hv);
}
template <int W>
__device__ __forceinline__ void load_h_row(InC32X3, const void* Hn, int B, int U, int b0, int c,
                                           int w, int g, float2 (&hv)[4]) {
  load_h_row<W>(InC32{}, Hn, B, U, b0, c, w, g, hv);
}
template <int W, typename IN>
__device__ __forceinline__ void load_h_row(IN tag, const void* Hn, int B, int U, int b0, int c,
                                           int w, int g, float2 (&hv)[4]) {
  const int brow = b0 + c;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int u = 16 * w + 4 * t + g;
    hv[t] = (brow < B && u < U) ? load_h(tag, Hn, brow, u, U) : make_float2(0.f, 0.f);
  }
}

// Q[n][:, s0 .. s0+15] and qnorm from v (lane layout, ST-precision norms).
// `at` is the A^T operand of A = G + beta I, Gd the raw diagonal G_uu.  With `Qs` (wave-private LDS of
// at least 16 x 16 complex, free during the output stage) and S <= 16, each
// 16-antenna output tile, contiguous in memory, is staged there and written
// with contiguous 8-byte pieces, whole cache lines per store instruction.
// ||q_s||^2 = v_s^H G v_s for the lane layout's 16 right-hand sides into
// Ns[0..15] (V staged in Ps).  The mat-vec runs on the A^T operand with its
// diagonal entries A_uu = G_uu + beta replaced by the raw G_uu (Gd), so beta
// never enters the sum: v^H A v - beta ||v||^2 would cancel as beta grows
// (at low SNR), leaving the FP32 rounding of A v at magnitude beta |v|.
template <int W, typename ST>
__device__ __forceinline__ void qnorm2_lds(const AOperand<W>& at, const float* Gd,
                                           const float2 (&vsol)[W][4],
                                           const float2* __restrict__ Ps, float* Ns, int c,
                                           int g) {
  AOperand<W> gt = at;
#pragma unroll
  for (int wc = 0; wc < W; ++wc) {
    const float gd = Gd[16 * wc + c];
#pragma unroll
    for (int t = 0; t < 4 * W; ++t)
      if (16 * wc + c == 4 * t + g) gt.a[wc][t] = make_float2(gd, 0.f);
  }
  float2 e[W][4];
  matvec_mfma<W>(gt, Ps, c, g, e);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ST part = ST(0);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const float2 v = vsol[w][j];
      part += (ST)v.x * (ST)e[w][j].x + (ST)v.y * (ST)e[w][j].y;
    }
    const ST qq = row_sum16(part);
    if (c == 0) Ns[4 * g + j] = (float)(qq > ST(0) ? qq : ST(0));
  }
}

template <int W, typename IN, typename ST>
__device__ __forceinline__ void precode_store(const PrecodeParams& prm, int64_t n, int s0,
                                              const void* Hn, const float2 (&vsol)[W][4],
                                              const AOperand<W>& at, const float* Gd,
                                              float2* Ps, float* Ns, int c, int g,
                                              float2* Qs = nullptr) {
  const int B = prm.B, U = prm.U, S = prm.S;
    // ---- ||q||^2 = v^H G v ; V stays staged in Ps for the output contraction
    stage_vec<W>(Ps, c, g, vsol);
    wave_lds_sync();
    qnorm2_lds<W, ST>(at, Gd, vsol, Ps, Ns, c, g);
    wave_lds_sync();

    // ---- q = H_u v (Algorithm 1 output) on MFMA: rows = antennas,
    // columns = right-hand sides, k = users (k-step t of tile w takes users
    // 16 w + 4 t + g; v is zero on padding users, so k-steps past U are
    // skipped).
    const int s = s0 + c;
    const bool stage = Qs != nullptr && S <= 16;
    const float nrm2 = Ns[c];
    const float scl = prm.normalize ? (nrm2 > 0.f ? __builtin_amdgcn_rsqf(nrm2) : 0.f) : 1.0f;
    float2 vv[W][4];
#pragma unroll
    for (int w = 0; w < W; ++w)
#pragma unroll
      for (int t = 0; t < 4; ++t) vv[w][t] = Ps[(16 * w + 4 * t + g) * kPST + c];
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
          if (16 * w + 4 * t >= U) break;
          p1 = mfma4(hv[t].x, vv[w][t].x, p1);
          p2 = mfma4(hv[t].y, vv[w][t].y, p2);
          p3 = mfma4(hv[t].x + hv[t].y, vs[w][t], p3);
        }
      }
      const f4 qr = p1 - p2;
      const f4 qi = p3 - p1 - p2;
      if (stage) {
        if (s < S) {
#pragma unroll
          for (int j = 0; j < 4; ++j) Qs[(4 * g + j) * S + s] = make_float2(qr[j] * scl, qi[j] * scl);
        }
        wave_lds_sync();
        const int rows = B - b0 < 16 ? B - b0 : 16;
        const __amdgpu_buffer_rsrc_t rq =
            make_rsrc(prm.Q + ((size_t)n * B + b0) * S, (uint32_t)(rows * S) * 8u);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = 64 * r + 16 * g + c;
          const float2 q = Qs[e < 16 * S ? e : 0];
          bstore2(rq, e < rows * S ? (uint32_t)e * 8u : kOOB, q.x, q.y);
        }
        wave_lds_sync();
      } else if (s < S) {
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
}

}  // namespace mimo

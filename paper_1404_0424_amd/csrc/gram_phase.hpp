// Regularized Gram matrix and matched filter on MFMA (Algorithm 1,
// initialization: A = H^H H + reg I, b = H^H y), one wavefront per
// subcarrier.
//
// The complex products are split into real MFMA products.  With
// Hr/Hi and Yr/Yi the real and imaginary parts,
//   Re G = Hr^T Hr + Hi^T Hi,      Im G = Hr^T Hi - Hi^T Hr,
//   Re b = Hr^T Yr + Hi^T Yi,      Im b = Hr^T Yi - Hi^T Yr,
// and the contraction index k of each MFMA runs over BS antennas.  Lane
// l = 16 g + c loads user column c (Gram) / right-hand side c (matched
// filter) of the antennas of k-group g, so A- and B-operands of the Gram
// come from the same registers.
//
// Output layout (MFMA D layout): lane (c, g) holds, in element j,
//   Gram tile (wr, wc):   G[16 wr + 4 g + j][16 wc + c]
//   matched filter w:     b[user 16 w + c][rhs s0 + 4 g + j]
// which is the layout the CG phase works in (lane = user, 4 rhs per lane).
#pragma once

#include "common.hpp"

namespace mimo {

template <int W>
struct GramAcc {
  static constexpr int NT = W * (W + 1) / 2;   // upper-triangular tiles
  f4 gr[NT], gi[NT];                           // Re / Im of G tiles
  f4 dr[W], di[W];                             // Re / Im of b tiles
  __device__ void clear() {
#pragma unroll
    for (int t = 0; t < NT; ++t) { gr[t] = zero4(); gi[t] = zero4(); }
#pragma unroll
    for (int w = 0; w < W; ++w) { dr[w] = zero4(); di[w] = zero4(); }
  }
};

__host__ __device__ constexpr int tile_index(int wr, int wc, int W) {
  return wr * W - (wr * (wr - 1)) / 2 + (wc - wr);
}

// ----------------------------------------------------------------- complex64
// H: [B][U] complex64 of one subcarrier, Y: [B][S].  Each MFMA step covers 4
// antennas (k-group g -> antenna 4 t + g), so the 16 lanes of a k-group read
// one contiguous antenna row of H and of Y.
template <int W, bool DO_GRAM, bool DO_MF>
__device__ __forceinline__ void gram_mf_c32(const float2* __restrict__ Hn,
                                            const float2* __restrict__ Yn, int B,
                                            int U, int S, int s0, int c, int g,
                                            GramAcc<W>& acc) {
  constexpr int UNR = 8;
  const int s = s0 + c;
  for (int b0 = 0; b0 < B; b0 += 4 * UNR) {
    float2 h[UNR][W];
    float2 y[UNR];
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      const int b = b0 + 4 * t + g;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const int u = 16 * w + c;
        h[t][w] = (b < B && u < U) ? Hn[(size_t)b * U + u] : make_float2(0.f, 0.f);
      }
      if (DO_MF) y[t] = (b < B && s < S) ? Yn[(size_t)b * S + s] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      if (DO_GRAM) {
#pragma unroll
        for (int wr = 0; wr < W; ++wr)
#pragma unroll
          for (int wc = wr; wc < W; ++wc) {
            const int ti = tile_index(wr, wc, W);
            acc.gr[ti] = mfma4(h[t][wr].x, h[t][wc].x, acc.gr[ti]);
            acc.gr[ti] = mfma4(h[t][wr].y, h[t][wc].y, acc.gr[ti]);
            acc.gi[ti] = mfma4(h[t][wr].x, h[t][wc].y, acc.gi[ti]);
            acc.gi[ti] = mfma4(-h[t][wr].y, h[t][wc].x, acc.gi[ti]);
          }
      }
      if (DO_MF) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          acc.dr[w] = mfma4(y[t].x, h[t][w].x, acc.dr[w]);
          acc.dr[w] = mfma4(y[t].y, h[t][w].y, acc.dr[w]);
          acc.di[w] = mfma4(y[t].y, h[t][w].x, acc.di[w]);
          acc.di[w] = mfma4(-y[t].x, h[t][w].y, acc.di[w]);
        }
      }
    }
  }
}

// ----------------------------------------------------------------- 16-bit
// Blocked storage [B/8][2][C][8] (part 0 = Re, 1 = Im) of one subcarrier:
// the 8 antennas of a block are contiguous for each column, so one 16-byte
// load gives a lane the 8 k-values of a 16x16x32 MFMA operand.  Each MFMA
// step covers 4 blocks (32 antennas), k-group g taking block 4 t + g.
template <typename V8>
__device__ __forceinline__ V8 neg8(V8 x) {
  uint4 u = __builtin_bit_cast(uint4, x);
  u.x ^= 0x80008000u; u.y ^= 0x80008000u; u.z ^= 0x80008000u; u.w ^= 0x80008000u;
  return __builtin_bit_cast(V8, u);
}

template <int W, bool DO_GRAM, bool DO_MF, typename V8>
__device__ __forceinline__ void gram_mf_16(const uint16_t* __restrict__ Hn,
                                           const uint16_t* __restrict__ Yn, int B,
                                           int U, int S, int s0, int c, int g,
                                           GramAcc<W>& acc) {
  constexpr int UNR = 2;
  const int nblk = B >> 3;
  const int s = s0 + c;
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  for (int k0 = 0; k0 < nblk; k0 += 4 * UNR) {
    V8 hr[UNR][W], hi[UNR][W], yr[UNR], yi[UNR];
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      const int kb = k0 + 4 * t + g;
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const int u = 16 * w + c;
        const bool ok = kb < nblk && u < U;
        const uint16_t* p = Hn + ((size_t)(2 * kb) * U + u) * 8;
        hr[t][w] = __builtin_bit_cast(V8, ok ? *(const uint4*)p : z);
        hi[t][w] = __builtin_bit_cast(V8, ok ? *(const uint4*)(p + (size_t)U * 8) : z);
      }
      if (DO_MF) {
        const bool ok = kb < nblk && s < S;
        const uint16_t* p = Yn + ((size_t)(2 * kb) * S + s) * 8;
        yr[t] = __builtin_bit_cast(V8, ok ? *(const uint4*)p : z);
        yi[t] = __builtin_bit_cast(V8, ok ? *(const uint4*)(p + (size_t)S * 8) : z);
      }
    }
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      if (DO_GRAM) {
#pragma unroll
        for (int wr = 0; wr < W; ++wr)
#pragma unroll
          for (int wc = wr; wc < W; ++wc) {
            const int ti = tile_index(wr, wc, W);
            acc.gr[ti] = mfma32(hr[t][wr], hr[t][wc], acc.gr[ti]);
            acc.gr[ti] = mfma32(hi[t][wr], hi[t][wc], acc.gr[ti]);
            acc.gi[ti] = mfma32(hr[t][wr], hi[t][wc], acc.gi[ti]);
            acc.gi[ti] = mfma32(neg8(hi[t][wr]), hr[t][wc], acc.gi[ti]);
          }
      }
      if (DO_MF) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          acc.dr[w] = mfma32(yr[t], hr[t][w], acc.dr[w]);
          acc.dr[w] = mfma32(yi[t], hi[t][w], acc.dr[w]);
          acc.di[w] = mfma32(yi[t], hr[t][w], acc.di[w]);
          acc.di[w] = mfma32(neg8(yr[t]), hi[t][w], acc.di[w]);
        }
      }
    }
  }
}

// Input storage tags
struct InC32 {};
struct InF16 {};
struct InBF16 {};

template <int W, bool DO_GRAM, bool DO_MF>
__device__ __forceinline__ void gram_mf(InC32, const void* Hn, const void* Yn, int B, int U,
                                        int S, int s0, int c, int g, GramAcc<W>& acc) {
  gram_mf_c32<W, DO_GRAM, DO_MF>((const float2*)Hn, (const float2*)Yn, B, U, S, s0, c, g, acc);
}
template <int W, bool DO_GRAM, bool DO_MF>
__device__ __forceinline__ void gram_mf(InF16, const void* Hn, const void* Yn, int B, int U,
                                        int S, int s0, int c, int g, GramAcc<W>& acc) {
  gram_mf_16<W, DO_GRAM, DO_MF, h8>((const uint16_t*)Hn, (const uint16_t*)Yn, B, U, S, s0, c,
                                    g, acc);
}
template <int W, bool DO_GRAM, bool DO_MF>
__device__ __forceinline__ void gram_mf(InBF16, const void* Hn, const void* Yn, int B, int U,
                                        int S, int s0, int c, int g, GramAcc<W>& acc) {
  gram_mf_16<W, DO_GRAM, DO_MF, bf8>((const uint16_t*)Hn, (const uint16_t*)Yn, B, U, S, s0, c,
                                     g, acc);
}

// Elements per subcarrier of an [R][C] complex array in each storage type,
// counted in units of the pointer type used above (float2 or uint16_t).
template <typename IN>
__host__ __device__ constexpr size_t elems_per(IN, size_t R, size_t C);
template <>
__host__ __device__ constexpr size_t elems_per(InC32, size_t R, size_t C) { return R * C; }
template <>
__host__ __device__ constexpr size_t elems_per(InF16, size_t R, size_t C) { return 2 * R * C; }
template <>
__host__ __device__ constexpr size_t elems_per(InBF16, size_t R, size_t C) { return 2 * R * C; }

template <typename IN>
__device__ __forceinline__ const void* offset_sc(IN tag, const void* base, int64_t n, int R, int C);
template <>
__device__ __forceinline__ const void* offset_sc(InC32, const void* base, int64_t n, int R, int C) {
  return (const float2*)base + (size_t)n * R * C;
}
template <>
__device__ __forceinline__ const void* offset_sc(InF16, const void* base, int64_t n, int R, int C) {
  return (const uint16_t*)base + (size_t)n * R * C * 2;
}
template <>
__device__ __forceinline__ const void* offset_sc(InBF16, const void* base, int64_t n, int R, int C) {
  return (const uint16_t*)base + (size_t)n * R * C * 2;
}

// Write the upper triangle (and its conjugate mirror) of the Gram tiles to
// the wave's LDS copy of A with reg added to the real diagonal; the raw
// diagonal G_ii goes to Gd.  Padding users (>= U) have zero columns, so
// their rows of A are reg * e_u and decouple from the real system.
template <int W>
__device__ __forceinline__ void store_gram_lds(const GramAcc<W>& acc, float2* As, float* Gd,
                                               int ast, float reg, int c, int g) {
#pragma unroll
  for (int wr = 0; wr < W; ++wr)
#pragma unroll
    for (int wc = wr; wc < W; ++wc) {
      const int ti = tile_index(wr, wc, W);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = 16 * wr + 4 * g + j;
        const int cc = 16 * wc + c;
        const float re = acc.gr[ti][j], im = acc.gi[ti][j];
        if (r < cc) {
          As[r * ast + cc] = make_float2(re, im);
          As[cc * ast + r] = make_float2(re, -im);
        } else if (r == cc) {
          As[r * ast + r] = make_float2(re + reg, 0.f);
          Gd[r] = re;
        }
      }
    }
}

}  // namespace mimo

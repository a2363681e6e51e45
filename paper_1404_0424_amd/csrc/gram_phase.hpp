// Regularized Gram matrix and matched filter on MFMA (Algorithm 1,
// initialization: A = H^H H + reg I, b = H^H y), one wavefront per
// subcarrier.
//
// With Hr/Hi and Yr/Yi the real and imaginary parts, over BS antennas k:
//   Re G = Hr^T Hr + Hi^T Hi,          Im G = M - M^T with M = Hr^T Hi
//   Re b = P1 + P2,  Im b = P3 - P1 + P2  with P1 = Yr^T Hr, P2 = Yi^T Hi,
//                                        P3 = (Yr + Yi)^T (Hr - Hi)
// (three real products per complex product; diagonal Gram tiles need only
// M, whose transpose is taken through LDS).  The 16-bit path keeps four
// products for b, because Yr + Yi would round in 16-bit storage.
//
// Lane l = 16 g + c loads user column c (Gram) / right-hand side c (matched
// filter) of the antennas of k-group g, so A- and B-operands of the Gram come
// from the same registers.  Loads are buffer loads whose descriptor covers
// exactly one subcarrier's array: rows past B and masked lanes (users >= U,
// rhs >= S) read zero from the hardware range check, with no branches.
//
// Output layout (MFMA D layout): lane (c, g) holds, in element j,
//   Gram tile (wr, wc):   G[16 wr + 4 g + j][16 wc + c]
//   matched filter w:     b[user 16 w + c][rhs s0 + 4 g + j]
// which is the layout the CG phase works in (lane = user, 4 rhs per lane).
//
// Packed form (storage tag InC32P: complex64 with U <= 8): the users fill
// only half of a 16-wide tile, so lanes c and c + 8 both load user c & 7 and
// give the MFMA its real part (c < 8) or imaginary part (c >= 8).  One
// product of that operand with itself is the whole real Gram,
//   C = [Hr Hi]^T [Hr Hi],  Re G = C[0:8, 0:8] + C[8:16, 8:16],
//                           Im G = C[0:8, 8:16] - C[8:16, 0:8],
// and two products with Yr and Yi give the matched filter (C1 = Yr^T [Hr Hi],
// C2 = Yi^T [Hr Hi]):  Re b^T = C1[:, 0:8] + C2[:, 8:16],
//                      Im b^T = C2[:, 0:8] - C1[:, 8:16],
// 3 MFMAs per k-step instead of 6.  finish_mf and store_gram fold the halves
// back into the standard layout.
#pragma once

#include "common.hpp"

namespace mimo {

constexpr uint32_t kOOB = 0x80000000u;   // offset outside every descriptor's range

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           0x00020000);
}
// Cache policy of the buffer loads and stores below.  Where a kernel reads
// each byte of H, Y (and writes each output byte) once per launch, the
// non-temporal policy (the nt bit, value 2 of the builtins' aux operand on
// gfx950) marks the lines as streaming so they stop displacing one another in
// L2 and the Infinity Cache; it changes no value (detection measured 147-149 us
// -> 136-138 us per launch on the 128x16 batch of 19,200 subcarriers).  Kernels
// that read H a second time (the streaming precoders, the inverse-based and
// CGLS methods) want those lines kept: their translation units define
// MIMO_CACHE_STREAMING 0 before including this header and get the default
// policy (each unit is compiled to its own device code object); a kernel there
// that reads H once passes the policy to the block loads explicitly.
#ifndef MIMO_CACHE_STREAMING
#define MIMO_CACHE_STREAMING 1
#endif
constexpr int kStreamCPol = MIMO_CACHE_STREAMING ? 2 : 0;

template <int CPOL = kStreamCPol>
__device__ __forceinline__ float2 bload2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, CPOL));
}
template <int CPOL = kStreamCPol>
__device__ __forceinline__ uint4 bload4(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, CPOL));
}

// Buffer stores: an offset outside the descriptor's range (kOOB, or any
// offset of a zero-size descriptor) is dropped by the hardware, so masked
// stores need no branch and every lane issues the same instructions.
typedef unsigned int u2 __attribute__((ext_vector_type(2)));
typedef unsigned int u3 __attribute__((ext_vector_type(3)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
// (CPOL 0, the default policy, suits outputs written in scattered 4- or 8-byte
// pieces: there L2 merges the pieces into whole lines before they leave.)
template <int CPOL = kStreamCPol>
__device__ __forceinline__ void bstore1(__amdgpu_buffer_rsrc_t r, uint32_t voff, float a) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, a), r, voff, 0, CPOL);
}
template <int CPOL = kStreamCPol>
__device__ __forceinline__ void bstore2(__amdgpu_buffer_rsrc_t r, uint32_t voff, float a,
                                        float b) {
  const u2 v = {__builtin_bit_cast(unsigned int, a), __builtin_bit_cast(unsigned int, b)};
  __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, 0, CPOL);
}
// ... with a wave-uniform part of the offset in soffset (range-checked too)
__device__ __forceinline__ void bstore2s(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                         float a, float b) {
  const u2 v = {__builtin_bit_cast(unsigned int, a), __builtin_bit_cast(unsigned int, b)};
  __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, kStreamCPol);
}
__device__ __forceinline__ void bstore3(__amdgpu_buffer_rsrc_t r, uint32_t voff, float a,
                                        float b, float c) {
  const u3 v = {__builtin_bit_cast(unsigned int, a), __builtin_bit_cast(unsigned int, b),
                __builtin_bit_cast(unsigned int, c)};
  __builtin_amdgcn_raw_buffer_store_b96(v, r, voff, 0, kStreamCPol);
}
__device__ __forceinline__ void bstore4(__amdgpu_buffer_rsrc_t r, uint32_t voff, float a,
                                        float b, float c, float d) {
  const u4 v = {__builtin_bit_cast(unsigned int, a), __builtin_bit_cast(unsigned int, b),
                __builtin_bit_cast(unsigned int, c), __builtin_bit_cast(unsigned int, d)};
  __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, 0, kStreamCPol);
}

template <int W>
struct GramAcc {
  static constexpr int NT = W * (W + 1) / 2;   // upper-triangular tiles
  f4 gr[NT];          // Re G
  f4 gi[NT];          // diagonal tiles: M = Hr^T Hi; off-diagonal tiles: Im G
  f4 dr[W], di[W];    // complex64: P1, P2; 16-bit: Re b, Im b
  f4 p3[W];           // complex64: P3
  __device__ void clear() {
#pragma unroll
    for (int t = 0; t < NT; ++t) { gr[t] = zero4(); gi[t] = zero4(); }
#pragma unroll
    for (int w = 0; w < W; ++w) { dr[w] = zero4(); di[w] = zero4(); p3[w] = zero4(); }
  }
};

__host__ __device__ constexpr int tile_index(int wr, int wc, int W) {
  return wr * W - (wr * (wr - 1)) / 2 + (wc - wr);
}

// Input storage tags
struct InC32 {};
struct InC32P {};   // complex64, U <= 8, packed form (one wavefront per subcarrier)
struct InF16 {};
struct InBF16 {};

// ----------------------------------------------------------------- complex64
// H: [B][U] complex64 of one subcarrier, Y: [B][S].  Each MFMA step covers 4
// antennas (k-group g -> antenna 4 t + g), so the 16 lanes of a k-group read
// one contiguous antenna row of H and of Y.  A block is UNR steps.
template <int W>
struct SubC32 {                       // per-subcarrier buffer descriptors and lane offsets
  __amdgpu_buffer_rsrc_t rh, ry;
  uint32_t oh[W], oy;
  int U, S;
  __device__ void init(const void* Hn, const void* Yn, int B, int U_, int S_, int s0, int c,
                       int g) {
    U = U_;
    S = S_;
    rh = make_rsrc(Hn, (uint32_t)B * U * 8u);
    ry = make_rsrc(Yn ? Yn : Hn, Yn ? (uint32_t)B * S * 8u : 0u);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int u = 16 * w + c;
      oh[w] = u < U ? (uint32_t)(g * U + u) * 8u : kOOB;
    }
    const int s = s0 + c;
    oy = s < S ? (uint32_t)(g * S + s) * 8u : kOOB;
  }
  // zero-size descriptors: every load reads zero without touching memory
  __device__ void disable() {
    rh = make_rsrc(nullptr, 0u);
    ry = make_rsrc(nullptr, 0u);
  }
};

template <int W, int UNR = 8>
struct BlockC32 {
  static constexpr int ANT = 4 * UNR;  // antennas per block
  float2 h[UNR][W];
  float2 y[UNR];
  template <bool DO_MF, int CPOL = kStreamCPol>
  __device__ __forceinline__ void load(const SubC32<W>& sb, int b0) {
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      const int b = b0 + 4 * t;
#pragma unroll
      for (int w = 0; w < W; ++w) h[t][w] = bload2<CPOL>(sb.rh, sb.oh[w], (uint32_t)b * sb.U * 8u);
      if (DO_MF) y[t] = bload2<CPOL>(sb.ry, sb.oy, (uint32_t)b * sb.S * 8u);
    }
  }
  template <bool DO_GRAM, bool DO_MF>
  __device__ __forceinline__ void mma(GramAcc<W>& acc) const {
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
            if (wr != wc) acc.gi[ti] = mfma4(-h[t][wr].y, h[t][wc].x, acc.gi[ti]);
          }
      }
      if (DO_MF) {
        const float ys = y[t].x + y[t].y;
#pragma unroll
        for (int w = 0; w < W; ++w) {
          acc.dr[w] = mfma4(y[t].x, h[t][w].x, acc.dr[w]);                 // P1
          acc.di[w] = mfma4(y[t].y, h[t][w].y, acc.di[w]);                 // P2
          acc.p3[w] = mfma4(ys, h[t][w].x - h[t][w].y, acc.p3[w]);         // P3
        }
      }
    }
  }
};

// Re b = P1 + P2, Im b = P3 - P1 + P2 (complex64 matched filter)
template <int W>
__device__ __forceinline__ void finish_mf(InC32, GramAcc<W>& acc) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const f4 p1 = acc.dr[w], p2 = acc.di[w];
    acc.dr[w] = p1 + p2;
    acc.di[w] = acc.p3[w] - p1 + p2;
  }
}

// ------------------------------------------------------ complex64, packed
struct SubC32P : SubC32<1> {
  __device__ void init(const void* Hn, const void* Yn, int B, int U_, int S_, int s0, int c,
                       int g) {
    SubC32<1>::init(Hn, Yn, B, U_, S_, s0, c, g);
    const int u = c & 7;
    oh[0] = u < U ? (uint32_t)(g * U + u) * 8u : kOOB;
  }
};

template <int UNR>
struct BlockC32P : BlockC32<1, UNR> {
  template <bool DO_GRAM, bool DO_MF>
  __device__ __forceinline__ void mma(GramAcc<1>& acc) const {
    const bool re = (__lane_id() & 8) == 0;
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      const float2 v = this->h[t][0];       // select by value: a select between member
      const float a = re ? v.x : v.y;       // addresses would keep the block in scratch
      if (DO_GRAM) acc.gr[0] = mfma4(a, a, acc.gr[0]);
      if (DO_MF) {
        acc.dr[0] = mfma4(this->y[t].x, a, acc.dr[0]);
        acc.di[0] = mfma4(this->y[t].y, a, acc.di[0]);
      }
    }
  }
};

// Re b = C1[s][u] + C2[s][u + 8], Im b = C2[s][u] - C1[s][u + 8] on the lanes
// of users u < 8 (partner lane u + 8), zero on the others.
__device__ __forceinline__ void finish_mf(InC32P, GramAcc<1>& acc) {
  const bool lo = (__lane_id() & 8) == 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float c1 = acc.dr[0][j], c2 = acc.di[0][j];
    const float c1h = __shfl_xor(c1, 8, 64), c2h = __shfl_xor(c2, 8, 64);
    acc.dr[0][j] = lo ? c1 + c2h : 0.f;
    acc.di[0][j] = lo ? c2 - c1h : 0.f;
  }
}

// ------------------------------------------- complex64, bf16-split products
// Storage tag InC32X3: complex64 H and Y, with the Gram and matched filter
// formed on the 16-bit matrix cores from an exact split of each FP32 value
// into three bf16 parts (round to nearest even at each level):
//   x = x0 + x1 + x2 + e,  |x1| <= 2^-8 |x|, |x2| <= 2^-16 |x|, |e| <= 2^-24 |x|,
// and the six leading partial products x_i y_j (i + j <= 2) of every
// product x y, each exact in FP32 and accumulated in FP32 by the MFMA.  The
// dropped terms are below 2^-23 |x y| in all, so the result has the accuracy
// of FP32 products with FP32 accumulation (a Gram error of 4.7e-7 against
// 2.7e-7 on the 128 x 16 workload).  On gfx950 FP32 MFMAs and VALU
// instructions share one issue pipe (a wave issuing FP32 MFMAs and one issuing
// VALU FMAs on the same SIMD take the sum of their times), while 16-bit MFMAs
// run beside VALU work; the split moves the Gram and matched filter off the
// shared pipe at the cost of ~110 VALU instructions per 16 antennas.
//
// A 16x16x32 MFMA takes 16 antennas: lane (c, g) holds H[b0 + 4 t + g][c],
// t = 0..3 (the same loads as the FP32 form), as the k-slice
// [re(h_0), im(h_0), .., re(h_3), im(h_3)] of user c; the matched filter's
// operand is built from Y the same way.  With X that stacked operand and
// R = (-im, re) per antenna (X rotated by i):
//   Re G = X^T X,  -Im G = X^T R,  Re b = Y^T X,  Im b = Y^T R
// (rows x columns of the MFMA D layout: Gram rows = users, MF rows = rhs),
// six products each; the Gram's imaginary part is accumulated negated.
struct InC32X3 {};

// bf16 parts of the complex values v[0..3]: p_i = part i of the (re, im)
// pairs and, with ROT, r_i = part i of the (-im, re) pairs (the same
// roundings, rotated).  Each level converts a pair with one packed
// conversion (round to nearest even) and subtracts the widened parts, which
// is exact.
typedef float fl2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf8 pack4(bf2 a, bf2 b, bf2 c, bf2 d) {
  return bf8{a[0], a[1], b[0], b[1], c[0], c[1], d[0], d[1]};
}
template <bool ROT>
__device__ __forceinline__ void split3(const float2 (&v)[4], bf8 (&p)[3], bf8 (&rt)[3]) {
  bf2 pp[3][4], rr[3][4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    fl2 r = fl2{v[e].x, v[e].y};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const bf2 q = __builtin_convertvector(r, bf2);
      pp[i][e] = q;
      if (ROT) rr[i][e] = __builtin_convertvector(fl2{-r[1], r[0]}, bf2);
      if (i < 2) r = r - __builtin_convertvector(q, fl2);
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    p[i] = pack4(pp[i][0], pp[i][1], pp[i][2], pp[i][3]);
    if (ROT) rt[i] = pack4(rr[i][0], rr[i][1], rr[i][2], rr[i][3]);
  }
}
// c += sum over i + j <= 2 of a_i^T b_j (smallest terms first)
__device__ __forceinline__ f4 mfma_x3(const bf8 (&a)[3], const bf8 (&b)[3], f4 c) {
  c = mfma32(a[2], b[0], c);
  c = mfma32(a[1], b[1], c);
  c = mfma32(a[0], b[2], c);
  c = mfma32(a[1], b[0], c);
  c = mfma32(a[0], b[1], c);
  return mfma32(a[0], b[0], c);
}

template <int W, int NG>
struct BlockC32X3 {
  static constexpr int ANT = 16 * NG;  // antennas per block
  float2 h[4 * NG][W];
  float2 y[4 * NG];
  template <bool DO_MF, int CPOL = kStreamCPol>
  __device__ __forceinline__ void load(const SubC32<W>& sb, int b0) {
#pragma unroll
    for (int t = 0; t < 4 * NG; ++t) {
      const int b = b0 + 4 * t;
#pragma unroll
      for (int w = 0; w < W; ++w) h[t][w] = bload2<CPOL>(sb.rh, sb.oh[w], (uint32_t)b * sb.U * 8u);
      if (DO_MF) y[t] = bload2<CPOL>(sb.ry, sb.oy, (uint32_t)b * sb.S * 8u);
    }
  }
  template <bool DO_GRAM, bool DO_MF>
  __device__ __forceinline__ void mma(GramAcc<W>& acc) const {
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      bf8 xp[W][3], xr[W][3];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        const float2 v[4] = {h[4 * q][w], h[4 * q + 1][w], h[4 * q + 2][w], h[4 * q + 3][w]};
        split3<true>(v, xp[w], xr[w]);
      }
      if (DO_GRAM) {
#pragma unroll
        for (int wr = 0; wr < W; ++wr)
#pragma unroll
          for (int wc = wr; wc < W; ++wc) {
            const int ti = tile_index(wr, wc, W);
            acc.gr[ti] = mfma_x3(xp[wr], xp[wc], acc.gr[ti]);
            acc.gi[ti] = mfma_x3(xp[wr], xr[wc], acc.gi[ti]);     // -Im G
          }
      }
      if (DO_MF) {
        bf8 yp[3], unused[3];
        const float2 v[4] = {y[4 * q], y[4 * q + 1], y[4 * q + 2], y[4 * q + 3]};
        split3<false>(v, yp, unused);
#pragma unroll
        for (int w = 0; w < W; ++w) {
          acc.dr[w] = mfma_x3(yp, xp[w], acc.dr[w]);
          acc.di[w] = mfma_x3(yp, xr[w], acc.di[w]);
        }
      }
    }
  }
};

// Re b and Im b are accumulated directly.
template <int W>
__device__ __forceinline__ void finish_mf(InC32X3, GramAcc<W>&) {}

// ----------------------------------------------------------------- 16-bit
// Blocked storage [B/8][2][C][8] (part 0 = Re, 1 = Im) of one subcarrier:
// the 8 antennas of a block are contiguous for each column, so one 16-byte
// load gives a lane the 8 k-values of a 16x16x32 MFMA operand.  Each MFMA
// step covers 4 blocks of 8 (32 antennas), k-group g taking block 4 t + g.
template <typename V8>
__device__ __forceinline__ V8 neg8(V8 x) {
  uint4 u = __builtin_bit_cast(uint4, x);
  u.x ^= 0x80008000u; u.y ^= 0x80008000u; u.z ^= 0x80008000u; u.w ^= 0x80008000u;
  return __builtin_bit_cast(V8, u);
}

template <int W>
struct Sub16 {
  __amdgpu_buffer_rsrc_t rh, ry;
  uint32_t oh[W], oy;
  int U, S;
  __device__ void init(const void* Hn, const void* Yn, int B, int U_, int S_, int s0, int c,
                       int g) {
    U = U_;
    S = S_;
    rh = make_rsrc(Hn, (uint32_t)B * U * 4u);
    ry = make_rsrc(Yn ? Yn : Hn, Yn ? (uint32_t)B * S * 4u : 0u);
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int u = 16 * w + c;
      oh[w] = u < U ? (uint32_t)(2 * g * U + u) * 16u : kOOB;      // block g, part 0
    }
    const int s = s0 + c;
    oy = s < S ? (uint32_t)(2 * g * S + s) * 16u : kOOB;
  }
  __device__ void disable() {
    rh = make_rsrc(nullptr, 0u);
    ry = make_rsrc(nullptr, 0u);
  }
};

template <int W, typename V8, int UNR = 2>
struct Block16 {
  static constexpr int ANT = 32 * UNR;
  V8 hr[UNR][W], hi[UNR][W], yr[UNR], yi[UNR];
  template <bool DO_MF, int CPOL = kStreamCPol>
  __device__ __forceinline__ void load(const Sub16<W>& sb, int b0) {
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      const uint32_t kb = (uint32_t)((b0 >> 3) + 4 * t);     // first 8-antenna block of the step
#pragma unroll
      for (int w = 0; w < W; ++w) {
        hr[t][w] = __builtin_bit_cast(V8, bload4<CPOL>(sb.rh, sb.oh[w], kb * 2u * sb.U * 16u));
        hi[t][w] = __builtin_bit_cast(V8, bload4<CPOL>(sb.rh, sb.oh[w], (kb * 2u + 1u) * sb.U * 16u));
      }
      if (DO_MF) {
        yr[t] = __builtin_bit_cast(V8, bload4<CPOL>(sb.ry, sb.oy, kb * 2u * sb.S * 16u));
        yi[t] = __builtin_bit_cast(V8, bload4<CPOL>(sb.ry, sb.oy, (kb * 2u + 1u) * sb.S * 16u));
      }
    }
  }
  template <bool DO_GRAM, bool DO_MF>
  __device__ __forceinline__ void mma(GramAcc<W>& acc) const {
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
            if (wr != wc) acc.gi[ti] = mfma32(neg8(hi[t][wr]), hr[t][wc], acc.gi[ti]);
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
};

template <int W>
__device__ __forceinline__ void finish_mf(InF16, GramAcc<W>&) {}
template <int W>
__device__ __forceinline__ void finish_mf(InBF16, GramAcc<W>&) {}

// Storage traits: per-subcarrier descriptor and block types.
template <typename IN, int W>
struct Storage;
template <int W>
struct Storage<InC32, W> {
  using Sub = SubC32<W>;
  using Block = BlockC32<W, W == 1 ? 8 : 4>;
  using SmallBlock = BlockC32<W, W == 1 ? 4 : 2>;
};
template <int W>
struct Storage<InF16, W> {
  using Sub = Sub16<W>;
  using Block = Block16<W, h8, W == 1 ? 2 : 1>;
  using SmallBlock = Block16<W, h8, 1>;
};
template <>
struct Storage<InC32P, 1> {
  using Sub = SubC32P;
  using Block = BlockC32P<8>;
  using SmallBlock = BlockC32P<4>;
};
template <int W>
struct Storage<InC32X3, W> {
  using Sub = SubC32<W>;
  using Block = BlockC32X3<W, 2>;
  using SmallBlock = BlockC32X3<W, 1>;
};
template <int W>
struct Storage<InBF16, W> {
  using Sub = Sub16<W>;
  using Block = Block16<W, bf8, W == 1 ? 2 : 1>;
  using SmallBlock = Block16<W, bf8, 1>;
};

// Whole Gram / matched filter of one subcarrier without cross-subcarrier
// prefetch (used by the generic and batched kernels): half-size blocks in
// two register buffers, the next block's loads in flight while the current
// block's MFMAs run.  The k-steps are accumulated in the same order as a
// single-buffer walk, so the values are the same.
template <int W, bool DO_GRAM, bool DO_MF, typename IN>
__device__ __forceinline__ void gram_mf(IN tag, const void* Hn, const void* Yn, int B, int U,
                                        int S, int s0, int c, int g, GramAcc<W>& acc) {
  typename Storage<IN, W>::Sub sb;
  sb.init(Hn, DO_MF ? Yn : nullptr, B, U, S, s0, c, g);
  using Blk = typename Storage<IN, W>::SmallBlock;
  Blk cur, nxt;
  cur.template load<DO_MF>(sb, 0);
  for (int b0 = 0; b0 < B; b0 += 2 * Blk::ANT) {
    if (b0 + Blk::ANT < B) nxt.template load<DO_MF>(sb, b0 + Blk::ANT);
    cur.template mma<DO_GRAM, DO_MF>(acc);
    if (b0 + Blk::ANT >= B) break;
    if (b0 + 2 * Blk::ANT < B) cur.template load<DO_MF>(sb, b0 + 2 * Blk::ANT);
    nxt.template mma<DO_GRAM, DO_MF>(acc);
  }
  if (DO_MF) finish_mf(tag, acc);
}

template <typename IN>
__device__ __forceinline__ const void* offset_sc(IN tag, const void* base, int64_t n, int R, int C);
template <>
__device__ __forceinline__ const void* offset_sc(InC32, const void* base, int64_t n, int R, int C) {
  return (const float2*)base + (size_t)n * R * C;
}
template <>
__device__ __forceinline__ const void* offset_sc(InC32P, const void* base, int64_t n, int R, int C) {
  return (const float2*)base + (size_t)n * R * C;
}
template <>
__device__ __forceinline__ const void* offset_sc(InC32X3, const void* base, int64_t n, int R, int C) {
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

// Bytes of LDS scratch store_gram_lds needs (M tiles for the transpose).
template <int W>
__host__ __device__ constexpr int gram_scratch_floats() { return W * 16 * 17; }

// Write the upper triangle (and its conjugate mirror) of the Gram tiles to
// the wave's LDS copy of A with reg added to the real diagonal; the raw
// diagonal G_ii goes to Gd.  Diagonal tiles first park M in `scratch` so
// that Im G = M - M^T can be formed.  Padding users (>= U) have zero
// columns, so their rows of A are reg * e_u and decouple from the system.
template <int W>
__device__ __forceinline__ void store_gram_lds(const GramAcc<W>& acc, float2* As, float* Gd,
                                               float* scratch, int ast, float reg, int c, int g) {
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int ti = tile_index(w, w, W);
#pragma unroll
    for (int j = 0; j < 4; ++j) scratch[w * 272 + (4 * g + j) * 17 + c] = acc.gi[ti][j];
  }
  wave_lds_sync();
#pragma unroll
  for (int wr = 0; wr < W; ++wr)
#pragma unroll
    for (int wc = wr; wc < W; ++wc) {
      const int ti = tile_index(wr, wc, W);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int rl = 4 * g + j;
        const int r = 16 * wr + rl;
        const int cc = 16 * wc + c;
        const float re = acc.gr[ti][j];
        const float im = (wr == wc) ? acc.gi[ti][j] - scratch[wr * 272 + c * 17 + rl]
                                    : acc.gi[ti][j];
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

// A = G + reg I from a cached Gram matrix Gn (complex64 [U][U], Hermitian
// with a real diagonal and an exactly conjugate lower triangle, as
// mimo_gram_mf writes it with reg = 0) into the wave's LDS copy, entry for
// entry the values store_gram_lds writes for a Gram formed from the same H:
// padding users (>= U) get zero rows and columns (an imaginary -0 below the
// diagonal, where the mirror negates a zero) and reg on the diagonal; Gd
// receives G_ii.
template <int W>
__device__ __forceinline__ void load_cached_gram(const float2* __restrict__ Gn, int U, float reg,
                                                 float2* As, float* Gd, int ast, int lane) {
  constexpr int NU = 16 * W;
  for (int idx = lane; idx < NU * NU; idx += kWave) {
    const int r = idx / NU, col = idx % NU;
    float2 v = (r < U && col < U) ? Gn[r * U + col] : make_float2(0.f, r > col ? -0.f : 0.f);
    if (r == col) {
      Gd[r] = v.x;
      v = make_float2(v.x + reg, 0.f);
    }
    As[r * ast + col] = v;
  }
}

// The split form accumulates -Im G on every tile (no M - M^T step); the
// upper triangle and a real diagonal are written as for the others.
template <int W>
__device__ __forceinline__ void store_gram(InC32X3, const GramAcc<W>& acc, float2* As, float* Gd,
                                           float*, int ast, float reg, int c, int g) {
#pragma unroll
  for (int wr = 0; wr < W; ++wr)
#pragma unroll
    for (int wc = wr; wc < W; ++wc) {
      const int ti = tile_index(wr, wc, W);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = 16 * wr + 4 * g + j;
        const int cc = 16 * wc + c;
        const float re = acc.gr[ti][j], im = -acc.gi[ti][j];
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

// store_gram_lds for any storage form: the packed form first folds
// C = [Hr Hi]^T [Hr Hi] into Re G and M (through `scratch`), then writes A
// as store_gram_lds does.
template <int W, typename IN>
__device__ __forceinline__ void store_gram(IN, const GramAcc<W>& acc, float2* As, float* Gd,
                                           float* scratch, int ast, float reg, int c, int g) {
  store_gram_lds<W>(acc, As, Gd, scratch, ast, reg, c, g);
}
__device__ __forceinline__ void store_gram(InC32P, const GramAcc<1>& acc, float2* As, float* Gd,
                                           float* scratch, int ast, float reg, int c, int g) {
#pragma unroll
  for (int j = 0; j < 4; ++j) scratch[(4 * g + j) * 17 + c] = acc.gr[0][j];
  wave_lds_sync();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r = 4 * g + j;
    float re = 0.f, im = 0.f;                         // users >= 8 are padding
    if (r < 8 && c < 8) {
      re = acc.gr[0][j] + scratch[(r + 8) * 17 + c + 8];
      im = scratch[r * 17 + c + 8] - scratch[(r + 8) * 17 + c];
    }
    if (r < c) {
      As[r * ast + c] = make_float2(re, im);
      As[c * ast + r] = make_float2(re, -im);
    } else if (r == c) {
      As[r * ast + r] = make_float2(re + reg, 0.f);
      Gd[r] = re;
    }
  }
}

}  // namespace mimo

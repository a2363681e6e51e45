// Device helpers shared by the gfx950 kernels: wave-level reductions over
// 16-lane DPP rows, LDS ordering inside one wavefront, complex arithmetic and
// MFMA wrappers.  Everything here assumes 64-wide wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mimo {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;

// ---------------------------------------------------------------- ordering
// One wavefront owns each LDS region, so cross-lane exchange through LDS
// needs no s_barrier: LDS instructions of one wave execute in order.  The
// asm statement is a compiler barrier for memory operations (its memory
// clobber) and waits for the wave's own outstanding LDS operations; it
// waits for nothing else.  (A workgroup-scope memory fence would also do,
// but while loads into LDS are in flight it waits for every outstanding
// vector-memory operation, which would drain a kernel's prefetch.)
__device__ __forceinline__ void wave_lds_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// Wait until at most N of the wave's vector-memory operations (loads,
// stores, loads into LDS) are outstanding; they complete in issue order.
// Loads into LDS are invisible to the compiler's own counter waits, so
// kernels that issue them wait explicitly; the memory clobber keeps LDS
// reads of the landed data below the wait.
template <int N>
__device__ __forceinline__ void vm_wait() {
  static_assert(N >= 0 && N <= 63, "vmcnt is a 6-bit counter");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// ---------------------------------------------------------------- DPP
// DPP controls within a row of 16 lanes.
constexpr int kQuadSwap1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kQuadSwap2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;  // lane i <- lane 7-i within 8
constexpr int kRowMirror = 0x140;      // lane i <- lane 15-i within 16

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 16 lanes of a DPP row; every lane of the row receives the
// bitwise-identical result (each step adds two partial sums that are the
// same pair in both lanes).
template <typename T>
__device__ __forceinline__ T row_sum16(T x) {
  x += dpp<kQuadSwap1>(x);
  x += dpp<kQuadSwap2>(x);
  x += dpp<kRowHalfMirror>(x);
  x += dpp<kRowMirror>(x);
  return x;
}

// Four independent row sums, advanced step by step so the DPP latencies of
// the four chains overlap.
template <typename T>
__device__ __forceinline__ void row_sum16_x4(T (&x)[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] += dpp<kQuadSwap1>(x[j]);
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] += dpp<kQuadSwap2>(x[j]);
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] += dpp<kRowHalfMirror>(x[j]);
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] += dpp<kRowMirror>(x[j]);
}

// Full-wave sum (64 lanes) via cross-lane shuffles; result in every lane.
template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// ---------------------------------------------------------------- complex
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a += b * c
__device__ __forceinline__ void cfma(float2& a, float2 b, float2 c) {
  a.x = __builtin_fmaf(b.x, c.x, a.x);
  a.x = __builtin_fmaf(-b.y, c.y, a.x);
  a.y = __builtin_fmaf(b.x, c.y, a.y);
  a.y = __builtin_fmaf(b.y, c.x, a.y);
}
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

// ---------------------------------------------------------------- MFMA
// D = A(16x4) B(4x16) + C with lane l supplying A[l%16][l/16] and
// B[l/16][l%16]; lane l receives D[4*(l/16)+j][l%16] in element j.
__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// 16x16x32 with 16-bit inputs: lane l supplies 8 consecutive k of row /
// column l%16 from k-group l/16; the k order is the same for A and B.
__device__ __forceinline__ f4 mfma32(h8 a, h8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma32(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f4 zero4() { return f4{0.f, 0.f, 0.f, 0.f}; }

}  // namespace mimo

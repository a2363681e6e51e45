// Kernel parameter blocks and launch geometry (C++ linkage, internal to the
// library; the public entry points are in abi.hip, the host launchers are
// declared in launch.hpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mimo {

struct DetectParams {
  const void* H;        // [n_sc][B][U] storage per in_dtype
  const void* Y;        // [n_sc][B][S]
  int B, U, S, K;
  int64_t n_sc;
  float reg;            // N0 / E_s
  float n0;             // N0
  float es;             // E_s
  float scale;          // constellation level unit sqrt(3 E_s / (2 (M - 1)))
  float inv_scale;      // 1 / scale
  float* llr;           // [n_sc][U][S][m]
  float2* xhat;         // [n_sc][U][S] or null
  float* mu;            // [n_sc][U][S] or null
  float* sinr;          // [n_sc][U][S] or null
  const float2* gram;   // [n_sc][U][U] cached G = H^H H of this H, or null (formed from H)
};

struct PrecodeParams {
  const void* H;        // [n_sc][B][U]
  const float2* T;      // [n_sc][U][S]
  int B, U, S, K;
  int64_t n_sc;
  float beta;
  int normalize;
  float2* Q;            // [n_sc][B][S]
  float* qnorm;         // [n_sc][S] or null
  const float2* gram;   // [n_sc][U][U] cached G = H_d H_d^H of this H, or null
};

// One uplink + downlink slot on a reciprocal channel: detection and
// precoding of the same subcarriers with the same H (ul.H == dl.H, equal B,
// U and n_sc; S and K may differ).
struct SlotParams {
  DetectParams ul;
  PrecodeParams dl;
};

struct GramParams {
  const void* H;
  const void* Y;        // may be null
  int B, U, S;
  int64_t n_sc;
  float reg;
  float2* A;            // [n_sc][U][U]
  float2* b;            // [n_sc][U][S] or null
};

// A wave-uniform int hidden from the optimizer.  The kernels pass their
// sizes through it at the top of each subcarrier iteration: the sizes then
// change per iteration as far as the compiler can tell, so the per-k-step
// and per-tile masks and offsets derived from them are recomputed on the
// scalar unit where they are used, instead of being hoisted out of the
// subcarrier loop and kept live across it.  Dozens of hoisted values
// overflow the scalar registers, and each spilled one then costs a VALU
// lane read at every use.
__device__ __forceinline__ int opaque_int(int x) {
  asm volatile("" : "+s"(x));
  return x;
}
__device__ __forceinline__ DetectParams opaque_sizes(DetectParams p) {
  p.B = opaque_int(p.B);
  p.U = opaque_int(p.U);
  p.S = opaque_int(p.S);
  p.K = opaque_int(p.K);
  return p;
}
__device__ __forceinline__ PrecodeParams opaque_sizes(PrecodeParams p) {
  p.B = opaque_int(p.B);
  p.U = opaque_int(p.U);
  p.S = opaque_int(p.S);
  p.K = opaque_int(p.K);
  return p;
}

__device__ __forceinline__ GramParams opaque_sizes(GramParams p) {
  p.B = opaque_int(p.B);
  p.U = opaque_int(p.U);
  p.S = opaque_int(p.S);
  return p;
}

// Batched launches: up to kMaxBatch frames of different shapes in one
// kernel, passed by value in the kernel arguments.
constexpr int kMaxBatch = 32;
struct FrameArgs {
  const void* H;        // [n_sc][B][U]
  const void* Y;        // detect: Y [n_sc][B][S]; precode: T complex64 [n_sc][U][S]
  void* out;            // detect: llr; precode: Q
  void* out2;           // detect: xhat or null; precode: qnorm or null
  const void* gram;     // cached G, complex64 [n_sc][U][U], or null
  int64_t sc_begin;     // first global subcarrier of the frame
  int64_t n_sc;
  int B, U, S, K;
  float reg, n0, es, scale, inv_scale;   // detection
  float beta;                            // precoding
  int normalize;
  int pad;
};
struct BatchArgs {
  int n;                // frames
  int pad;
  int64_t total;        // subcarriers over all frames
  FrameArgs f[kMaxBatch];
};

// Frame of global subcarrier gsc: the last f with sc_begin <= gsc.
__device__ __forceinline__ int find_frame(const BatchArgs& a, int64_t gsc) {
  int lo = 0, hi = a.n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.f[mid].sc_begin <= gsc) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// A kernel schedule: the kernel form of an operation and its grid.
// blocks_per_cu = 0 launches one wavefront per subcarrier; k > 0 launches a
// persistent grid of k blocks (4 wavefronts each) per compute unit that
// loops over subcarriers.
struct Schedule {
  int variant;
  int blocks_per_cu;
};
enum { kDetectGeneric = 0, kDetectStream = 1, kDetectStreamSmall = 2, kDetectPlain = 3,
       kDetectRing = 4, kDetectSplit = 5, kDetectValu = 6, kDetectX3 = 7, kDetectVariants = 8 };
enum { kPrecodeGeneric = 0, kPrecodeStream = 1, kPrecodeStreamSmall = 2, kPrecodeResident = 3,
       kPrecodeSplit = 4, kPrecodeX3 = 5, kPrecodeVariants = 6 };
// uplink + downlink slot: two launches (detection and precoding with their
// own schedules), or one fused H-resident kernel (FP32-MFMA or bf16-split
// Gram and matched filter)
enum { kSlotSeparate = 0, kSlotFused = 1, kSlotFusedX3 = 2, kSlotVariants = 3 };

int num_compute_units();   // of the current device (cached per device)

inline unsigned int sched_grid(int64_t n_sc, const Schedule& s) {
  int64_t blocks = (n_sc + 3) / 4;
  if (s.blocks_per_cu > 0) {
    const int64_t cap = (int64_t)num_compute_units() * s.blocks_per_cu;
    if (blocks > cap) blocks = cap;
  }
  if (blocks > (1 << 20)) blocks = 1 << 20;
  if (blocks < 1) blocks = 1;
  return (unsigned int)blocks;
}

}  // namespace mimo

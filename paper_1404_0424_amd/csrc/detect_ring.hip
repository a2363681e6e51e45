// LDS-ring form of the fused CG-D detection kernel (Sec. III-B, III-C-2,
// Algorithm 1, eqs. (4), (13)-(15)) for complex64 storage, U <= 16, S <= 16.
//
// Each wavefront (one per workgroup) walks its subcarriers with the input
// streamed through a ring of kRingSlots LDS slots by loads that write LDS
// directly (buffer_load ... lds, 16 bytes per lane, 1 KiB per instruction).
// A slot holds one chunk of 16 antennas of H and of Y in their global
// layout ([rows][U] and [rows][S] complex64).  The wave keeps kRingSlots
// chunks in flight at all times -- the chunks after the one whose MFMAs run,
// across subcarrier boundaries -- so the next subcarrier's loads stay in
// flight through the CG, SINR and LLR phases without holding registers.  The
// Gram / matched-filter MFMAs take their operands from the slot in the same
// k-steps and order as the register-streaming kernels, so the results are
// bitwise identical to theirs.
//
// The compiler's counter waits do not see loads into LDS, so the kernel
// waits with explicit vmcnt immediates.  Every path issues the same
// vector-memory instructions -- RingGeom::NI loads per chunk (lanes past the
// chunk and chunks past the wave's last subcarrier address nothing) and
// kStagedStores stores per subcarrier -- and they complete in issue order,
// so the number issued after a chunk's loads is a compile-time constant:
//   chunks 0 .. R-1 of a subcarrier after the wave's first: the R-1 chunks
//   issued after it plus the previous subcarrier's stores;
//   every other chunk: the R-1 chunks issued after it.
// (This needs at least R chunks per subcarrier and no optional xhat, mu or
// SINR outputs; the host takes the register-streaming kernel otherwise.)
#include "detect_core.hpp"
#include "launch.hpp"

namespace mimo {

constexpr int kRingSlots = 3;   // R: chunks in flight per wave
constexpr int kRingRows = 16;   // antennas per chunk (4 MFMA k-steps)

template <int W>
struct RingGeom {
  static constexpr int H_BYTES = kRingRows * 16 * W * 8;   // up to 16 W users
  static constexpr int Y_BYTES = kRingRows * 16 * 8;       // up to 16 rhs
  static constexpr int SLOT = H_BYTES + Y_BYTES;
  static constexpr int NI_H = H_BYTES / 1024;              // 1 KiB per load
  static constexpr int NI_Y = Y_BYTES / 1024;
  static constexpr int NI = NI_H + NI_Y;                   // loads per chunk
};

typedef __attribute__((address_space(3))) void* lds_void_ptr;

// One load of 16 bytes per lane into LDS: lane l writes dst + 16 l.  An
// offset outside the descriptor's range reads nothing.
__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t r, char* dst, uint32_t voff) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_void_ptr)dst, 16, voff, 0, 0, kStreamCPol);
}

// Issues the wave's chunks in order: chunk ci of subcarrier m, then the next.
template <int W>
struct RingFeed {
  const float2* H;
  const float2* Y;
  int B, U, S, nch;
  int64_t n_sc, stride;
  int64_t m;   // subcarrier of the next chunk to issue
  int ci;      // its chunk index
  __device__ void issue(char* slot, int lane) {
    using G = RingGeom<W>;
    const bool live = m < n_sc;
    const int64_t mm = live ? m : 0;
    const __amdgpu_buffer_rsrc_t rh =
        make_rsrc(H + mm * B * U, live ? (uint32_t)B * U * 8u : 0u);
    const __amdgpu_buffer_rsrc_t ry =
        make_rsrc(Y + mm * B * S, live ? (uint32_t)B * S * 8u : 0u);
    const int rows = B - kRingRows * ci < kRingRows ? B - kRingRows * ci : kRingRows;
    const uint32_t hb = (uint32_t)rows * U * 8u, yb = (uint32_t)rows * S * 8u;
    const uint32_t h0 = (uint32_t)(kRingRows * ci) * U * 8u;
    const uint32_t y0 = (uint32_t)(kRingRows * ci) * S * 8u;
#pragma unroll
    for (int k = 0; k < G::NI_H; ++k) {
      const uint32_t o = (uint32_t)(k * 1024 + lane * 16);
      dma16(rh, slot + k * 1024, o < hb ? h0 + o : kOOB);
    }
#pragma unroll
    for (int k = 0; k < G::NI_Y; ++k) {
      const uint32_t o = (uint32_t)(k * 1024 + lane * 16);
      dma16(ry, slot + G::H_BYTES + k * 1024, o < yb ? y0 + o : kOOB);
    }
    if (++ci == nch) {
      ci = 0;
      m += stride;
    }
  }
};

// LDS address of a generic pointer into __shared__ memory.
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)(uintptr_t)(lds_void_ptr)p;
}

typedef float f2v __attribute__((ext_vector_type(2)));

// Reads of one k-step's operands from a ring slot, written in asm: the
// compiler treats any LDS read of the ring as possibly overlapping a load
// into LDS in flight and would wait for all of them (draining the ring); the
// kernel's explicit waits already order these reads after their chunk
// landed.  The asm waits for its own reads before returning its outputs.
__device__ __forceinline__ void ring_lds_read(f2v& h0, f2v& y, uint32_t ah0, uint32_t ay) {
  asm volatile(
      "ds_read_b64 %0, %2\n\t"
      "ds_read_b64 %1, %3\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(h0), "=&v"(y)
      : "v"(ah0), "v"(ay)
      : "memory");
}
__device__ __forceinline__ void ring_lds_read(f2v& h0, f2v& h1, f2v& y, uint32_t ah0,
                                              uint32_t ah1, uint32_t ay) {
  asm volatile(
      "ds_read_b64 %0, %3\n\t"
      "ds_read_b64 %1, %4\n\t"
      "ds_read_b64 %2, %5\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(h0), "=&v"(h1), "=&v"(y)
      : "v"(ah0), "v"(ah1), "v"(ay)
      : "memory");
}

// MFMA operands of one chunk from its slot: k-step t, lane (c, g) takes
// antenna row 4 t + g, user 16 w + c of H (the packed form: user c & 7) and
// rhs c of Y; rows past the chunk, users >= U and rhs >= S are zero.
template <int W, bool PACKED>
__device__ __forceinline__ void ring_read(BlockC32<W, 4>& blk, const char* slot, int U, int S,
                                          int rows, int c, int g) {
  static_assert(W == 1 || W == 2, "one or two user tiles");
  using G = RingGeom<W>;
  const uint32_t hs = lds_addr(slot), ys = hs + G::H_BYTES;
  const float2 z = make_float2(0.f, 0.f);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int r = 4 * t + g;
    const bool okr = r < rows;
    bool okh[W];
    uint32_t ah[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int u = PACKED ? (c & 7) : 16 * w + c;
      okh[w] = okr && u < U;
      ah[w] = hs + (uint32_t)(okh[w] ? r * U + u : 0) * 8u;
    }
    const bool oky = okr && c < S;
    const uint32_t ay = ys + (uint32_t)(oky ? r * S + c : 0) * 8u;
    f2v hv[W], yv;
    if constexpr (W == 1) ring_lds_read(hv[0], yv, ah[0], ay);
    else ring_lds_read(hv[0], hv[1], yv, ah[0], ah[1], ay);
#pragma unroll
    for (int w = 0; w < W; ++w) blk.h[t][w] = okh[w] ? make_float2(hv[w].x, hv[w].y) : z;
    blk.y[t] = oky ? make_float2(yv.x, yv.y) : z;
  }
}

template <int W, bool PACKED, typename ST, int M_BITS>
__global__ __launch_bounds__(64) void detect_ring_kernel(DetectParams prm) {
  using G = RingGeom<W>;
  constexpr int R = kRingSlots;
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;
  constexpr int AP = 2 * (NU * AST + NU * kPST);   // A then P (floats)
  constexpr int STG = NU * 16 * M_BITS;            // LLR staging tile (floats)
  constexpr int WAIT = (R - 1) * G::NI;
  constexpr int WAIT_AFTER_STORES = WAIT + kStagedStores<W, M_BITS>;
  static_assert(WAIT_AFTER_STORES <= 63, "vmcnt immediate out of range");
  using Blk = typename std::conditional<PACKED, BlockC32P<4>, BlockC32<W, 4>>::type;
  using Tag = typename std::conditional<PACKED, InC32P, InC32>::type;
  __shared__ __align__(16) char ring[R][G::SLOT];
  __shared__ __align__(16) float W_s[AP > STG ? AP : STG];
  __shared__ float G_s[NU];
  const int lane = threadIdx.x;
  const int c = lane & 15, g = lane >> 4;
  float2* As = (float2*)W_s;
  float2* Ps = As + NU * AST;
  const int B = prm.B, U = prm.U, S = prm.S;
  const int nch = (B + kRingRows - 1) / kRingRows;
  const int64_t stride = gridDim.x;

  int64_t n = blockIdx.x;
  RingFeed<W> feed{(const float2*)prm.H, (const float2*)prm.Y, B, U, S, nch, prm.n_sc, stride,
                   n, 0};
#pragma unroll
  for (int r = 0; r < R; ++r) feed.issue(ring[r], lane);
  int slot = 0;             // slot of the next chunk to consume
  bool after_stores = false;
  while (n < prm.n_sc) {
    // ---- A = H^H H + (N0/E_s) I and b = H^H y (Algorithm 1, initialization)
    GramAcc<W> acc;
    acc.clear();
    for (int i = 0; i < nch; ++i) {
      if (after_stores && i < R) vm_wait<WAIT_AFTER_STORES>();
      else vm_wait<WAIT>();
      Blk blk;
      const int rows = B - kRingRows * i < kRingRows ? B - kRingRows * i : kRingRows;
      ring_read<W, PACKED>(blk, ring[slot], U, S, rows, c, g);
      blk.template mma<true, true>(acc);
      wave_lds_sync();                       // the slot's reads are done: refill it
      feed.issue(ring[slot], lane);
      slot = slot + 1 == R ? 0 : slot + 1;
    }
    finish_mf(Tag{}, acc);
    AOperand<W> at;
    float d[W];
    gram_to_operands<W>(Tag{}, acc, As, G_s, Ps, AST, prm.reg, U, c, g, at, d);
    cg_llr_epilogue<W, ST, M_BITS, true, true, true>(prm, n, 0, acc, at, d, G_s, Ps, c, g, W_s);
    after_stores = true;
    n += stride;
  }
  vm_wait<0>();             // no load into this workgroup's LDS outlives it
}

bool detect_ring_eligible(const DetectParams& p, int in_dtype) {
  const int nch = (p.B + kRingRows - 1) / kRingRows;
  return in_dtype == 0 && p.U <= 16 && p.S <= 16 && nch >= kRingSlots && !p.xhat && !p.mu &&
         !p.sinr &&
         ((int64_t)p.B * p.U) % 2 == 0 && ((int64_t)p.B * p.S) % 2 == 0;
}

template <int W, bool PACKED, typename ST>
static hipError_t launch_ring_m(const DetectParams& p, int m_bits, unsigned int blocks,
                                hipStream_t stream) {
  const dim3 grid(blocks), block(kWave);
  switch (m_bits) {
    case 2: hipLaunchKernelGGL((detect_ring_kernel<W, PACKED, ST, 2>), grid, block, 0, stream, p); break;
    case 4: hipLaunchKernelGGL((detect_ring_kernel<W, PACKED, ST, 4>), grid, block, 0, stream, p); break;
    case 6: hipLaunchKernelGGL((detect_ring_kernel<W, PACKED, ST, 6>), grid, block, 0, stream, p); break;
    case 8: hipLaunchKernelGGL((detect_ring_kernel<W, PACKED, ST, 8>), grid, block, 0, stream, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int W, bool PACKED>
static hipError_t launch_ring_st(const DetectParams& p, int f64, int m_bits, unsigned int blocks,
                                 hipStream_t stream) {
  return f64 ? launch_ring_m<W, PACKED, double>(p, m_bits, blocks, stream)
             : launch_ring_m<W, PACKED, float>(p, m_bits, blocks, stream);
}

// Persistent grid of single-wave workgroups: 4 k per compute unit for a
// schedule of k blocks per CU (the same wave count as k four-wave blocks),
// 8 per CU for k = 0; LDS holds about 8 of them per CU.
hipError_t launch_detect_ring(const DetectParams& p, int scalar_f64, int m_bits,
                              const Schedule& sch, hipStream_t stream) {
  const int64_t per_cu = sch.blocks_per_cu > 0 ? 4 * sch.blocks_per_cu : 8;
  int64_t blocks = (int64_t)num_compute_units() * per_cu;
  if (blocks > p.n_sc) blocks = p.n_sc;
  if (blocks < 1) blocks = 1;
  if (p.U <= 8) return launch_ring_st<1, true>(p, scalar_f64, m_bits, (unsigned int)blocks, stream);
  return launch_ring_st<1, false>(p, scalar_f64, m_bits, (unsigned int)blocks, stream);
}

}  // namespace mimo

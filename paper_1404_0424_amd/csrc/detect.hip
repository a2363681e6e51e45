// Fused CG-D kernel: Gram + matched filter (MFMA) -> K CG iterations with the
// approximate in-loop SINR tracker -> max-log LLR epilogue, one wavefront per
// subcarrier (Sec. III-B, III-C-2, Algorithm 1, eqs. (4), (13)-(15)).
#include <type_traits>

#include "detect_core.hpp"
#include "launch.hpp"

namespace mimo {

// Streaming kernel for S <= 16 (one right-hand-side chunk).  Each wavefront
// keeps the next block of H / Y loads in flight while the MFMAs of the
// current block run, and issues the first block of its next subcarrier
// before the CG / LLR phase of the current one, so HBM latency overlaps
// compute within the wave as well as across waves.
// VALU: CG mat-vec on VALU FMAs (schedule variant "stream-valu").
// CACHED: A from the cached Gram matrix prm.gram (the blocks feed only the
// matched filter), as detect_one's cached branch.
template <int W, typename IN, typename ST, int M_BITS, bool SMALL, bool VALU = false,
          bool CACHED = false>
__global__ __launch_bounds__(256, 2) void detect_stream_kernel(DetectParams kprm) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;   // LDS row stride (complex) of A
  using Sub = typename Storage<IN, W>::Sub;
  using Blk = typename std::conditional<SMALL, typename Storage<IN, W>::SmallBlock,
                                        typename Storage<IN, W>::Block>::type;
  // per wave: A then P (float2), reused as the LLR staging tile
  constexpr int AP = 2 * (NU * AST + NU * kPST);                     // floats
  constexpr int STG = NU * 16 * M_BITS;
  __shared__ __align__(16) float W_s[kWavesPerBlock][AP > STG ? AP : STG];
  __shared__ float G_s[kWavesPerBlock][NU];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  float2* As = (float2*)W_s[wv];
  float2* Ps = As + NU * AST;
  float* Gs = G_s[wv];
  const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;

  int64_t n = (int64_t)blockIdx.x * kWavesPerBlock + wv;
  Sub cur;
  Blk blk;
  if (n < kprm.n_sc) {
    const int B = kprm.B, U = kprm.U, S = kprm.S;
    cur.init(offset_sc(IN{}, kprm.H, n, B, U), offset_sc(IN{}, kprm.Y, n, B, S), B, U, S, 0, c,
             g);
    blk.template load<true>(cur, 0);
  }
  while (n < kprm.n_sc) {
    const DetectParams prm = opaque_sizes(kprm);
    const int B = prm.B, U = prm.U, S = prm.S;
    const int64_t nn = n + stride;
    const int64_t nc = nn < prm.n_sc ? nn : n;        // descriptors only used if nn < n_sc
    Sub nxt;
    nxt.init(offset_sc(IN{}, prm.H, nc, B, U), offset_sc(IN{}, prm.Y, nc, B, S), B, U, S, 0, c, g);
    if (nn >= prm.n_sc) nxt.disable();       // last subcarrier: prefetch reads nothing
    // ---- A = H^H H + (N0/E_s) I and b = H^H y (Algorithm 1, initialization)
    GramAcc<W> acc;
    acc.clear();
    // ping-pong between two block buffers: blk holds the block at b0, alt
    // receives the next one, and the last block's partner is the next
    // subcarrier's first block.  The blocks are walked in pairs: with an odd
    // block count the last pair's second block lies past B and reads zero
    // (no memory traffic), and its MFMAs add exact zeros to accumulators that
    // start at +0 and therefore never hold -0, so the values are those of the
    // unpadded walk bit for bit.  The loop then has a single exit, after which
    // only blk's loads (the next subcarrier's first block) are in flight: no
    // path leaves a load into alt pending, so nothing in the CG / LLR phase
    // waits for the prefetch.  With kUncondMem the prefetch is issued on
    // every path (an empty descriptor after the last subcarrier), so each
    // wait covers exactly the block consumed.
    Blk alt;
    for (int b0 = 0;; b0 += 2 * Blk::ANT) {
      alt.template load<true>(cur, b0 + Blk::ANT);
      blk.template mma<!CACHED, true>(acc);
      const bool more2 = b0 + 2 * Blk::ANT < B;
      if (kUncondMem<IN>)
        blk.template load<true>(more2 ? cur : nxt, more2 ? b0 + 2 * Blk::ANT : 0);
      else if (more2)
        blk.template load<true>(cur, b0 + 2 * Blk::ANT);
      else if (nn < prm.n_sc)
        blk.template load<true>(nxt, 0);
      alt.template mma<!CACHED, true>(acc);
      if (!more2) break;                           // blk holds the next subcarrier's block 0
    }
    finish_mf(IN{}, acc);
    AOperand<W> at;
    float d[W];
    if constexpr (CACHED)
      cached_gram_to_operands<W>(prm.gram + (size_t)n * U * U, U, prm.reg, As, Gs, AST, c, g,
                                 at, d);
    else
      gram_to_operands<W>(IN{}, acc, As, Gs, Ps, AST, prm.reg, U, c, g, at, d);
    cg_llr_epilogue<W, ST, M_BITS, kUncondMem<IN>, true, false, VALU>(prm, n, 0, acc, at, d, Gs,
                                                                       Ps, c, g, W_s[wv]);
    n = nn;
    cur = nxt;
  }
}

// All right-hand sides of subcarrier n, in chunks of 16; the Gram is
// computed with the first chunk and kept in LDS.
template <int W, typename IN, typename ST, int M_BITS>
// With all right-hand sides in one chunk (S <= 16) the LLR tile is staged in
// `stg` (A and P of the wave, contiguous, at least 16 W x 16 x M_BITS floats).
__device__ __forceinline__ void detect_one(const DetectParams& prm, int64_t n, float2* As,
                                           float2* Ps, float* Gs, int c, int g, float* stg) {
  constexpr int AST = 16 * W + 2;
  const int B = prm.B, U = prm.U, S = prm.S;
  const void* Hn = offset_sc(IN{}, prm.H, n, B, U);
  const void* Yn = offset_sc(IN{}, prm.Y, n, B, S);
  AOperand<W> at;
  float d[W];
  for (int s0 = 0; s0 < S; s0 += 16) {
    GramAcc<W> acc;
    acc.clear();
    if (s0 == 0 && prm.gram) {        // cached G: only the matched filter reads H
      gram_mf<W, false, true>(IN{}, Hn, Yn, B, U, S, s0, c, g, acc);
      cached_gram_to_operands<W>(prm.gram + (size_t)n * U * U, U, prm.reg, As, Gs, AST, c, g,
                                 at, d);
    } else if (s0 == 0) {
      gram_mf<W, true, true>(IN{}, Hn, Yn, B, U, S, s0, c, g, acc);
      gram_to_operands<W>(IN{}, acc, As, Gs, Ps, AST, prm.reg, U, c, g, at, d);
    } else {
      gram_mf<W, false, true>(IN{}, Hn, Yn, B, U, S, s0, c, g, acc);
    }
    if (S <= 16)
      cg_llr_epilogue<W, ST, M_BITS, kUncondMem<IN>, true>(prm, n, s0, acc, at, d, Gs, Ps, c, g,
                                                           stg);
    else
      cg_llr_epilogue<W, ST, M_BITS, kUncondMem<IN>>(prm, n, s0, acc, at, d, Gs, Ps, c, g);
  }
}

// Generic kernel (any S).
template <int W, typename IN, typename ST, int M_BITS>
__global__ __launch_bounds__(256, 2) void detect_approx_kernel(DetectParams prm) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;   // LDS row stride (complex) of A
  // per wave: A then P (float2), reused as the LLR staging tile
  constexpr int AP = 2 * (NU * AST + NU * kPST);                     // floats
  constexpr int STG = NU * 16 * M_BITS;
  __shared__ __align__(16) float W_s[kWavesPerBlock][AP > STG ? AP : STG];
  __shared__ float G_s[kWavesPerBlock][NU];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  float2* As = (float2*)W_s[wv];
  float2* Ps = As + NU * AST;
  for (int64_t n = (int64_t)blockIdx.x * kWavesPerBlock + wv; n < prm.n_sc;
       n += (int64_t)gridDim.x * kWavesPerBlock)
    detect_one<W, IN, ST, M_BITS>(opaque_sizes(prm), n, As, Ps, G_s[wv], c, g, W_s[wv]);
}

// Batched kernel: frames of different shapes (same user class, QAM order,
// storage and scalar precision) in one launch.  Frame f covers global
// subcarriers [sc_begin_f, sc_begin_f + n_sc_f); each wave finds its frame
// by a binary search over the (wave-uniform) descriptor table.
template <int W, typename IN, typename ST, int M_BITS>
__global__ __launch_bounds__(256, 2) void detect_batch_kernel(BatchArgs args) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;
  // per wave: A then P (float2), reused as the LLR staging tile
  constexpr int AP = 2 * (NU * AST + NU * kPST);                     // floats
  constexpr int STG = NU * 16 * M_BITS;
  __shared__ __align__(16) float W_s[kWavesPerBlock][AP > STG ? AP : STG];
  __shared__ float G_s[kWavesPerBlock][NU];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  float2* As = (float2*)W_s[wv];
  float2* Ps = As + NU * AST;
  for (int64_t gsc = (int64_t)blockIdx.x * kWavesPerBlock + wv; gsc < args.total;
       gsc += (int64_t)gridDim.x * kWavesPerBlock) {
    const int f = find_frame(args, gsc);
    const FrameArgs& F = args.f[f];
    DetectParams prm{F.H, F.Y, F.B, F.U, F.S, F.K, F.n_sc, F.reg, F.n0, F.es, F.scale,
                     F.inv_scale, (float*)F.out, (float2*)F.out2, nullptr, nullptr,
                     (const float2*)F.gram};
    if constexpr (std::is_same<IN, InC32>::value) {
      if (F.U <= 8) {               // packed form, as a single call of this frame runs
        detect_one<1, InC32P, ST, M_BITS>(prm, gsc - F.sc_begin, As, Ps, G_s[wv], c, g,
                                          W_s[wv]);
        continue;
      }
    }
    detect_one<W, IN, ST, M_BITS>(prm, gsc - F.sc_begin, As, Ps, G_s[wv], c, g, W_s[wv]);
  }
}

template <int W, typename IN, typename ST, int M>
static void launch_one(const DetectParams& p, const Schedule& sch, hipStream_t stream) {
  const dim3 grid(sched_grid(p.n_sc, sch)), block(kWave * kWavesPerBlock);
  if (p.S > 16 || sch.variant == kDetectGeneric || sch.variant == kDetectPlain)
    hipLaunchKernelGGL((detect_approx_kernel<W, IN, ST, M>), grid, block, 0, stream, p);
  else if (p.gram) {                   // cached Gram: launch_detect_approx leaves the two forms
    if (sch.variant == kDetectStream)
      hipLaunchKernelGGL((detect_stream_kernel<W, IN, ST, M, false, false, true>), grid, block, 0,
                         stream, p);
    else
      hipLaunchKernelGGL((detect_stream_kernel<W, IN, ST, M, true, false, true>), grid, block, 0,
                         stream, p);
  }
  else if (sch.variant == kDetectStreamSmall)
    hipLaunchKernelGGL((detect_stream_kernel<W, IN, ST, M, true>), grid, block, 0, stream, p);
  else if (sch.variant == kDetectValu) {
    if constexpr (std::is_same<IN, InC32>::value || std::is_same<IN, InC32P>::value)
      hipLaunchKernelGGL((detect_stream_kernel<W, IN, ST, M, true, true>), grid, block, 0, stream,
                         p);
    else
      hipLaunchKernelGGL((detect_stream_kernel<W, IN, ST, M, true>), grid, block, 0, stream, p);
  }
  else
    hipLaunchKernelGGL((detect_stream_kernel<W, IN, ST, M, false>), grid, block, 0, stream, p);
}

template <int W, typename IN, typename ST>
static hipError_t launch_m(const DetectParams& p, int m_bits, const Schedule& sch,
                           hipStream_t stream) {
  switch (m_bits) {
    case 2: launch_one<W, IN, ST, 2>(p, sch, stream); break;
    case 4: launch_one<W, IN, ST, 4>(p, sch, stream); break;
    case 6: launch_one<W, IN, ST, 6>(p, sch, stream); break;
    case 8: launch_one<W, IN, ST, 8>(p, sch, stream); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int W, typename IN>
static hipError_t launch_st(const DetectParams& p, int f64, int m_bits, const Schedule& sch,
                            hipStream_t stream) {
  return f64 ? launch_m<W, IN, double>(p, m_bits, sch, stream)
             : launch_m<W, IN, float>(p, m_bits, sch, stream);
}

template <int W>
static hipError_t launch_in(const DetectParams& p, int in_dtype, int f64, int m_bits,
                            const Schedule& sch, hipStream_t stream) {
  switch (in_dtype) {
    case 0:
      if (sch.variant == kDetectX3)        // Gram and matched filter from bf16 splits
        return launch_st<W, InC32X3>(p, f64, m_bits, Schedule{kDetectStreamSmall,
                                                                sch.blocks_per_cu}, stream);
      if constexpr (W == 1)
        if (p.U <= 8) return launch_st<1, InC32P>(p, f64, m_bits, sch, stream);
      return launch_st<W, InC32>(p, f64, m_bits, sch, stream);
    case 1: return launch_st<W, InF16>(p, f64, m_bits, sch, stream);
    case 2: return launch_st<W, InBF16>(p, f64, m_bits, sch, stream);
  }
  return hipErrorInvalidValue;
}

template <int W, typename IN, typename ST>
static hipError_t launch_batch_m(const BatchArgs& a, int m_bits, const Schedule& sch,
                                 hipStream_t stream) {
  const dim3 grid(sched_grid(a.total, sch)), block(kWave * kWavesPerBlock);
  switch (m_bits) {
    case 2: hipLaunchKernelGGL((detect_batch_kernel<W, IN, ST, 2>), grid, block, 0, stream, a); break;
    case 4: hipLaunchKernelGGL((detect_batch_kernel<W, IN, ST, 4>), grid, block, 0, stream, a); break;
    case 6: hipLaunchKernelGGL((detect_batch_kernel<W, IN, ST, 6>), grid, block, 0, stream, a); break;
    case 8: hipLaunchKernelGGL((detect_batch_kernel<W, IN, ST, 8>), grid, block, 0, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int W, typename IN>
static hipError_t launch_batch_st(const BatchArgs& a, int f64, int m_bits, const Schedule& sch,
                                  hipStream_t stream) {
  return f64 ? launch_batch_m<W, IN, double>(a, m_bits, sch, stream)
             : launch_batch_m<W, IN, float>(a, m_bits, sch, stream);
}

template <int W>
static hipError_t launch_batch_in(const BatchArgs& a, int in_dtype, int f64, int m_bits,
                                  const Schedule& sch, hipStream_t stream) {
  switch (in_dtype) {
    case 0: return launch_batch_st<W, InC32>(a, f64, m_bits, sch, stream);
    case 1: return launch_batch_st<W, InF16>(a, f64, m_bits, sch, stream);
    case 2: return launch_batch_st<W, InBF16>(a, f64, m_bits, sch, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_detect_batch(const BatchArgs& a, int max_u, int in_dtype, int scalar_f64,
                               int m_bits, const Schedule& sch, hipStream_t stream) {
  if (max_u <= 16) return launch_batch_in<1>(a, in_dtype, scalar_f64, m_bits, sch, stream);
  return launch_batch_in<2>(a, in_dtype, scalar_f64, m_bits, sch, stream);
}

hipError_t launch_detect_approx(const DetectParams& p, int in_dtype, int scalar_f64, int m_bits,
                                const Schedule& sch, hipStream_t stream) {
  // a cached Gram runs the generic kernel or the streaming forms (others map to
  // stream-small)
  if (p.gram && sch.variant != kDetectGeneric && sch.variant != kDetectStream &&
      sch.variant != kDetectStreamSmall)
    return launch_detect_approx(p, in_dtype, scalar_f64, m_bits,
                                Schedule{kDetectStreamSmall, sch.blocks_per_cu}, stream);
  if (sch.variant == kDetectPlain && in_dtype == 0)
    return launch_detect_plain(p, scalar_f64, m_bits, sch, stream);
  if (sch.variant == kDetectSplit) {
    if (split_eligible(in_dtype, p.U, p.S, p.B, false))
      return launch_detect_split(p, scalar_f64, m_bits, sch, stream);
    return launch_detect_approx(p, in_dtype, scalar_f64, m_bits,
                                Schedule{kDetectStreamSmall, sch.blocks_per_cu}, stream);
  }
  if (sch.variant == kDetectRing) {
    if (detect_ring_eligible(p, in_dtype))
      return launch_detect_ring(p, scalar_f64, m_bits, sch, stream);
    return launch_detect_approx(p, in_dtype, scalar_f64, m_bits,
                                Schedule{kDetectStreamSmall, sch.blocks_per_cu}, stream);
  }
  if (p.U <= 16) return launch_in<1>(p, in_dtype, scalar_f64, m_bits, sch, stream);
  return launch_in<2>(p, in_dtype, scalar_f64, m_bits, sch, stream);
}

}  // namespace mimo

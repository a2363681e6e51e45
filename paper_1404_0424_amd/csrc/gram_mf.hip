// Standalone regularized Gram matrix and matched filter (Algorithm 1,
// initialization), and the ingest kernel that rounds complex64 channel /
// receive data to the blocked FP16 / BF16 storage the MFMA phase reads.
#include "gram_phase.hpp"
#include "launch.hpp"

namespace mimo {

template <int W, typename IN, bool HAS_Y>
__global__ __launch_bounds__(256) void gram_mf_kernel(GramParams prm) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;
  __shared__ __align__(16) float2 A_s[kWavesPerBlock][NU * AST];
  __shared__ float G_s[kWavesPerBlock][NU];
  __shared__ float X_s[kWavesPerBlock][gram_scratch_floats<W>()];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  float2* As = A_s[wv];
  const int B = prm.B, U = prm.U, S = prm.S;
  for (int64_t n = (int64_t)blockIdx.x * kWavesPerBlock + wv; n < prm.n_sc;
       n += (int64_t)gridDim.x * kWavesPerBlock) {
    const void* Hn = offset_sc(IN{}, prm.H, n, B, U);
    const void* Yn = HAS_Y ? offset_sc(IN{}, prm.Y, n, B, S) : nullptr;
    const int nchunk = HAS_Y ? (S + 15) / 16 : 1;
    for (int ch = 0; ch < nchunk; ++ch) {
      const int s0 = 16 * ch;
      GramAcc<W> acc;
      acc.clear();
      if (ch == 0) {
        gram_mf<W, true, HAS_Y>(IN{}, Hn, Yn, B, U, S, s0, c, g, acc);
        store_gram_lds<W>(acc, As, G_s[wv], X_s[wv], AST, prm.reg, c, g);
        wave_lds_sync();
        float2* An = prm.A + (size_t)n * U * U;
        for (int idx = lane; idx < U * U; idx += kWave) An[idx] = As[(idx / U) * AST + idx % U];
        wave_lds_sync();
      } else {
        gram_mf<W, false, HAS_Y>(IN{}, Hn, Yn, B, U, S, s0, c, g, acc);
      }
      if (HAS_Y && prm.b) {
#pragma unroll
        for (int w = 0; w < W; ++w)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int u = 16 * w + c, s = s0 + 4 * g + j;
            if (u < U && s < S)
              prm.b[((size_t)n * U + u) * S + s] = make_float2(acc.dr[w][j], acc.di[w][j]);
          }
      }
    }
  }
}

// Streaming form for S <= 16 (one right-hand-side chunk): the H / Y blocks
// ping-pong between two register buffers with the next block's loads in
// flight during the current block's MFMAs, and the first block of the
// wave's next subcarrier is issued before A and b of the current one are
// written.  Loads are issued on every path (an empty descriptor after the
// last subcarrier).  Same arithmetic in the same order as gram_mf_kernel.
template <int W, typename IN, bool HAS_Y>
__global__ __launch_bounds__(256, W == 1 ? 3 : 2) void gram_mf_stream_kernel(GramParams kprm) {
  constexpr int NU = 16 * W;
  constexpr int AST = NU + 2;
  using Sub = typename Storage<IN, W>::Sub;
  using Blk = typename Storage<IN, W>::SmallBlock;
  __shared__ __align__(16) float2 A_s[kWavesPerBlock][NU * AST];
  __shared__ float G_s[kWavesPerBlock][NU];
  __shared__ float X_s[kWavesPerBlock][gram_scratch_floats<W>()];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
  const int c = lane & 15, g = lane >> 4;
  float2* As = A_s[wv];
  const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock;
  auto y_of = [&](int64_t m, int B, int S) {
    return HAS_Y ? offset_sc(IN{}, kprm.Y, m, B, S) : nullptr;
  };

  int64_t n = (int64_t)blockIdx.x * kWavesPerBlock + wv;
  Sub cur;
  Blk blk;
  if (n < kprm.n_sc) {
    const int B = kprm.B, U = kprm.U, S = kprm.S;
    cur.init(offset_sc(IN{}, kprm.H, n, B, U), y_of(n, B, S), B, U, S, 0, c, g);
    blk.template load<HAS_Y>(cur, 0);
  }
  while (n < kprm.n_sc) {
    const GramParams prm = opaque_sizes(kprm);
    const int B = prm.B, U = prm.U, S = prm.S;
    const int64_t nn = n + stride;
    const int64_t nc = nn < prm.n_sc ? nn : n;
    Sub nxt;
    nxt.init(offset_sc(IN{}, prm.H, nc, B, U), y_of(nc, B, S), B, U, S, 0, c, g);
    if (nn >= prm.n_sc) nxt.disable();
    GramAcc<W> acc;
    acc.clear();
    Blk alt;
    // pairs of blocks; an odd count's last partner lies past B and reads
    // zero, adding exact zeros (one loop exit, so nothing after the Gram
    // waits for the next subcarrier's block in flight)
    for (int b0 = 0;; b0 += 2 * Blk::ANT) {
      alt.template load<HAS_Y>(cur, b0 + Blk::ANT);
      blk.template mma<true, HAS_Y>(acc);
      const bool more2 = b0 + 2 * Blk::ANT < B;
      blk.template load<HAS_Y>(more2 ? cur : nxt, more2 ? b0 + 2 * Blk::ANT : 0);
      alt.template mma<true, HAS_Y>(acc);
      if (!more2) break;
    }
    if (HAS_Y) finish_mf(IN{}, acc);
    store_gram_lds<W>(acc, As, G_s[wv], X_s[wv], AST, prm.reg, c, g);
    wave_lds_sync();
    float2* An = prm.A + (size_t)n * U * U;
    for (int idx = lane; idx < U * U; idx += kWave) An[idx] = As[(idx / U) * AST + idx % U];
    if (HAS_Y && prm.b) {
#pragma unroll
      for (int w = 0; w < W; ++w)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int u = 16 * w + c, s = 4 * g + j;
          if (u < U && s < S)
            prm.b[((size_t)n * U + u) * S + s] = make_float2(acc.dr[w][j], acc.di[w][j]);
        }
    }
    wave_lds_sync();
    n = nn;
    cur = nxt;
  }
}

template <int W, typename IN>
static hipError_t launch_y(const GramParams& p, const Schedule& sch, hipStream_t stream) {
  const dim3 grid(sched_grid(p.n_sc, sch)), block(kWave * kWavesPerBlock);
  const bool stream_form = sch.variant == kGramStream && (!p.Y || p.S <= 16);
  if (p.Y && stream_form)
    hipLaunchKernelGGL((gram_mf_stream_kernel<W, IN, true>), grid, block, 0, stream, p);
  else if (stream_form)
    hipLaunchKernelGGL((gram_mf_stream_kernel<W, IN, false>), grid, block, 0, stream, p);
  else if (p.Y)
    hipLaunchKernelGGL((gram_mf_kernel<W, IN, true>), grid, block, 0, stream, p);
  else
    hipLaunchKernelGGL((gram_mf_kernel<W, IN, false>), grid, block, 0, stream, p);
  return hipGetLastError();
}

template <int W>
static hipError_t launch_in(const GramParams& p, int in_dtype, const Schedule& sch,
                            hipStream_t stream) {
  switch (in_dtype) {
    case 0: return launch_y<W, InC32>(p, sch, stream);
    case 1: return launch_y<W, InF16>(p, sch, stream);
    case 2: return launch_y<W, InBF16>(p, sch, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gram_mf(const GramParams& p, int in_dtype, const Schedule& sch,
                          hipStream_t stream) {
  if (p.U <= 16) return launch_in<1>(p, in_dtype, sch, stream);
  return launch_in<2>(p, in_dtype, sch, stream);
}

// ---------------------------------------------------------------- ingest
// Round-to-nearest-even float -> bf16 on the bit pattern (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  const uint32_t u = __builtin_bit_cast(uint32_t, x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ uint16_t f32_to_f16_rne(float x) {
  return __builtin_bit_cast(uint16_t, (_Float16)x);   // v_cvt_f16_f32, RNE mode
}

// One thread per (subcarrier, 8-row block, column): reads 8 complex values
// of a column (coalesced across threads along the column index) and writes
// 8 contiguous real parts and 8 contiguous imaginary parts.
template <bool BF16>
__global__ __launch_bounds__(256) void convert_kernel(const float2* __restrict__ src,
                                                      uint16_t* __restrict__ dst, int64_t n,
                                                      int R, int C) {
  const int64_t nblk = (int64_t)(R >> 3);
  const int64_t total = n * nblk * C;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(i % C);
    const int64_t rb = i / C;                 // global 8-row block (n * nblk + kb)
    const float2* s = src + rb * 8 * C + col;
    uint16_t re[8], im[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float2 x = s[(size_t)e * C];
      re[e] = BF16 ? f32_to_bf16_rne(x.x) : f32_to_f16_rne(x.x);
      im[e] = BF16 ? f32_to_bf16_rne(x.y) : f32_to_f16_rne(x.y);
    }
    uint16_t* d = dst + ((rb * 2) * C + col) * 8;
    uint4 vr, vi;
    vr.x = re[0] | ((uint32_t)re[1] << 16); vr.y = re[2] | ((uint32_t)re[3] << 16);
    vr.z = re[4] | ((uint32_t)re[5] << 16); vr.w = re[6] | ((uint32_t)re[7] << 16);
    vi.x = im[0] | ((uint32_t)im[1] << 16); vi.y = im[2] | ((uint32_t)im[3] << 16);
    vi.z = im[4] | ((uint32_t)im[5] << 16); vi.w = im[6] | ((uint32_t)im[7] << 16);
    *(uint4*)d = vr;
    *(uint4*)(d + (size_t)C * 8) = vi;
  }
}

hipError_t launch_convert(const float2* src, uint16_t* dst, int dst_dtype, int64_t n, int R,
                          int C, hipStream_t stream) {
  const int64_t total = n * (R >> 3) * (int64_t)C;
  int64_t blocks = (total + 255) / 256;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  if (blocks < 1) blocks = 1;
  if (dst_dtype == 2)
    hipLaunchKernelGGL((convert_kernel<true>), dim3((unsigned)blocks), dim3(256), 0, stream, src,
                       dst, n, R, C);
  else
    hipLaunchKernelGGL((convert_kernel<false>), dim3((unsigned)blocks), dim3(256), 0, stream, src,
                       dst, n, R, C);
  return hipGetLastError();
}

}  // namespace mimo

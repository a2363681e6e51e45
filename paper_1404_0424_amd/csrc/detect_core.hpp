// Per-subcarrier CG / SINR / LLR stage of the CG-D detection kernels
// (Algorithm 1 loop body, eqs. (4), (13)-(15)) and the hand-over from the
// Gram phase, shared by the register-streaming kernels and the LDS-ring
// kernel.
#pragma once

#include <type_traits>

#include "cg_core.hpp"
#include "gram_phase.hpp"
#include "kernels.hpp"
#include "llr.hpp"

namespace mimo {

// Output descriptors of one subcarrier: LLR, xhat, mu and sinr as buffer
// resources over that subcarrier's [U][S] entries (zero-size when the
// optional output is absent), so every lane issues the same stores and
// masked entries are dropped by the range check: no branches around the
// stores, and the compiler's memory-counter waits stay exact.
template <int M_BITS>
struct DetectStore {
  __amdgpu_buffer_rsrc_t llr, xhat, mu, sinr;
  __device__ void init(const DetectParams& p, int64_t n) {
    const uint32_t per = (uint32_t)(p.U * p.S);
    llr = make_rsrc(p.llr + (size_t)n * per * M_BITS, per * M_BITS * 4u);
    xhat = make_rsrc(p.xhat ? (const void*)(p.xhat + (size_t)n * per) : p.llr,
                     p.xhat ? per * 8u : 0u);
    mu = make_rsrc(p.mu ? (const void*)(p.mu + (size_t)n * per) : p.llr, p.mu ? per * 4u : 0u);
    sinr = make_rsrc(p.sinr ? (const void*)(p.sinr + (size_t)n * per) : p.llr,
                     p.sinr ? per * 4u : 0u);
  }
  // xhat, mu, sinr of entry e = u * S + s (or -1 for a masked lane)
  __device__ void store_aux(int e, float2 x, float m, float rho) const {
    const bool ok = e >= 0;
    bstore2<0>(xhat, ok ? (uint32_t)e * 8u : kOOB, x.x, x.y);
    const uint32_t o4 = ok ? (uint32_t)e * 4u : kOOB;
    bstore1<0>(mu, o4, m);
    bstore1<0>(sinr, o4, rho);
  }
  // entry e = u * S + s, or -1 for a masked lane
  __device__ void store(int e, const float (&out)[M_BITS], float2 x, float m, float rho) const {
    const bool ok = e >= 0;
    const uint32_t ol = ok ? (uint32_t)e * (M_BITS * 4u) : kOOB;
    if constexpr (M_BITS == 2) {
      bstore2(llr, ol, out[0], out[1]);
    } else if constexpr (M_BITS == 4) {
      bstore4(llr, ol, out[0], out[1], out[2], out[3]);
    } else if constexpr (M_BITS == 6) {
      bstore3(llr, ol, out[0], out[1], out[2]);
      bstore3(llr, ol + 12u, out[3], out[4], out[5]);
    } else {
      bstore4(llr, ol, out[0], out[1], out[2], out[3]);
      bstore4(llr, ol + 16u, out[4], out[5], out[6], out[7]);
    }
    bstore2<0>(xhat, ok ? (uint32_t)e * 8u : kOOB, x.x, x.y);
    const uint32_t o4 = ok ? (uint32_t)e * 4u : kOOB;
    bstore1<0>(mu, o4, m);
    bstore1<0>(sinr, o4, rho);
  }
};

// Memory-op form per storage type, chosen by measurement on MI355X: with
// complex64 storage the unconditional prefetch and buffer-descriptor stores
// are faster (the compiler's load-counter waits then cover exactly the
// block consumed); with 16-bit storage the branchy form is faster.
template <typename IN>
constexpr bool kUncondMem = std::is_same<IN, InC32>::value || std::is_same<IN, InC32P>::value ||
                            std::is_same<IN, InC32X3>::value;

// LLR stores.  BUF: stores through buffer descriptors (no branches) or plain
// stores.  STAGE (all right-hand sides in this chunk): the subcarrier's LLR
// tile, U x S x M_BITS floats contiguous in memory, is assembled in `stg`
// (wave-private LDS, free once the CG is done) and written with one
// contiguous 16-byte (or 8-byte) piece per lane, so every store instruction
// covers whole cache lines; scattered 12-byte pieces let partly written lines
// leave L2 under load and reach HBM more than once.
// 8-byte store instructions that write a staged tile of up to 16 W users x
// 16 right-hand sides x M_BITS floats (FIXED_STORES form below).
template <int W, int M_BITS>
constexpr int kStagedStores = (16 * W * 16 * M_BITS / 2 + kWave - 1) / kWave;
// FIXED_STORES (with STAGE): the tile is written with exactly
// kStagedStores<W, M_BITS> 8-byte store instructions whatever U and S are
// (pieces past the tile are dropped by the range check) and the optional
// xhat, mu and SINR outputs are not written, so a caller that counts
// outstanding memory operations knows that this call adds exactly
// kStagedStores<W, M_BITS> of them.
// mu (eq. (14)), rho (eq. (15)), z = xhat / mu and the LLRs (eq. (4)) of
// right-hand sides s0 + 4 g + j of subcarrier n, from the CG solution v and
// the tracker's v~ (tv), and their stores (BUF, STAGE, FIXED_STORES above).
template <int W, typename ST, int M_BITS, bool BUF, bool STAGE = false, bool FIXED_STORES = false>
__device__ __forceinline__ void llr_stage(const DetectParams& prm, int64_t n, int s0,
                                          const float2 (&v)[W][4], const ST (&tv)[W][4],
                                          const float* Gs, int c, int g,
                                          float* __restrict__ stg = nullptr) {
  const int U = prm.U, S = prm.S;
  DetectStore<M_BITS> os;
  if (BUF || STAGE) os.init(prm, n);
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const int u = 16 * w + c;
    const float Guu = Gs[u < U ? u : 0];
    const float rho = Guu / prm.n0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int s = s0 + 4 * g + j;
      const float mu = (float)(tv[w][j] * (ST)Guu);
      const float2 x = v[w][j];
      // |mu| < FLT_MIN only when the right-hand side froze at (near) zero:
      // z = 0 as for b = 0.
      const float imu = fabsf(mu) >= __FLT_MIN__ ? __builtin_amdgcn_rcpf(mu) : 0.f;
      const float2 z = make_float2(x.x * imu, x.y * imu);
      float out[M_BITS];
      llr_maxlog<M_BITS>(z, rho, prm.scale, prm.inv_scale, out);
      if (STAGE) {
        if (u < U && s < S) {
          float* sp = stg + (u * S + s) * M_BITS;
#pragma unroll
          for (int q = 0; q < M_BITS; ++q) sp[q] = out[q];
        }
        if (!FIXED_STORES) os.store_aux((u < U && s < S) ? u * S + s : -1, x, mu, rho);
      } else if (BUF) {
        os.store((u < U && s < S) ? u * S + s : -1, out, x, mu, rho);
      } else if (u < U && s < S) {
        const size_t idx = ((size_t)n * U + u) * S + s;
        float* lp = prm.llr + idx * M_BITS;
#pragma unroll
        for (int q = 0; q < M_BITS; ++q) lp[q] = out[q];
        if (prm.xhat) prm.xhat[idx] = x;
        if (prm.mu) prm.mu[idx] = mu;
        if (prm.sinr) prm.sinr[idx] = rho;
      }
    }
  }
  if (STAGE) {
    wave_lds_sync();
    const int lane = 16 * g + c;
    const int total = U * S * M_BITS;             // floats, even (M_BITS is even)
    if constexpr (FIXED_STORES) {
      const float2* src = (const float2*)stg;
      const int np = total / 2;
#pragma unroll
      for (int i = 0; i < kStagedStores<W, M_BITS>; ++i) {
        const int o = i * kWave + lane;
        const float2 q = src[o < np ? o : 0];
        bstore2(os.llr, o < np ? (uint32_t)o * 8u : kOOB, q.x, q.y);
      }
    } else if ((total & 3) == 0) {                // 16-byte aligned tile
      const float4* src = (const float4*)stg;
      for (int o = lane; o < total / 4; o += kWave) {
        const float4 q = src[o];
        bstore4(os.llr, (uint32_t)o * 16u, q.x, q.y, q.z, q.w);
      }
    } else {
      const float2* src = (const float2*)stg;
      for (int o = lane; o < total / 2; o += kWave) {
        const float2 q = src[o];
        bstore2(os.llr, (uint32_t)o * 8u, q.x, q.y);
      }
    }
    wave_lds_sync();                              // stg is A / P of the next subcarrier
  }
}

// K iterations of Algorithm 1 with the tracker of eq. (13), then llr_stage
// for right-hand sides s0 + 4 g + j of subcarrier n.  A^T, d and G_ii come
// from the Gram phase, b = H^H y from acc.
template <int W, typename ST, int M_BITS, bool BUF, bool STAGE = false, bool FIXED_STORES = false,
          bool VALU = false>
__device__ __forceinline__ void cg_llr_epilogue(const DetectParams& prm, int64_t n, int s0,
                                                const GramAcc<W>& acc, const AOperand<W>& at,
                                                const float (&d)[W], const float* Gs,
                                                float2* Ps, int c, int g,
                                                float* __restrict__ stg = nullptr) {
  float2 b[W][4];
#pragma unroll
  for (int w = 0; w < W; ++w)
#pragma unroll
    for (int j = 0; j < 4; ++j) b[w][j] = make_float2(acc.dr[w][j], acc.di[w][j]);
  CGState<W, ST> st;
  cg_init<W, ST>(st, b);
  Tracker<W, ST> tk;
  tk.init();
  for (int k = 0; k < prm.K; ++k) {
    ST al[4], be[4];
    cg_step<W, ST, VALU>(st, at, Ps, c, g, al, be);
    tracker_step<W, ST>(tk, d, al, be);
  }
  llr_stage<W, ST, M_BITS, BUF, STAGE, FIXED_STORES>(prm, n, s0, st.v, tk.tv, Gs, c, g, stg);
}

// A cached Gram matrix (load_cached_gram) -> LDS A, A^T operand and
// diagonal d = A_ii, as gram_to_operands gives for a Gram formed here.
template <int W>
__device__ __forceinline__ void cached_gram_to_operands(const float2* Gn, int U, float reg,
                                                        float2* As, float* Gs, int ast, int c,
                                                        int g, AOperand<W>& at, float (&d)[W]) {
  load_cached_gram<W>(Gn, U, reg, As, Gs, ast, 16 * g + c);
  wave_lds_sync();
  at.load(As, ast, c, g, U);
#pragma unroll
  for (int w = 0; w < W; ++w) d[w] = As[(16 * w + c) * ast + 16 * w + c].x;
}

// Gram tiles -> LDS A, A^T operand and diagonal d = A_ii.
template <int W, typename IN>
__device__ __forceinline__ void gram_to_operands(IN tag, const GramAcc<W>& acc, float2* As,
                                                 float* Gs, float2* Ps, int ast, float reg, int U,
                                                 int c, int g, AOperand<W>& at, float (&d)[W]) {
  store_gram(tag, acc, As, Gs, (float*)Ps, ast, reg, c, g);
  wave_lds_sync();
  at.load(As, ast, c, g, U);
#pragma unroll
  for (int w = 0; w < W; ++w) d[w] = As[(16 * w + c) * ast + 16 * w + c].x;
}

}  // namespace mimo

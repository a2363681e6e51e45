// H-resident forms (U <= 16, S <= 16, B <= BMAX): a subcarrier's channel
// stays in registers from the Gram to the output contraction q = H_u v
// (Sec. III-D, Algorithm 1 output), so H crosses HBM once per subcarrier.
// Used by the resident precoder and by the uplink + downlink slot kernel.
//
// The registers hold the Gram's k-steps (complex64: lane (c, g) holds
// H[4 t + g][c] for k-step t; 16-bit: Re and Im of the eight antennas of
// block 4 t + g for user c), but the output contraction needs H[16 i + c]
// [4 t + g] in FP32, so each 16-antenna tile passes through the wave's LDS;
// the registers a k-step leaves receive the same k-step of the wave's next
// subcarrier, which is then in flight during the rest of the output stage
// (and, in the slot kernel, during the uplink CG that follows it).  Two LDS
// tile buffers alternate, so tile i + 1 is staged while tile i's MFMAs run.
// The 16 x S output tile is staged in LDS too, so that each store
// instruction writes 512 contiguous bytes.
#pragma once

#include "precode_out.hpp"

namespace mimo {

template <typename IN>
struct ResidentBlock;
template <>
struct ResidentBlock<InC32> {
  using type = BlockC32<1, 1>;    // one k-step: 4 antennas
};
template <>
struct ResidentBlock<InC32P> {
  using type = BlockC32P<1>;      // packed form (U <= 8)
};
template <>
struct ResidentBlock<InC32X3> {
  using type = BlockC32X3<1, 1>;  // one block: 16 antennas (bf16-split Gram)
};
template <>
struct ResidentBlock<InF16> {
  using type = Block16<1, h8, 1>;   // one k-step: 32 antennas
};
template <>
struct ResidentBlock<InBF16> {
  using type = Block16<1, bf8, 1>;
};

// Output tile i (antennas 16 i .. 16 i + 15) of the resident channel to LDS
// as Hs[antenna][slot] in FP32 (row stride kPST), user u in slot
// 4 (u % 4) + u / 4: the contraction's k-step t takes users 4 t + g, which
// then sit in the four adjacent slots 4 g .. 4 g + 3 of a row.
__device__ __forceinline__ int user_slot(int u) { return ((u & 3) << 2) | (u >> 2); }
// (Packed form: lanes c and c + 8 hold the same user c & 7, so slots of
// users 8..15 receive copies; the contraction never reads them for U <= 8.)
template <typename BLK, int NK>
__device__ __forceinline__ void stage_h_tile(const BLK (&hb)[NK], int i, float2* __restrict__ Hs,
                                             int c, int g) {
  const int sl = user_slot(c);
#pragma unroll
  for (int t = 0; t < 4; ++t) Hs[(4 * t + g) * kPST + sl] = hb[4 * i + t].h[0][0];
}
template <int NK>
__device__ __forceinline__ void stage_h_tile(const BlockC32X3<1, 1> (&hb)[NK], int i,
                                             float2* __restrict__ Hs, int c, int g) {
  const int sl = user_slot(c);
#pragma unroll
  for (int t = 0; t < 4; ++t) Hs[(4 * t + g) * kPST + sl] = hb[i].h[t][0];
}
template <int NK, typename V8>
__device__ __forceinline__ void stage_h_tile(const Block16<1, V8, 1> (&hb)[NK], int i,
                                             float2* __restrict__ Hs, int c, int g) {
  // k-step i / 2 holds blocks 4 (i / 2) + g; tile i is blocks 2 i and 2 i + 1
  if ((g >> 1) == (i & 1)) {
    const V8 re = hb[i >> 1].hr[0][0], im = hb[i >> 1].hi[0][0];
    const int sl = user_slot(c);
#pragma unroll
    for (int e = 0; e < 8; ++e)
      Hs[(8 * (g & 1) + e) * kPST + sl] = make_float2((float)re[e], (float)im[e]);
  }
}

// The resident forms read each byte of H once per launch: their loads of H
// take the non-temporal policy (nt) whatever the translation unit's default.
constexpr int kOnceCPol = 2;

// Output stage of the resident forms for subcarrier n, given the CG solution
// v (lane layout) of (G + beta I) v = t and the A^T operand `at` of that
// system (only its off-diagonal entries are used; Gs holds the raw diagonal
// G_uu):
//   ||q||^2 = v^H G v  (V staged in T1, qnorm2_lds),
//   q = H_u v on MFMA tile by tile from hb, P1 = Hr Vr, P2 = Hi Vi,
//   P3 = (Hr + Hi)(Vr + Vi), Re q = P1 - P2, Im q = P3 - P1 - P2,
//   scaled by 1 / ||q|| when normalizing, staged in Qs and stored,
// then qnorm.  Tile i goes through T0 (i even) or T1 (i odd); k-steps of
// hb receive the next subcarrier's channel (descriptor nxt) as soon as
// their tile is staged.  Qs, T0, T1: wave-private LDS of 16 x kPST complex
// each; Ns: 16 floats.
template <int BMAX, typename IN, typename ST, typename RB, int NK, typename Sub>
__device__ __forceinline__ void resident_output(const PrecodeParams& prm, int64_t n,
                                                RB (&hb)[NK], const Sub& nxt,
                                                const AOperand<1>& at, const float* Gs,
                                                const float2 (&vsol)[1][4], float2* Qs,
                                                float2* T0, float2* T1, float* Ns, int c, int g,
                                                int lane) {
  constexpr bool C32 = std::is_same<IN, InC32>::value || std::is_same<IN, InC32P>::value;
  constexpr bool X3 = std::is_same<IN, InC32X3>::value;    // one 16-antenna block per tile
  const int B = prm.B, U = prm.U, S = prm.S;
  // ---- ||q||^2 = v^H G v (V stays staged in T1)
  stage_vec<1>(T1, c, g, vsol);
  wave_lds_sync();
  qnorm2_lds<1, ST>(at, Gs, vsol, T1, Ns, c, g);
  wave_lds_sync();

  // ---- q = H_u v on MFMA with H from registers
  const float nrm2 = Ns[c];
  const float scl = prm.normalize ? (nrm2 > 0.f ? __builtin_amdgcn_rsqf(nrm2) : 0.f) : 1.0f;
  float2 vv[4];
  float vs[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    vv[t] = T1[(4 * t + g) * kPST + c];
    vs[t] = vv[t].x + vv[t].y;
  }
  const __amdgpu_buffer_rsrc_t rq = make_rsrc(prm.Q + (size_t)n * B * S, (uint32_t)B * S * 8u);
  // tile i is staged in buffer i % 2 (T0, T1) one tile ahead
  wave_lds_sync();
  stage_h_tile(hb, 0, T0, c, g);
  if (C32) {
#pragma unroll
    for (int t = 0; t < 4; ++t) hb[t].template load<false, kOnceCPol>(nxt, t * RB::ANT);
  } else if (X3) {
    hb[0].template load<false, kOnceCPol>(nxt, 0);
  }
#pragma unroll
  for (int i = 0; i < BMAX / 16; ++i) {
    float2* cur_t = (i & 1) ? T1 : T0;
    float2* nxt_t = (i & 1) ? T0 : T1;
    if (16 * i < B) {
      wave_lds_sync();
      float2 hv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) hv[t] = cur_t[c * kPST + 4 * g + t];   // user 4 t + g
      if (i + 1 < BMAX / 16 && 16 * (i + 1) < B) stage_h_tile(hb, i + 1, nxt_t, c, g);
      f4 p1 = zero4(), p2 = zero4(), p3 = zero4();
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (4 * t >= U) break;                        // users past U: v is zero
        p1 = mfma4(hv[t].x, vv[t].x, p1);
        p2 = mfma4(hv[t].y, vv[t].y, p2);
        p3 = mfma4(hv[t].x + hv[t].y, vs[t], p3);
      }
      const f4 qr = p1 - p2;
      const f4 qi = p3 - p1 - p2;
      if (c < S) {
#pragma unroll
        for (int j = 0; j < 4; ++j) Qs[(4 * g + j) * S + c] = make_float2(qr[j] * scl, qi[j] * scl);
      }
      wave_lds_sync();
      float2 q[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = 64 * r + lane;
        q[r] = Qs[e < 16 * S ? e : 0];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = 64 * r + lane;
        bstore2s(rq, e < 16 * S ? (uint32_t)e * 8u : kOOB, (uint32_t)(16 * i * S) * 8u, q[r].x,
                 q[r].y);
      }
    }
    // k-steps of tile i + 1 (now staged) receive the next subcarrier's
    if (C32) {
      if (i + 1 < BMAX / 16) {
#pragma unroll
        for (int t = 4 * (i + 1); t < 4 * (i + 1) + 4; ++t)
          hb[t].template load<false, kOnceCPol>(nxt, t * RB::ANT);
      }
    } else if (X3) {
      if (i + 1 < BMAX / 16) hb[i + 1].template load<false, kOnceCPol>(nxt, (i + 1) * RB::ANT);
    } else if (i & 1) {
      hb[i >> 1].template load<false, kOnceCPol>(nxt, (i >> 1) * RB::ANT);
    }
  }
  {
    const __amdgpu_buffer_rsrc_t rn =
        prm.qnorm ? make_rsrc(prm.qnorm + (size_t)n * S, (uint32_t)S * 4u) : make_rsrc(nullptr, 0u);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int ss = 4 * g + j;
      bstore1(rn, (c == 0 && ss < S) ? (uint32_t)ss * 4u : kOOB, sqrtf(Ns[ss]));
    }
  }
}

}  // namespace mimo

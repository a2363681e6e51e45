// CG-D detection, CG-P precoding and the standalone Gram and matched filter
// for 32 < U <= 64 (the paper's U <= B allows any U; Sec. II-A), complex64
// storage: one workgroup of four wavefronts per subcarrier.  Wavefront w takes role r = (w + n) mod 4 on
// subcarrier n and owns users 16 r .. 16 r + 15; the rotation spreads the
// roles' unequal Gram work evenly over the four SIMDs.
//
// Gram: the ten 16 x 16 tiles of the Hermitian G = H^H H are divided over
// the roles (r, r), (r, r + 1) and, for r < 2, (r, r + 2) (tile indices mod
// 4), each tile in three real products on MFMA, the channel streamed from
// HBM in groups of antennas with the next group in flight; role r also
// forms the matched filter b = H^H y of its users.  The tiles and their
// conjugate mirrors make A = G + reg I in LDS, whose rows 16 r .. come back
// as the A^T operand of the role's part of the mat-vec.  Per CG iteration
// (Algorithm 1 loop body) the wavefronts exchange P through a shared LDS
// array and the partial inner products Re(p^H e) and ||r||^2 of their users
// through a small LDS table, summed over the four roles in a fixed order, so
// every wavefront computes the same step sizes.  The approximate SINR
// tracker of eq. (13), mu, rho and the LLRs (eq. (4)) are per user and stay
// in the owning wavefront.  Precoding forms ||q||^2 = v^H G v the same way
// and then q = H_u v (Algorithm 1 output) with V from LDS, each wavefront
// taking every fourth 16-antenna tile.
#include <type_traits>

#include "detect_core.hpp"
#include "launch.hpp"
#include "precode_out.hpp"

namespace mimo {

constexpr int kWideTiles = 4;
constexpr int kWideUsers = 16 * kWideTiles;
constexpr int kWideAst = kWideUsers + 2;   // LDS row stride (complex) of A

template <typename ST>
struct WideLds {
  float2 A[kWideUsers * kWideAst];           // A = G + reg I, row-major
  float2 P[kWideUsers * kPST];               // P[user][rhs] of all users
  ST red[2][kWideTiles][16];                 // partial sums per role and rhs
  float G[kWideUsers];                       // raw diagonal G_uu
};

// After the Gram phase A's LDS holds each role's LLR tile (16 users x 16
// right-hand sides x up to 8 bits), or the precoder's 16 x 16 output tile.
static_assert(kWideTiles * 16 * 16 * 8 * sizeof(float) <= sizeof(float2) * kWideUsers * kWideAst,
              "LLR staging tiles must fit in A's LDS");

// Lane (c, g) of the wavefront in role r: user 16 r + c, right-hand sides
// s0 + 4 g + j.
struct WideLane {
  int r, c, g, lane;
};

// Accumulators of role r: Gram tiles (r, r + j) for j < 3 as P1 = ar br,
// P2 = ai bi, P3 = (ar + ai)(br - bi) over the row operand a (conjugated)
// and the column operand b, so that Re G = P1 + P2 and Im G = P1 - P2 - P3;
// and the matched filter of the role's users, Re b = p1 + p2,
// Im b = p3 - p1 + p2 with p3 = (yr + yi)(hr - hi).
struct WideAcc {
  f4 t[3][3];
  f4 p1, p2, p3;
};

// k-steps (4 antennas each) per load group: two groups are in registers
constexpr int kWideUnrDetect = 2;
constexpr int kWideUnrPrecode = 2;
// Cache policy of the Gram-phase loads of H and Y: the default one.  Two or
// three roles load each antenna row of H at different times, and the
// precoder reads H again for q = H v; marked non-temporal, lines left the
// caches before their other readers came (detection 1.11 vs 1.12 ms,
// precoding 1.38 vs 1.45 ms per 19,200 subcarriers of 128x64).
constexpr int kWideGramCPol = 0;

// One group of 4 UNR antennas: lane (c, g) holds H[b0 + 4 t + g][16 q_j + c]
// of the NH tiles q_j the role needs (q_0 = r) and Y[b0 + 4 t + g][s0 + c].
template <int NH, int UNR, bool DO_MF, int CPOL>
struct WideGroup {
  float2 h[UNR][NH];
  float2 y[UNR];
  __device__ __forceinline__ void load(__amdgpu_buffer_rsrc_t rh, const uint32_t (&oh)[3],
                                       __amdgpu_buffer_rsrc_t ry, uint32_t oy, int U, int S,
                                       int b0) {
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      const int b = b0 + 4 * t;
#pragma unroll
      for (int j = 0; j < NH; ++j) h[t][j] = bload2<CPOL>(rh, oh[j], (uint32_t)b * U * 8u);
      if (DO_MF) y[t] = bload2<CPOL>(ry, oy, (uint32_t)b * S * 8u);
    }
  }
  template <bool DO_GRAM>
  __device__ __forceinline__ void mma(WideAcc& acc) const {
#pragma unroll
    for (int t = 0; t < UNR; ++t) {
      const float2 a = h[t][0];
      const float da = a.x - a.y;
      if (DO_GRAM) {
        const float sa = a.x + a.y;
#pragma unroll
        for (int j = 0; j < NH; ++j) {
          const float2 b = h[t][j];
          const float db = j == 0 ? da : b.x - b.y;
          acc.t[j][0] = mfma4(a.x, b.x, acc.t[j][0]);
          acc.t[j][1] = mfma4(a.y, b.y, acc.t[j][1]);
          acc.t[j][2] = mfma4(sa, db, acc.t[j][2]);
        }
      }
      if (DO_MF) {
        acc.p1 = mfma4(y[t].x, a.x, acc.p1);
        acc.p2 = mfma4(y[t].y, a.y, acc.p2);
        acc.p3 = mfma4(y[t].x + y[t].y, da, acc.p3);
      }
    }
  }
};

// The antennas in groups of 4 UNR, the next group's loads in flight while
// the current group's MFMAs run.
template <int NH, int UNR, bool DO_GRAM, bool DO_MF, int CPOL>
__device__ __forceinline__ void wide_stream(__amdgpu_buffer_rsrc_t rh, const uint32_t (&oh)[3],
                                            __amdgpu_buffer_rsrc_t ry, uint32_t oy, int B, int U,
                                            int S, WideAcc& acc) {
  constexpr int GA = 4 * UNR;                      // antennas per group
  WideGroup<NH, UNR, DO_MF, CPOL> g0, g1;
  g0.load(rh, oh, ry, oy, U, S, 0);
  for (int b0 = 0; b0 < B; b0 += 2 * GA) {
    if (b0 + GA < B) g1.load(rh, oh, ry, oy, U, S, b0 + GA);
    g0.template mma<DO_GRAM>(acc);
    if (b0 + GA >= B) break;
    if (b0 + 2 * GA < B) g0.load(rh, oh, ry, oy, U, S, b0 + 2 * GA);
    g1.template mma<DO_GRAM>(acc);
  }
}

// Role r's Gram tiles (DO_GRAM) and matched filter for right-hand sides
// s0 .. s0 + 15 (DO_MF).  A role whose users are all padding (16 r >= U)
// has zero tiles and b.
template <int UNR, int CPOL, bool DO_GRAM, bool DO_MF>
__device__ __forceinline__ void wide_gram_mf(const void* Hn, const void* Yn, int B, int U, int S,
                                             int s0, const WideLane& L, WideAcc& acc) {
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int e = 0; e < 3; ++e) acc.t[j][e] = zero4();
  acc.p1 = acc.p2 = acc.p3 = zero4();
  if (16 * L.r >= U) return;
  const __amdgpu_buffer_rsrc_t rh = make_rsrc(Hn, (uint32_t)B * U * 8u);
  const __amdgpu_buffer_rsrc_t ry =
      make_rsrc(DO_MF ? Yn : Hn, DO_MF ? (uint32_t)B * S * 8u : 0u);
  uint32_t oh[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int u = 16 * ((L.r + j) & 3) + L.c;
    oh[j] = u < U ? (uint32_t)(L.g * U + u) * 8u : kOOB;
  }
  const int s = s0 + L.c;
  const uint32_t oy = s < S ? (uint32_t)(L.g * S + s) * 8u : kOOB;
  if (!DO_GRAM) wide_stream<1, UNR, false, DO_MF, CPOL>(rh, oh, ry, oy, B, U, S, acc);
  else if (L.r < 2) wide_stream<3, UNR, true, DO_MF, CPOL>(rh, oh, ry, oy, B, U, S, acc);
  else wide_stream<2, UNR, true, DO_MF, CPOL>(rh, oh, ry, oy, B, U, S, acc);
}

// Role r's tiles and their conjugate mirrors into A = G + reg I in LDS
// (diagonal tiles: the upper part, mirrored; the diagonal real, G_uu to
// lds.G), then the role's A^T operand a[t] = A[16 r + c][4 t + g] and
// d = A_uu.
template <typename ST>
__device__ __forceinline__ void wide_store_a(const WideAcc& acc, WideLds<ST>& lds, float reg,
                                             const WideLane& L, float2 (&a)[16], float& d) {
  const int nt = L.r < 2 ? 3 : 2;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (j < nt) {
      const int q = (L.r + j) & 3;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int i = 4 * L.g + jj;               // row within tile r
        const int row = 16 * L.r + i, col = 16 * q + L.c;
        const float p1 = acc.t[j][0][jj], p2 = acc.t[j][1][jj], p3 = acc.t[j][2][jj];
        const float re = p1 + p2, im = p1 - p2 - p3;
        if (j > 0 || i < L.c) {
          lds.A[row * kWideAst + col] = make_float2(re, im);
          lds.A[col * kWideAst + row] = make_float2(re, -im);
        } else if (i == L.c) {
          lds.A[row * kWideAst + row] = make_float2(re + reg, 0.f);
          lds.G[row] = re;
        }
      }
    }
  }
  __syncthreads();
  const float2* Ar = &lds.A[(16 * L.r + L.c) * kWideAst];
#pragma unroll
  for (int t = 0; t < 16; ++t) a[t] = Ar[4 * t + L.g];
  d = Ar[16 * L.r + L.c].x;
}

// Sum of the four roles' partial sums x[j] (rhs 4 g + j, the row sum of
// the role's users already taken) through lds.red[slot]: the same value, in
// the same order, in every wavefront.
template <typename ST>
__device__ __forceinline__ void wide_sum(ST (&x)[4], WideLds<ST>& lds, int slot,
                                         const WideLane& L) {
  if (L.c == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) lds.red[slot][L.r][4 * L.g + j] = x[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int s = 4 * L.g + j;
    x[j] = ((lds.red[slot][0][s] + lds.red[slot][1][s]) + lds.red[slot][2][s]) +
           lds.red[slot][3][s];
  }
}

// e = A p for the wavefront's users from P of all users in LDS (E^T = P^T
// A^T on MFMA, k over users; k-steps past U are zero and skipped).
__device__ __forceinline__ void wide_matvec(const float2 (&a)[16], const float2* Ps, int nk,
                                            const WideLane& L, float2 (&e)[4]) {
  f4 er = zero4(), ei = zero4();
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    if (t < nk) {                                    // wave-uniform
      const float2 pk = Ps[(4 * t + L.g) * kPST + L.c];
      er = mfma4(pk.x, a[t].x, er);
      ei = mfma4(pk.x, a[t].y, ei);
      er = mfma4(-pk.y, a[t].y, er);
      ei = mfma4(pk.y, a[t].x, ei);
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) e[j] = make_float2(er[j], ei[j]);
}

template <typename ST>
__device__ __forceinline__ void wide_stage(const float2 (&x)[4], float2* Ps, const WideLane& L) {
  float4* d = (float4*)&Ps[(16 * L.r + L.c) * kPST + 4 * L.g];
  d[0] = make_float4(x[0].x, x[0].y, x[1].x, x[1].y);
  d[1] = make_float4(x[2].x, x[2].y, x[3].x, x[3].y);
}

template <typename ST>
__device__ __forceinline__ void wide_cg_init(CGState<1, ST>& st, const float2 (&b)[4],
                                             WideLds<ST>& lds, const WideLane& L) {
  __syncthreads();                                   // last readers of lds.red and P are done
  ST part[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    part[j] = (ST)b[j].x * (ST)b[j].x + (ST)b[j].y * (ST)b[j].y;
    st.v[0][j] = make_float2(0.f, 0.f);
    st.r[0][j] = b[j];
    st.p[0][j] = b[j];
  }
  row_sum16_x4(part);
  wide_sum(part, lds, 1, L);
#pragma unroll
  for (int j = 0; j < 4; ++j) st.rr[j] = part[j];
}

// One iteration of Algorithm 1 over the four wavefronts of the subcarrier:
// the arithmetic of cg_update with the inner products summed over users of
// all roles.  Three barriers: P staged; Re(p^H e) and ||r||^2 exchanged (the
// last readers of P and of both tables passed one of them before the next
// write; wide_cg_init's barrier covers the first iteration).
template <typename ST>
__device__ __forceinline__ void wide_cg_step(CGState<1, ST>& st, const float2 (&a)[16], int nk,
                                             WideLds<ST>& lds, const WideLane& L,
                                             ST (&alpha)[4], ST (&beta)[4]) {
  wide_stage<ST>(st.p[0], lds.P, L);
  __syncthreads();
  float2 e[4];
  wide_matvec(a, lds.P, nk, L, e);
  ST pe[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
    pe[j] = (ST)st.p[0][j].x * (ST)e[j].x + (ST)st.p[0][j].y * (ST)e[j].y;
  row_sum16_x4(pe);
  wide_sum(pe, lds, 0, L);                           // Re(p^H e)
  bool live[4];
  ST rr_new[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    live[j] = live_floor<ST>(st.rr[j], pe[j]);
    alpha[j] = live[j] ? div_fast<ST>(st.rr[j], pe[j]) : ST(0);
    const float af = (float)alpha[j];
    st.v[0][j].x = __builtin_fmaf(af, st.p[0][j].x, st.v[0][j].x);
    st.v[0][j].y = __builtin_fmaf(af, st.p[0][j].y, st.v[0][j].y);
    st.r[0][j].x = __builtin_fmaf(-af, e[j].x, st.r[0][j].x);
    st.r[0][j].y = __builtin_fmaf(-af, e[j].y, st.r[0][j].y);
    rr_new[j] = (ST)st.r[0][j].x * (ST)st.r[0][j].x + (ST)st.r[0][j].y * (ST)st.r[0][j].y;
  }
  row_sum16_x4(rr_new);
  wide_sum(rr_new, lds, 1, L);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    beta[j] = live[j] ? div_fast<ST>(rr_new[j], st.rr[j]) : ST(0);
    const float bf = (float)beta[j];
    const float px = __builtin_fmaf(bf, st.p[0][j].x, st.r[0][j].x);
    const float py = __builtin_fmaf(bf, st.p[0][j].y, st.r[0][j].y);
    st.p[0][j].x = live[j] ? px : st.p[0][j].x;
    st.p[0][j].y = live[j] ? py : st.p[0][j].y;
    // (a conditional store rather than a select: the select of the two
    // array elements becomes a select of their addresses with FP64 scalars,
    // which keeps both arrays in scratch memory)
    if (live[j]) st.rr[j] = rr_new[j];
  }
}

// mu (eq. (14)), rho (eq. (15)), z = xhat / mu and the max-log LLRs (eq. (4))
// of the role's users for right-hand sides s0 + 4 g + j, and their stores
// (masked entries dropped by the descriptors' range check).  STAGE (one
// chunk of right-hand sides, S <= 16): the role's LLRs, 16 users x S x
// M_BITS floats contiguous in memory, are assembled in `stg` (LDS of the
// role, 16 x 16 x M_BITS floats) and written in 16- or 8-byte pieces, so
// every store instruction covers whole cache lines; scattered pieces would
// let partly written lines leave L2 and reach HBM more than once.
template <typename ST, int M_BITS, bool STAGE>
__device__ __forceinline__ void wide_llr(const DetectParams& prm, int64_t n, int s0,
                                         const float2 (&v)[4], const ST (&tv)[4], const float* Gs,
                                         const WideLane& L, float* __restrict__ stg) {
  const int U = prm.U, S = prm.S;
  DetectStore<M_BITS> os;
  os.init(prm, n);
  const int u = 16 * L.r + L.c;
  const bool uok = u < U;
  const float Guu = Gs[uok ? u : 0];
  const float rho = Guu / prm.n0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int s = s0 + 4 * L.g + j;
    const float mu = (float)(tv[j] * (ST)Guu);
    // |mu| < FLT_MIN only when the right-hand side froze at (near) zero
    const float imu = fabsf(mu) >= __FLT_MIN__ ? __builtin_amdgcn_rcpf(mu) : 0.f;
    const float2 z = make_float2(v[j].x * imu, v[j].y * imu);
    float out[M_BITS];
    llr_maxlog<M_BITS>(z, rho, prm.scale, prm.inv_scale, out);
    const int e = (uok && s < S) ? u * S + s : -1;
    if (STAGE) {
      if (e >= 0) {
        float* sp = stg + (L.c * S + s) * M_BITS;
#pragma unroll
        for (int q = 0; q < M_BITS; ++q) sp[q] = out[q];
      }
      os.store_aux(e, v[j], mu, rho);
    } else {
      os.store(e, out, v[j], mu, rho);
    }
  }
  if (STAGE) {
    wave_lds_sync();
    const int nu = U - 16 * L.r < 16 ? U - 16 * L.r : 16;    // >= 1: the role has users
    const int total = nu * S * M_BITS;                       // floats, even
    const uint32_t per = (uint32_t)(U * S * M_BITS);
    const __amdgpu_buffer_rsrc_t rl =
        make_rsrc(prm.llr + (size_t)n * per + (size_t)(16 * L.r) * S * M_BITS,
                  (uint32_t)total * 4u);
    if ((total & 3) == 0) {                                  // 16-byte pieces
      const float4* src = (const float4*)stg;
      for (int o = L.lane; o < total / 4; o += kWave) {
        const float4 q = src[o];
        bstore4(rl, (uint32_t)o * 16u, q.x, q.y, q.z, q.w);
      }
    } else {
      const float2* src = (const float2*)stg;
      for (int o = L.lane; o < total / 2; o += kWave) {
        const float2 q = src[o];
        bstore2(rl, (uint32_t)o * 8u, q.x, q.y);
      }
    }
  }
}

// Role of wavefront w on subcarrier n.
__device__ __forceinline__ WideLane wide_lane(int64_t n) {
  const int lane = threadIdx.x & 63;
  const int r = __builtin_amdgcn_readfirstlane((int)(((threadIdx.x >> 6) + n) & 3));
  return WideLane{r, lane & 15, lane >> 4, lane};
}

template <typename ST, int M_BITS>
__global__ __launch_bounds__(256, 2) void detect_wide_kernel(DetectParams kprm) {
  __shared__ __align__(16) WideLds<ST> lds;
  for (int64_t n = blockIdx.x; n < kprm.n_sc; n += gridDim.x) {
    const DetectParams prm = opaque_sizes(kprm);
    const int B = prm.B, U = prm.U, S = prm.S;
    const int nk = (U + 3) >> 2;
    const WideLane L = wide_lane(n);
    const void* Hn = offset_sc(InC32{}, prm.H, n, B, U);
    const void* Yn = offset_sc(InC32{}, prm.Y, n, B, S);
    float2 a[16];
    float d[1];
    for (int s0 = 0; s0 < S; s0 += 16) {
      WideAcc acc;
      if (s0 == 0) {
        wide_gram_mf<kWideUnrDetect, kWideGramCPol, true, true>(Hn, Yn, B, U, S, s0, L, acc);
        wide_store_a<ST>(acc, lds, prm.reg, L, a, d[0]);
      } else {
        wide_gram_mf<kWideUnrDetect, kWideGramCPol, false, true>(Hn, Yn, B, U, S, s0, L, acc);
      }
      float2 b[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float p1 = acc.p1[j], p2 = acc.p2[j];
        b[j] = make_float2(p1 + p2, acc.p3[j] - p1 + p2);
      }
      CGState<1, ST> st;
      wide_cg_init<ST>(st, b, lds, L);
      Tracker<1, ST> tk;
      tk.init();
      for (int k = 0; k < prm.K; ++k) {
        ST al[4], be[4];
        wide_cg_step<ST>(st, a, nk, lds, L, al, be);
        tracker_step<1, ST>(tk, d, al, be);
      }
      // the LLR tile of each role goes through its part of A's LDS (A is
      // in registers since the Gram phase; the CG's barriers follow every
      // read of it)
      if (16 * L.r < U) {
        float* stg = (float*)lds.A + L.r * (16 * 16 * M_BITS);
        if (S <= 16) wide_llr<ST, M_BITS, true>(prm, n, s0, st.v[0], tk.tv[0], lds.G, L, stg);
        else wide_llr<ST, M_BITS, false>(prm, n, s0, st.v[0], tk.tv[0], lds.G, L, stg);
      }
    }
    __syncthreads();                                 // LDS of this subcarrier read by all
  }
}

// H[b0 + c][4 t + g] for t < 16 (antenna row b0 + c, users 4 t + g): the
// A operand of q = H_u v over k-steps of 4 users.  Rows past B and users
// past U read as zero.
__device__ __forceinline__ void wide_load_hrows(__amdgpu_buffer_rsrc_t rh, int U, int b0,
                                                const WideLane& L, float2 (&h)[16]) {
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int u = 4 * t + L.g;
    h[t] = bload2(rh, u < U ? (uint32_t)(L.c * U + u) * 8u : kOOB, (uint32_t)b0 * U * 8u);
  }
}

template <typename ST>
__global__ __launch_bounds__(256, 2) void precode_wide_kernel(PrecodeParams kprm) {
  __shared__ __align__(16) WideLds<ST> lds;
  for (int64_t n = blockIdx.x; n < kprm.n_sc; n += gridDim.x) {
    const PrecodeParams prm = opaque_sizes(kprm);
    const int B = prm.B, U = prm.U, S = prm.S;
    const int nk = (U + 3) >> 2;
    const WideLane L = wide_lane(n);
    const int u = 16 * L.r + L.c;
    const void* Hn = offset_sc(InC32{}, prm.H, n, B, U);
    float2 a[16];
    float d;
    {
      WideAcc acc;
      wide_gram_mf<kWideUnrPrecode, kWideGramCPol, true, false>(Hn, nullptr, B, U, S, 0, L, acc);
      wide_store_a<ST>(acc, lds, prm.beta, L, a, d);
    }
    const __amdgpu_buffer_rsrc_t rh = make_rsrc(Hn, (uint32_t)B * U * 8u);
    const __amdgpu_buffer_rsrc_t rt =
        make_rsrc(prm.T + (size_t)n * U * S, (uint32_t)U * S * 8u);
    const __amdgpu_buffer_rsrc_t rq = make_rsrc(prm.Q + (size_t)n * B * S, (uint32_t)B * S * 8u);
    for (int s0 = 0; s0 < S; s0 += 16) {
      float2 b[4];                                   // b = t
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int s = s0 + 4 * L.g + j;
        b[j] = bload2(rt, (u < U && s < S) ? (uint32_t)(u * S + s) * 8u : kOOB, 0u);
      }
      CGState<1, ST> st;
      wide_cg_init<ST>(st, b, lds, L);
      for (int k = 0; k < prm.K; ++k) {
        ST al[4], be[4];
        wide_cg_step<ST>(st, a, nk, lds, L, al, be);
      }
      // ---- ||q||^2 = v^H G v over all users (the mat-vec on A's operand
      // with the diagonal entries replaced by G_uu, so beta never enters the
      // sum); V stays in LDS for q = H v.  The last CG iteration's barriers
      // follow every read of P.
      float2 hc[16];                                 // first antenna tile of q = H v
      const int bw = 16 * L.r;
      if (bw < B) wide_load_hrows(rh, U, bw, L, hc);
      wide_stage<ST>(st.v[0], lds.P, L);
      __syncthreads();
      float2 e[4];
      {
        float2 ga[16];
#pragma unroll
        for (int t = 0; t < 16; ++t)
          ga[t] = (u == 4 * t + L.g) ? make_float2(lds.G[u], 0.f) : a[t];
        wide_matvec(ga, lds.P, nk, L, e);
      }
      ST qq[4];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        qq[j] = (ST)st.v[0][j].x * (ST)e[j].x + (ST)st.v[0][j].y * (ST)e[j].y;
      row_sum16_x4(qq);
      wide_sum(qq, lds, 0, L);
      float nrm2[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) nrm2[j] = (float)(qq[j] > ST(0) ? qq[j] : ST(0));
      // ||q||^2 of rhs c = 4 g' + j' for the lanes of column c: lane
      // 16 g' + j' holds it in nrm2[j'] (every lane of a row holds its row's
      // four sums)
      const int jc = L.c & 3;
      const float mine = jc == 0 ? nrm2[0] : jc == 1 ? nrm2[1] : jc == 2 ? nrm2[2] : nrm2[3];
      const float nc = __shfl(mine, 16 * (L.c >> 2) + jc, 64);
      const float scl = prm.normalize ? (nc > 0.f ? __builtin_amdgcn_rsqf(nc) : 0.f) : 1.0f;
      // ---- q = H_u v (Algorithm 1 output): 16-antenna tiles 16 r, 16 r + 64,
      // ..., the next tile's loads in flight; P1 = Hr Vr, P2 = Hi Vi,
      // P3 = (Hr + Hi)(Vr + Vi), Re q = P1 - P2, Im q = P3 - P1 - P2
      float2 vv[16];
      float vs[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        vv[t] = lds.P[(4 * t + L.g) * kPST + L.c];
        vs[t] = vv[t].x + vv[t].y;
      }
      const int s = s0 + L.c;
      for (int b0 = bw; b0 < B; b0 += 16 * kWideTiles) {
        float2 hn[16];
        const int b1 = b0 + 16 * kWideTiles;
        if (b1 < B) wide_load_hrows(rh, U, b1, L, hn);
        f4 p1 = zero4(), p2 = zero4(), p3 = zero4();
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          if (t < nk) {                              // users 4 t .. exist
            p1 = mfma4(hc[t].x, vv[t].x, p1);
            p2 = mfma4(hc[t].y, vv[t].y, p2);
            p3 = mfma4(hc[t].x + hc[t].y, vs[t], p3);
          }
        }
        if (S <= 16) {
          // the tile's 16 x S outputs are contiguous in Q: staged in the
          // role's part of A's LDS (A is in registers since the Gram) and
          // written in 8-byte pieces, whole lines per store instruction;
          // rows past B fall outside the descriptor's range
          float2* Qs = lds.A + L.r * 256;
          if (s < S) {
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              const float qr = p1[jj] - p2[jj], qi = p3[jj] - p1[jj] - p2[jj];
              Qs[(4 * L.g + jj) * S + L.c] = make_float2(qr * scl, qi * scl);
            }
          }
          wave_lds_sync();
#pragma unroll
          for (int r4 = 0; r4 < 4; ++r4) {
            const int e = 64 * r4 + L.lane;
            const float2 q = Qs[e < 16 * S ? e : 0];
            bstore2s(rq, e < 16 * S ? (uint32_t)e * 8u : kOOB, (uint32_t)(b0 * S) * 8u, q.x, q.y);
          }
          wave_lds_sync();
        } else {
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const int bb = b0 + 4 * L.g + jj;
            const float qr = p1[jj] - p2[jj], qi = p3[jj] - p1[jj] - p2[jj];
            bstore2(rq, (bb < B && s < S) ? (uint32_t)(bb * S + s) * 8u : kOOB, qr * scl,
                    qi * scl);
          }
        }
        if (b1 < B) {
#pragma unroll
          for (int t = 0; t < 16; ++t) hc[t] = hn[t];
        }
      }
      if (prm.qnorm && L.r == 0 && L.c == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int ss = s0 + 4 * L.g + j;
          if (ss < S) prm.qnorm[(size_t)n * S + ss] = sqrtf(nrm2[j]);
        }
      }
    }
    __syncthreads();
  }
}

// Standalone A = G + reg I and b = H^H y (Algorithm 1, initialization) for
// 32 < U <= 64: the Gram and matched-filter phase of the kernels above, with
// A assembled in LDS and each role writing its rows of it.
template <bool HAS_Y>
__global__ __launch_bounds__(256, 2) void gram_mf_wide_kernel(GramParams kprm) {
  __shared__ __align__(16) WideLds<float> lds;
  for (int64_t n = blockIdx.x; n < kprm.n_sc; n += gridDim.x) {
    const GramParams prm = opaque_sizes(kprm);
    const int B = prm.B, U = prm.U, S = prm.S;
    const WideLane L = wide_lane(n);
    const void* Hn = offset_sc(InC32{}, prm.H, n, B, U);
    const void* Yn = HAS_Y ? offset_sc(InC32{}, prm.Y, n, B, S) : nullptr;
    const int nchunk = HAS_Y ? (S + 15) / 16 : 1;
    for (int ch = 0; ch < nchunk; ++ch) {
      const int s0 = 16 * ch;
      WideAcc acc;
      if (ch == 0) {
        wide_gram_mf<kWideUnrDetect, kWideGramCPol, true, HAS_Y>(Hn, Yn, B, U, S, s0, L, acc);
        float2 a[16];
        float d;
        wide_store_a<float>(acc, lds, prm.reg, L, a, d);   // the operand reads go unused
        float2* An = prm.A + (size_t)n * U * U;
        for (int idx = L.lane; idx < 16 * U; idx += kWave) {
          const int row = 16 * L.r + idx / U, col = idx % U;
          if (row < U) An[(size_t)row * U + col] = lds.A[row * kWideAst + col];
        }
      } else {
        wide_gram_mf<kWideUnrDetect, kWideGramCPol, false, HAS_Y>(Hn, Yn, B, U, S, s0, L, acc);
      }
      if (HAS_Y && prm.b) {
        const int u = 16 * L.r + L.c;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int s = s0 + 4 * L.g + j;
          const float p1 = acc.p1[j], p2 = acc.p2[j];
          if (u < U && s < S)
            prm.b[((size_t)n * U + u) * S + s] = make_float2(p1 + p2, acc.p3[j] - p1 + p2);
        }
      }
    }
    __syncthreads();                                 // A's LDS read by all
  }
}

// One workgroup per subcarrier, up to 2^20 workgroups walking the rest.
static unsigned int wide_grid(int64_t n_sc) {
  return (unsigned int)(n_sc < (1 << 20) ? (n_sc > 0 ? n_sc : 1) : (1 << 20));
}

template <typename ST>
static hipError_t launch_detect_wide_st(const DetectParams& p, int m_bits, hipStream_t stream) {
  const dim3 grid(wide_grid(p.n_sc)), block(kWave * kWideTiles);
  switch (m_bits) {
    case 2: hipLaunchKernelGGL((detect_wide_kernel<ST, 2>), grid, block, 0, stream, p); break;
    case 4: hipLaunchKernelGGL((detect_wide_kernel<ST, 4>), grid, block, 0, stream, p); break;
    case 6: hipLaunchKernelGGL((detect_wide_kernel<ST, 6>), grid, block, 0, stream, p); break;
    case 8: hipLaunchKernelGGL((detect_wide_kernel<ST, 8>), grid, block, 0, stream, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_detect_wide(const DetectParams& p, int scalar_f64, int m_bits,
                              hipStream_t stream) {
  return scalar_f64 ? launch_detect_wide_st<double>(p, m_bits, stream)
                    : launch_detect_wide_st<float>(p, m_bits, stream);
}

hipError_t launch_precode_wide(const PrecodeParams& p, int scalar_f64, hipStream_t stream) {
  const dim3 grid(wide_grid(p.n_sc)), block(kWave * kWideTiles);
  if (scalar_f64)
    hipLaunchKernelGGL((precode_wide_kernel<double>), grid, block, 0, stream, p);
  else
    hipLaunchKernelGGL((precode_wide_kernel<float>), grid, block, 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_gram_mf_wide(const GramParams& p, hipStream_t stream) {
  const dim3 grid(wide_grid(p.n_sc)), block(kWave * kWideTiles);
  if (p.Y)
    hipLaunchKernelGGL((gram_mf_wide_kernel<true>), grid, block, 0, stream, p);
  else
    hipLaunchKernelGGL((gram_mf_wide_kernel<false>), grid, block, 0, stream, p);
  return hipGetLastError();
}

}  // namespace mimo

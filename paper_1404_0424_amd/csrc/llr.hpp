// Max-log LLRs of eq. (4) for square Gray-labelled QAM.
//
// |z - a|^2 splits into an in-phase and a quadrature term; the term of the
// other axis is the same in both minima of eq. (4), so each bit needs only
// the L = 2^(m/2) levels of its own axis.  Levels are scale * (2 j - (L-1)),
// labelled by the Gray code j ^ (j >> 1), MSB first; in-phase bits first.
#pragma once

#include "common.hpp"

namespace mimo {

template <int M_BITS>
__device__ __forceinline__ void llr_maxlog(float2 z, float rho, float scale, float (&out)[M_BITS]) {
  constexpr int HB = M_BITS / 2;
  constexpr int L = 1 << HB;
#pragma unroll
  for (int axis = 0; axis < 2; ++axis) {
    const float comp = axis ? z.y : z.x;
    float m0[HB], m1[HB];
#pragma unroll
    for (int q = 0; q < HB; ++q) { m0[q] = __builtin_huge_valf(); m1[q] = __builtin_huge_valf(); }
#pragma unroll
    for (int jl = 0; jl < L; ++jl) {
      const float lev = scale * (float)(2 * jl - (L - 1));
      const float dlt = comp - lev;
      const float d = dlt * dlt;
      const int gray = jl ^ (jl >> 1);
#pragma unroll
      for (int q = 0; q < HB; ++q) {
        if ((gray >> (HB - 1 - q)) & 1) m1[q] = fminf(m1[q], d);
        else m0[q] = fminf(m0[q], d);
      }
    }
#pragma unroll
    for (int q = 0; q < HB; ++q) out[axis * HB + q] = rho * (m0[q] - m1[q]);
  }
}

}  // namespace mimo

// Max-log LLRs of eq. (4) for square Gray-labelled QAM.
//
// |z - a|^2 splits into an in-phase and a quadrature term; the term of the
// other axis is the same in both minima of eq. (4), so each bit needs only
// the L = 2^(m/2) levels of its own axis.  Levels are scale * (2 j - (L-1)),
// labelled by the Gray code j ^ (j >> 1), MSB first; in-phase bits first.
//
// In units of `scale` (zn = comp / scale, integer levels a_j) the distance
// is scale^2 ((zn - a_j)^2); zn^2 is common to both minima and drops out, so
// each level costs one FMA, a_j^2 - 2 a_j zn, with compile-time constants,
// and L = rho scale^2 (min_0 - min_1).
#pragma once

#include "common.hpp"

namespace mimo {

template <int M_BITS>
__device__ __forceinline__ void llr_maxlog(float2 z, float rho, float scale, float inv_scale,
                                           float (&out)[M_BITS]) {
  constexpr int HB = M_BITS / 2;
  constexpr int L = 1 << HB;
  const float kk = rho * scale * scale;
#pragma unroll
  for (int axis = 0; axis < 2; ++axis) {
    const float zn = (axis ? z.y : z.x) * inv_scale;
    float d[L];
#pragma unroll
    for (int jl = 0; jl < L; ++jl) {
      const float a = (float)(2 * jl - (L - 1));
      d[jl] = __builtin_fmaf(-2.0f * a, zn, a * a);
    }
#pragma unroll
    for (int q = 0; q < HB; ++q) {
      float m0 = __builtin_huge_valf(), m1 = __builtin_huge_valf();
#pragma unroll
      for (int jl = 0; jl < L; ++jl) {
        const int gray = jl ^ (jl >> 1);
        if ((gray >> (HB - 1 - q)) & 1) m1 = fminf(m1, d[jl]);
        else m0 = fminf(m0, d[jl]);
      }
      out[axis * HB + q] = kk * (m0 - m1);
    }
  }
}

}  // namespace mimo

// Host-side launchers of the library's kernels (C++ linkage, internal; the
// public entry points are in abi.hip).  Declarations only: each launcher
// is defined next to its kernels.
#pragma once

#include "kernels.hpp"

namespace mimo {

hipError_t launch_detect_approx(const DetectParams& p, int in_dtype, int scalar_f64, int m_bits,
                                const Schedule& sch, hipStream_t stream);
hipError_t launch_detect_exact(const DetectParams& p, int in_dtype, int scalar_f64, int m_bits,
                               hipStream_t stream);
hipError_t launch_precode(const PrecodeParams& p, int in_dtype, int scalar_f64,
                          const Schedule& sch, hipStream_t stream);
// LDS-ring detection (complex64, U <= 16, S <= 16, at least 3 chunks of 16 antennas,
// 16-byte aligned per-subcarrier arrays, LLRs only); other calls take
// stream-small.
bool detect_ring_eligible(const DetectParams& p, int in_dtype);
hipError_t launch_detect_ring(const DetectParams& p, int scalar_f64, int m_bits,
                              const Schedule& sch, hipStream_t stream);
// Split forms: four wavefronts per subcarrier, antenna quarters (complex64,
// U <= 32, S <= 16; precoding also B <= 256); other calls take the
// register-streaming kernels.
bool split_eligible(int in_dtype, int U, int S, int B, bool precode);
hipError_t launch_detect_split(const DetectParams& p, int scalar_f64, int m_bits,
                               const Schedule& sch, hipStream_t stream);
hipError_t launch_precode_split(const PrecodeParams& p, int scalar_f64, const Schedule& sch,
                                hipStream_t stream);
// Uplink + downlink slot in one H-resident kernel (complex64 or 16-bit
// storage, U <= 16, S <= 16 in both directions, B <= 128); other calls take
// two launches.
bool slot_eligible(const SlotParams& p, int in_dtype);
hipError_t launch_slot(const SlotParams& p, int in_dtype, int scalar_f64, int m_bits,
                       const Schedule& sch, hipStream_t stream);
// Four wavefronts per subcarrier, one 16-user tile each (complex64,
// 32 < U <= 64, approximate SINR; any B and S).
hipError_t launch_detect_wide(const DetectParams& p, int scalar_f64, int m_bits,
                              hipStream_t stream);
hipError_t launch_precode_wide(const PrecodeParams& p, int scalar_f64, hipStream_t stream);
hipError_t launch_gram_mf_wide(const GramParams& p, hipStream_t stream);
hipError_t launch_detect_plain(const DetectParams& p, int scalar_f64, int m_bits,
                               const Schedule& sch, hipStream_t stream);
hipError_t launch_detect_batch(const BatchArgs& a, int max_u, int in_dtype, int scalar_f64,
                               int m_bits, const Schedule& sch, hipStream_t stream);
hipError_t launch_precode_batch(const BatchArgs& a, int max_u, int in_dtype, int scalar_f64,
                                const Schedule& sch, hipStream_t stream);
// Comparison methods of Sec. III-F built on an explicit inverse of A.
enum { kInvCholesky = 0, kInvNeumann = 1 };
hipError_t launch_detect_inverse(const DetectParams& p, int method, int in_dtype, int m_bits,
                                 hipStream_t stream);
hipError_t launch_precode_inverse(const PrecodeParams& p, int method, int in_dtype,
                                  hipStream_t stream);
// CGLS on the augmented systems (Sec. III-E); dynamic LDS of the kernels.
size_t cgls_lds_bytes(int B, bool precode);
hipError_t launch_detect_cgls(const DetectParams& p, int in_dtype, int scalar_f64, int m_bits,
                              hipStream_t stream);
hipError_t launch_precode_cgls(const PrecodeParams& p, int in_dtype, int scalar_f64,
                               hipStream_t stream);
// Standalone Gram + matched filter: generic, or streaming (next block and
// next subcarrier in flight; S <= 16, larger S uses the generic kernel).
enum { kGramGeneric = 0, kGramStream = 1, kGramVariants = 2 };
hipError_t launch_gram_mf(const GramParams& p, int in_dtype, const Schedule& sch,
                          hipStream_t stream);
hipError_t launch_convert(const float2* src, uint16_t* dst, int dst_dtype, int64_t n, int R,
                          int C, hipStream_t stream);

// Sets the calling thread's mimo_last_error() message (abi.hip).
void set_last_error(const char* msg);

// Grid for one-wavefront-per-subcarrier kernels (4 waves per block); the
// kernels loop over subcarriers with a grid stride, so any n_sc is covered.
inline unsigned int wave_grid(int64_t n_sc) {
  int64_t blocks = (n_sc + 3) / 4;
  const int64_t cap = 1 << 20;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  return (unsigned int)blocks;
}

}  // namespace mimo

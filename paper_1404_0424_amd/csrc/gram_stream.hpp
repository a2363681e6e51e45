// Streaming Gram + matched filter of one subcarrier for kernels that walk
// several subcarriers per wavefront: two register blocks ping-pong, the next
// block's loads in flight while the current block's MFMAs run, and after the
// last block the first block of the next subcarrier is issued (from `nxt`,
// an empty descriptor after the last subcarrier), so it is in flight during
// the rest of the current subcarrier's work.  Loads are issued on every path,
// so each load-counter wait covers exactly the block consumed.  The MFMAs
// run in the same order as gram_mf (Algorithm 1, initialization).
#pragma once

#include "gram_phase.hpp"

namespace mimo {

// On entry `blk` holds block 0 of `cur` (loaded or in flight); on return it
// holds block 0 of `nxt`.  The matched filter is finished when DO_MF.
template <int W, bool DO_MF, typename IN, typename Sub, typename Blk>
__device__ __forceinline__ void gram_stream(IN tag, Blk& blk, const Sub& cur, const Sub& nxt,
                                            int B, GramAcc<W>& acc) {
  Blk alt;
  // pairs of blocks; an odd count's last partner lies past B and reads
  // zero, adding exact zeros (one loop exit, so nothing after the Gram
  // waits for the next subcarrier's block in flight)
  for (int b0 = 0;; b0 += 2 * Blk::ANT) {
    alt.template load<DO_MF>(cur, b0 + Blk::ANT);
    blk.template mma<true, DO_MF>(acc);
    const bool more2 = b0 + 2 * Blk::ANT < B;
    blk.template load<DO_MF>(more2 ? cur : nxt, more2 ? b0 + 2 * Blk::ANT : 0);
    alt.template mma<true, DO_MF>(acc);
    if (!more2) break;
  }
  if (DO_MF) finish_mf(tag, acc);
}

}  // namespace mimo

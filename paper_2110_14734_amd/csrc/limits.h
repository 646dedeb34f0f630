// Host-side size limits of the WSPD work list (internal, header-only so that
// a plain C++ test can check them without a GPU).
#pragma once

#include <cstdint>

namespace w1 {

// An expansion round classifies f frontier items and sums, in one 64-bit
// scan word per item, the kept count (low 32 bits, at most f) and the grown
// count (high 32 bits, at most 2 f).  Both sums fit when f < 2^31.
inline bool worklist_round_fits(int64_t frontier) { return frontier >= 0 && frontier < (int64_t(1) << 31); }

// The final work list is indexed by int32 in the chunk table and in the
// persistent passes, and sorted with a u32 permutation: fewer than 2^31
// items.
inline bool worklist_items_fit(int64_t items) { return items >= 0 && items < (int64_t(1) << 31); }

// Chunks of the persistent passes are numbered by int32.
inline bool worklist_chunks_fit(int64_t chunks) { return chunks >= 0 && chunks < (int64_t(1) << 31); }

}  // namespace w1

// Host-side size limits of the WSPD work list and of the network's sorted
// row form (internal, header-only so that a plain C++ test can check them
// without a GPU).
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

// Slotted emission (short work lists on the network path, no count pass):
// at most this many record slots over all chunks (12 bytes each at most).
constexpr int64_t kSlottedMaxRecords = int64_t(1) << 25;

// Geometry of the partition passes that sort the network into rows: buckets
// of 2^RB consecutive cells (RB in 9..12, the smallest giving at most 1024
// buckets over the launch group's n_cells), entries of 32 bits holding the
// tail within its bucket (RB bits) and the head (DB bits, enough for every
// local node id below the largest pair's cell count).  The network can be
// built when there are at most 1024 buckets (at most 2^22 cells in a launch
// group) and RB + DB <= 32.
struct CsrGeometry {
  int RB, DB;
  int64_t NB;
  bool ok;
};
inline CsrGeometry csr_geometry(int64_t n_cells, int64_t max_pair_cells) {
  CsrGeometry g{9, 1, 0, false};
  while ((int64_t(1) << g.DB) < max_pair_cells) ++g.DB;
  while (g.RB < 12 && ((n_cells + (int64_t(1) << g.RB) - 1) >> g.RB) > 1024) ++g.RB;
  g.NB = (n_cells + (int64_t(1) << g.RB) - 1) >> g.RB;
  g.ok = n_cells >= 0 && g.NB <= 1024 && g.RB + g.DB <= 32;
  return g;
}

}  // namespace w1

// Host network simplex (internal).
#pragma once

#include <cstdint>

namespace w1 {

struct FlowResult {
  int64_t cost;
  int64_t pivots;
  int status;       // 0 optimal, 1 pivot cap reached
  int64_t* flow;    // optional, m entries
  int64_t* pot;     // optional, n entries
};

// Returns 0, -1 (infeasible / invalid) or -3 (out of memory).
int network_simplex(int64_t n_nodes, int64_t m, const uint32_t* src, const uint32_t* dst, const int32_t* cost,
                    const int64_t* supply, int64_t pivot_cap, FlowResult* out);

}  // namespace w1

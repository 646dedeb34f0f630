// Host network simplex (internal).
#pragma once

#include <cstdint>
#include <vector>

namespace w1 {

struct FlowResult {
  int64_t cost;     // flow cost, -1 when no feasible flow was reached
  int64_t pivots;
  int status;       // 0 optimal, 1 pivot cap reached
  int feasible;     // 1 when the returned flow meets every supply
  int64_t* flow;    // optional, m entries
  int64_t* pot;     // optional, n entries
};

// Network in CSR form: the arcs of node v are row_ptr[v] .. row_ptr[v+1]-1,
// with heads col[] and costs cost[]; m = row_ptr[n_nodes].
// Returns 0, -1 (infeasible / invalid) or -3 (out of memory).
int network_simplex(int64_t n_nodes, const int64_t* row_ptr, const uint32_t* col, const int32_t* cost,
                    const int64_t* supply, int64_t pivot_cap, FlowResult* out);

// The same with 64-bit costs (the Euclidean network); the largest cost times
// (n_nodes + 1) must be below 2^60.
int network_simplex64(int64_t n_nodes, const int64_t* row_ptr, const uint32_t* col, const int64_t* cost,
                      const int64_t* supply, int64_t pivot_cap, FlowResult* out);

// The same for the method's transshipment networks (nodes n_nodes - 2 and
// n_nodes - 1 the diagonal nodes of A and B, rows sorted by head): the
// start tree is the flow through the diagonal (every surplus to A's
// diagonal node, every deficit from B's), so the solve starts feasible.
// The optimum is the same as network_simplex's.
int network_simplex_diag(int64_t n_nodes, const int64_t* row_ptr, const uint32_t* col, const int32_t* cost,
                         const int64_t* supply, int64_t pivot_cap, FlowResult* out);
int network_simplex64_diag(int64_t n_nodes, const int64_t* row_ptr, const uint32_t* col, const int64_t* cost,
                           const int64_t* supply, int64_t pivot_cap, FlowResult* out);

// The same for an arc list (src, dst, cost); flow entries follow the list.
int network_simplex_arcs(int64_t n_nodes, int64_t m, const uint32_t* src, const uint32_t* dst, const int32_t* cost,
                         const int64_t* supply, int64_t pivot_cap, FlowResult* out);

// Rows of one of the method's networks (cells 0 .. n_cells - 1 with grid
// coordinates (ci, cj), then the A- and B-diagonal nodes) without the cell
// arcs that some optimal flow never uses; the optimum is the whole network's.
// cost_shift = -1 marks integer L-infinity costs (units g/2); >= 0 the
// Euclidean costs in units of g 2^-cost_shift.
template <typename C>
struct SolveRows {
  std::vector<int64_t> row_ptr;
  std::vector<uint32_t> col;
  std::vector<C> cost;
};
void drop_dominated_arcs(int64_t n_cells, const int64_t* row_ptr, const uint32_t* col, const int32_t* cost,
                         const int32_t* ci, const int32_t* cj, int cost_shift, SolveRows<int32_t>& out);
void drop_dominated_arcs(int64_t n_cells, const int64_t* row_ptr, const uint32_t* col, const int64_t* cost,
                         const int32_t* ci, const int32_t* cj, int cost_shift, SolveRows<int64_t>& out);

}  // namespace w1

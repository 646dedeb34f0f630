// Host min-cost flow of the sparse transshipment network: primal network
// simplex for uncapacitated networks with integer costs (Sec. 5.4).
//
//  * Basis: a spanning tree rooted at an artificial node; the start tree
//    links every node to the root with an artificial arc of cost larger than
//    any simple path, oriented so the tree is strongly feasible (zero-flow
//    tree arcs point away from the root).
//  * Entering arc: block search pivot rule (the paper's choice): arcs are
//    scanned cyclically in blocks of about sqrt(m) / 4; the most negative
//    reduced cost of the first block that has one enters.  Pricing dominates
//    on these networks (few nodes, many arcs), and the shorter blocks price
//    fewer arcs per pivot: 1.6-1.8x faster than sqrt(m) blocks here, with more
//    pivots.  The optimal cost does not depend on the block size.
//  * Leaving arc: the last blocking arc met when the pivot cycle is traversed
//    in the direction of the entering arc starting at the apex; this keeps
//    every basis strongly feasible, so degenerate pivots cannot cycle (this
//    takes over the job of the paper's random jitter, which it used against
//    stalling).
//  * Arcs come as a CSR network (row_ptr, col, cost): the arcs of a row
//    share their tail, so pricing reads one potential per row and one per
//    arc, over runs that do not wrap past the last arc, with branch-free
//    running minima.  The tail of a single arc (a tree arc after a pivot)
//    is found by binary search in row_ptr.
//  * Arc numbers are int64 throughout (network arcs 0..m-1, the artificial
//    arc of node v is m + v), so m is limited by memory only; node numbers
//    are int32.
//  * Tree storage: parent, predecessor arc, depth and doubly linked child
//    lists; after a pivot the detached subtree is re-rooted along the path to
//    the entering arc and its potentials and depths are shifted by a
//    preorder walk of the child lists (no stack).
//  * Flow: without capacities every non-tree arc carries zero flow, so the
//    flow is kept per node, on its predecessor arc.  The pivot's cycle walk
//    then touches node arrays only, not the m-arc arrays; arc flows are
//    formed once at the end.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "flow.h"

namespace w1 {

namespace {

// Most negative reduced cost c[b] + pit - pi[h[b]] over arcs b in [a, end)
// of one row (tail potential pit) that is below *best; on success *best and
// *enter take the value and the first arc that reaches it.  Two running
// minima (even and odd offsets) halve the dependent chain; they merge by
// value, then by the earlier arc, so the pick is the one of a single scan.
template <typename C>
void price_run(const int32_t* h, const C* c, const int64_t* pi, int64_t pit, int64_t a, int64_t end,
               int64_t* best, int64_t* enter) {
  int64_t sv = *best, si = -1, sv1 = *best, si1 = -1;
  int64_t b = a;
  for (; b + 2 <= end; b += 2) {
    const int64_t r0 = (int64_t)c[b] + pit - pi[h[b]];
    const int64_t r1 = (int64_t)c[b + 1] + pit - pi[h[b + 1]];
    const bool l0 = r0 < sv, l1 = r1 < sv1;
    sv = l0 ? r0 : sv;
    si = l0 ? b : si;
    sv1 = l1 ? r1 : sv1;
    si1 = l1 ? b + 1 : si1;
  }
  if (si1 >= 0 && (sv1 < sv || (sv1 == sv && (si < 0 || si1 < si)))) {
    sv = sv1;
    si = si1;
  }
  for (; b < end; ++b) {
    const int64_t r = (int64_t)c[b] + pit - pi[h[b]];
    const bool lt = r < sv;
    sv = lt ? r : sv;
    si = lt ? b : si;
  }
  if (si >= 0) {
    *best = sv;
    *enter = si;
  }
}

// Row of arc a: the last r with row_ptr[r] <= a (a < row_ptr[n]).
int32_t row_of(const int64_t* row_ptr, int32_t n, int64_t a) {
  return (int32_t)(std::upper_bound(row_ptr, row_ptr + n + 1, a) - row_ptr) - 1;
}

// Prices the arcs [a, end) row by row, starting in row *r (which holds a).
template <typename C>
void price_range(const int64_t* row_ptr, const int32_t* h, const C* c, const int64_t* pi, int32_t* r,
                 int64_t a, int64_t end, int64_t* best, int64_t* enter) {
  while (a < end) {
    while (row_ptr[*r + 1] <= a) ++*r;
    const int64_t e = std::min(end, row_ptr[*r + 1]);
    price_run(h, c, pi, pi[*r], a, e, best, enter);
    a = e;
  }
}

struct Simplex {
  int32_t n = 0, root = 0;
  int64_t m = 0;
  // Network arcs 0..m-1 are read in place from the caller's CSR arrays; the
  // artificial arc m + v joins v and the root, leaving v when art_out[v].
  const int64_t* row_ptr = nullptr;
  const int32_t* col = nullptr;
  std::vector<uint8_t> art_out;
  int32_t tail(int64_t a) const { return a < m ? row_of(row_ptr, n, a) : (art_out[a - m] ? (int32_t)(a - m) : root); }
  std::vector<int64_t> tflow;  // flow on pred[v], per node
  std::vector<int64_t> pred;   // tree arc joining v to its parent
  std::vector<int32_t> parent, depth, first_child, next_sib, prev_sib;
  std::vector<uint8_t> up;  // pred arc runs node -> parent
  std::vector<int64_t> pi;
  std::vector<int32_t> path;

  void unlink(int32_t x) {
    const int32_t p = parent[x];
    if (prev_sib[x] >= 0) next_sib[prev_sib[x]] = next_sib[x];
    else first_child[p] = next_sib[x];
    if (next_sib[x] >= 0) prev_sib[next_sib[x]] = prev_sib[x];
    next_sib[x] = prev_sib[x] = -1;
  }
  void link(int32_t x, int32_t p) {
    parent[x] = p;
    prev_sib[x] = -1;
    next_sib[x] = first_child[p];
    if (first_child[p] >= 0) prev_sib[first_child[p]] = x;
    first_child[p] = x;
  }
};

// The solver for either cost width: int32 (L-infinity costs in units of
// g/2) or int64 (Euclidean costs in units of g 2^-K, scaled so that the
// artificial cost (max cost + 1)(n + 1) stays below 2^60 and every reduced
// cost fits int64).
// Arc u -> w of a row sorted by head, or -1.
int64_t find_arc(const int64_t* row_ptr, const int32_t* col, int32_t u, int32_t w) {
  const int32_t* b = col + row_ptr[u];
  const int32_t* e = col + row_ptr[u + 1];
  const int32_t* f = std::lower_bound(b, e, w);
  return f != e && *f == w ? (int64_t)(f - col) : -1;
}

// diag_a / diag_b >= 0: the network is a transshipment network whose nodes
// diag_a and diag_b are the diagonal nodes of A and B, with rows sorted by
// head.  The start tree is then the flow that sends every node's surplus
// to diag_a and takes every deficit from diag_b (the diagonal arcs), with
// diag_b -> diag_a carrying the rest, instead of artificial arcs only; if
// an arc it needs is missing, the artificial start is used.
template <typename C>
int simplex(int64_t n_nodes, const int64_t* row_ptr, const uint32_t* col, const C* cost, const int64_t* supply,
            int64_t pivot_cap, FlowResult* out, int32_t diag_a = -1, int32_t diag_b = -1) {
  out->cost = -1;
  out->pivots = 0;
  out->status = 0;
  out->feasible = 0;
  if (n_nodes < 0 || n_nodes >= (int64_t(1) << 31) - 1 || !row_ptr || (n_nodes > 0 && !supply)) return -1;
  const int32_t n = (int32_t)n_nodes;
  if (row_ptr[0] != 0) return -1;
  for (int32_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) return -1;
  const int64_t m = row_ptr[n];
  if (m > 0 && (!col || !cost)) return -1;
  int64_t total = 0;
  for (int32_t v = 0; v < n; ++v) total += supply[v];
  if (total != 0) return -1;
  int64_t maxc = 0;
  for (int64_t a = 0; a < m; ++a) {
    if (cost[a] < 0 || col[a] >= (uint64_t)n_nodes) return -1;
    maxc = std::max<int64_t>(maxc, (int64_t)cost[a]);
  }
  if (maxc >= ((int64_t)1 << 60) / ((int64_t)n + 1)) return -1;  // the artificial cost must stay below 2^60
  Simplex S;
  S.n = n;
  S.root = n;
  S.m = m;
  S.row_ptr = row_ptr;
  // Node indices are below 2^31 - 1 (checked above), so the unsigned arc
  // heads read as int32 unchanged.
  S.col = reinterpret_cast<const int32_t*>(col);
  try {
    S.art_out.assign((size_t)n, 0);
    S.tflow.assign((size_t)n + 1, 0);
    S.parent.assign((size_t)n + 1, -1);
    S.pred.assign((size_t)n + 1, -1);
    S.depth.assign((size_t)n + 1, 0);
    S.first_child.assign((size_t)n + 1, -1);
    S.next_sib.assign((size_t)n + 1, -1);
    S.prev_sib.assign((size_t)n + 1, -1);
    S.up.assign((size_t)n + 1, 0);
    S.pi.assign((size_t)n + 1, 0);
  } catch (...) {
    return -3;
  }
  const int64_t ART = (maxc + 1) * ((int64_t)n + 1);
  // warm start from the diagonal flow (see above): the arcs each node needs
  std::vector<int64_t> warm;
  int64_t x_ba = 0, e_ba = -1;
  if (diag_a >= 0 && diag_b >= 0 && diag_a < n && diag_b < n && diag_a != diag_b && supply[diag_a] <= 0 &&
      supply[diag_b] >= 0) {
    try {
      warm.assign((size_t)n, -1);
    } catch (...) {
      return -3;
    }
    bool ok = true;
    x_ba = supply[diag_b];
    for (int32_t v = 0; v < n && ok; ++v) {
      if (v == diag_a || v == diag_b) continue;
      if (supply[v] > 0) {
        warm[(size_t)v] = find_arc(row_ptr, S.col, v, diag_a);
        ok = warm[(size_t)v] >= 0;
      } else {
        warm[(size_t)v] = find_arc(row_ptr, S.col, diag_b, v);  // may be absent for a node without supply
        ok = supply[v] == 0 || warm[(size_t)v] >= 0;
        x_ba += supply[v];
      }
    }
    if (ok && x_ba > 0) {
      e_ba = find_arc(row_ptr, S.col, diag_b, diag_a);
      ok = e_ba >= 0;
    }
    if (!ok || x_ba < 0) warm.clear();
  }
  if (!warm.empty()) {
    // strongly feasible: every zero-flow tree arc leaves the root's side
    auto art_down = [&](int32_t v) {  // artificial root -> v, no flow
      S.art_out[v] = 0;
      S.pred[v] = m + v;
      S.tflow[v] = 0;
      S.up[v] = 0;
      S.pi[v] = ART;
      S.depth[v] = 1;
      S.link(v, S.root);
    };
    art_down(diag_a);
    if (x_ba > 0) {
      S.pred[diag_b] = e_ba;
      S.tflow[diag_b] = x_ba;
      S.up[diag_b] = 1;
      S.pi[diag_b] = S.pi[diag_a] - (int64_t)cost[e_ba];
      S.depth[diag_b] = 2;
      S.link(diag_b, diag_a);
    } else {
      art_down(diag_b);
    }
    for (int32_t v = 0; v < n; ++v) {
      if (v == diag_a || v == diag_b) continue;
      const int64_t e = warm[(size_t)v];
      if (supply[v] > 0) {  // v -> diag_a carries the surplus
        S.pred[v] = e;
        S.tflow[v] = supply[v];
        S.up[v] = 1;
        S.pi[v] = S.pi[diag_a] - (int64_t)cost[e];
        S.depth[v] = S.depth[diag_a] + 1;
        S.link(v, diag_a);
      } else if (e >= 0) {  // diag_b -> v carries the deficit (or nothing)
        S.pred[v] = e;
        S.tflow[v] = -supply[v];
        S.up[v] = 0;
        S.pi[v] = S.pi[diag_b] + (int64_t)cost[e];
        S.depth[v] = S.depth[diag_b] + 1;
        S.link(v, diag_b);
      } else {
        art_down(v);
      }
    }
  }
  for (int32_t v = 0; v < n && warm.empty(); ++v) {
    if (supply[v] > 0) {
      S.art_out[v] = 1;
      S.tflow[v] = supply[v];
      S.up[v] = 1;
      S.pi[v] = -ART;
    } else {
      S.tflow[v] = -supply[v];
      S.up[v] = 0;
      S.pi[v] = ART;
    }
    S.pred[v] = m + v;
    S.depth[v] = 1;
    S.link(v, S.root);
  }

  const int64_t block = std::max<int64_t>(10, (int64_t)(0.25 * std::sqrt((double)std::max<int64_t>(m, 1))));
  int64_t next_arc = 0;
  int32_t next_row = 0;  // row holding next_arc
  int64_t pivots = 0;
  int status = 0;
  for (;;) {
    // ---- entering arc: block search.  Tree arcs have reduced cost exactly 0
    // (integer potentials), so they never enter and need no test.
    int64_t enter = -1, best = 0;
    int32_t k = -1;
    if (m > 0) {
      const int64_t* pi = S.pi.data();
      int64_t a = next_arc, scanned = 0;
      int32_t r = next_row;
      while (scanned < m) {
        // One block, split where it wraps past the last arc; the part before
        // the wrap comes first in scan order, so it wins ties.
        const int64_t len = std::min(block, m - scanned);
        const int64_t end1 = std::min(m, a + len);
        price_range(row_ptr, S.col, cost, pi, &r, a, end1, &best, &enter);
        if (a + len > m) {
          r = 0;
          price_range(row_ptr, S.col, cost, pi, &r, 0, a + len - m, &best, &enter);
          a = a + len - m;
        } else {
          a = end1;
          if (a == m) {
            a = 0;
            r = 0;
          }
        }
        scanned += len;
        if (enter >= 0) break;
      }
      next_arc = a;
      next_row = r;
    }
    if (enter < 0) break;
    if (pivot_cap > 0 && pivots >= pivot_cap) {
      status = 1;
      break;
    }
    ++pivots;
    k = row_of(row_ptr, n, enter);
    const int32_t l = S.col[enter];
    // ---- apex
    int32_t x = k, y = l;
    while (S.depth[x] > S.depth[y]) x = S.parent[x];
    while (S.depth[y] > S.depth[x]) y = S.parent[y];
    while (x != y) {
      x = S.parent[x];
      y = S.parent[y];
    }
    const int32_t apex = x;
    // ---- leaving arc (last blocking arc from the apex along k -> l)
    const int64_t INF = INT64_MAX;
    int64_t delta = INF;
    int32_t leave_node = -1;
    bool leave_on_k = false;
    for (int32_t v = k; v != apex; v = S.parent[v])
      if (S.up[v] && S.tflow[v] < delta) {
        delta = S.tflow[v];
        leave_node = v;
        leave_on_k = true;
      }
    for (int32_t v = l; v != apex; v = S.parent[v])
      if (!S.up[v] && S.tflow[v] <= delta) {
        delta = S.tflow[v];
        leave_node = v;
        leave_on_k = false;
      }
    if (leave_node < 0) return -1;  // unbounded: impossible with non-negative costs
    // ---- flow update
    if (delta > 0) {
      for (int32_t v = k; v != apex; v = S.parent[v]) S.tflow[v] += S.up[v] ? -delta : delta;
      for (int32_t v = l; v != apex; v = S.parent[v]) S.tflow[v] += S.up[v] ? delta : -delta;
    }
    // ---- tree update: detach the subtree at leave_node, re-root it at the
    // entering arc's endpoint inside it, hang it below the other endpoint.
    const int32_t u_in = leave_on_k ? k : l, v_in = leave_on_k ? l : k;
    S.path.clear();
    for (int32_t v = u_in;; v = S.parent[v]) {
      S.path.push_back(v);
      if (v == leave_node) break;
    }
    for (int32_t v : S.path) S.unlink(v);
    // Each path node takes over its predecessor's tree arc and that arc's
    // flow; the first takes the entering arc, which now carries delta, and
    // the leaving arc (flow 0) drops out.  The first node's tail test uses
    // the entering arc's known tail.
    int32_t new_parent = v_in;
    int64_t new_pred = enter, new_flow = delta;
    for (size_t i = 0; i < S.path.size(); ++i) {
      const int32_t v = S.path[i];
      const int64_t old_pred = S.pred[v], old_flow = S.tflow[v];
      S.link(v, new_parent);
      S.pred[v] = new_pred;
      S.tflow[v] = new_flow;
      S.up[v] = (i == 0 ? k : S.tail(new_pred)) == v ? 1 : 0;
      new_parent = v;
      new_pred = old_pred;
      new_flow = old_flow;
    }
    const int64_t dpi = leave_on_k ? -best : best;
    for (int32_t v = u_in;;) {
      S.pi[v] += dpi;
      S.depth[v] = S.depth[S.parent[v]] + 1;
      if (S.first_child[v] >= 0) {
        v = S.first_child[v];
        continue;
      }
      while (v != u_in && S.next_sib[v] < 0) v = S.parent[v];
      if (v == u_in) break;
      v = S.next_sib[v];
    }
  }
  out->pivots = pivots;
  out->status = status;
  // Flow cost over the network arcs.  A stalled solve may leave supply on
  // artificial arcs: its network flow is then not feasible, and no cost is
  // reported for it (feasible = 0, cost = -1).
  int64_t c = 0;
  bool feasible = true;
  for (int32_t v = 0; v < n; ++v) {
    const int64_t a = S.pred[v];
    if (a < m) c += (int64_t)cost[a] * S.tflow[v];
    else if (S.tflow[v] != 0) feasible = false;
  }
  if (!feasible && status == 0) return -1;  // supplies cannot be routed
  out->feasible = feasible ? 1 : 0;
  out->cost = feasible ? c : -1;
  if (out->flow) {
    std::fill(out->flow, out->flow + m, int64_t(0));
    for (int32_t v = 0; v < n; ++v)
      if (S.pred[v] < m) out->flow[S.pred[v]] = S.tflow[v];
  }
  if (out->pot) std::copy(S.pi.begin(), S.pi.begin() + n, out->pot);
  return 0;
}

}  // namespace

int network_simplex(int64_t n_nodes, const int64_t* row_ptr, const uint32_t* col, const int32_t* cost,
                    const int64_t* supply, int64_t pivot_cap, FlowResult* out) {
  return simplex<int32_t>(n_nodes, row_ptr, col, cost, supply, pivot_cap, out);
}

int network_simplex_diag(int64_t n_nodes, const int64_t* row_ptr, const uint32_t* col, const int32_t* cost,
                         const int64_t* supply, int64_t pivot_cap, FlowResult* out) {
  if (n_nodes < 2) return simplex<int32_t>(n_nodes, row_ptr, col, cost, supply, pivot_cap, out);
  return simplex<int32_t>(n_nodes, row_ptr, col, cost, supply, pivot_cap, out, (int32_t)(n_nodes - 2),
                          (int32_t)(n_nodes - 1));
}

int network_simplex64_diag(int64_t n_nodes, const int64_t* row_ptr, const uint32_t* col, const int64_t* cost,
                           const int64_t* supply, int64_t pivot_cap, FlowResult* out) {
  if (n_nodes < 2) return simplex<int64_t>(n_nodes, row_ptr, col, cost, supply, pivot_cap, out);
  return simplex<int64_t>(n_nodes, row_ptr, col, cost, supply, pivot_cap, out, (int32_t)(n_nodes - 2),
                          (int32_t)(n_nodes - 1));
}

int network_simplex64(int64_t n_nodes, const int64_t* row_ptr, const uint32_t* col, const int64_t* cost,
                      const int64_t* supply, int64_t pivot_cap, FlowResult* out) {
  return simplex<int64_t>(n_nodes, row_ptr, col, cost, supply, pivot_cap, out);
}

int network_simplex_arcs(int64_t n_nodes, int64_t m, const uint32_t* src, const uint32_t* dst, const int32_t* cost,
                         const int64_t* supply, int64_t pivot_cap, FlowResult* out) {
  out->cost = -1;
  out->pivots = 0;
  out->status = 0;
  out->feasible = 0;
  if (n_nodes < 0 || m < 0 || n_nodes >= (int64_t(1) << 31) - 1) return -1;
  if (m > 0 && (!src || !dst || !cost)) return -1;
  for (int64_t a = 0; a < m; ++a)
    if (src[a] >= (uint64_t)n_nodes || dst[a] >= (uint64_t)n_nodes) return -1;
  // Arcs in CSR order (stable counting sort by tail); flows map back.
  std::vector<int64_t> row_ptr, perm;
  std::vector<uint32_t> col;
  std::vector<int32_t> cst;
  std::vector<int64_t> flow_csr;
  try {
    row_ptr.assign((size_t)n_nodes + 1, 0);
    for (int64_t a = 0; a < m; ++a) ++row_ptr[(size_t)src[a] + 1];
    for (int64_t v = 0; v < n_nodes; ++v) row_ptr[(size_t)v + 1] += row_ptr[(size_t)v];
    perm.resize((size_t)m);
    col.resize((size_t)m);
    cst.resize((size_t)m);
    std::vector<int64_t> fill(row_ptr.begin(), row_ptr.end() - 1);
    for (int64_t a = 0; a < m; ++a) {
      const int64_t q = fill[src[a]]++;
      perm[(size_t)q] = a;
      col[(size_t)q] = dst[a];
      cst[(size_t)q] = cost[a];
    }
    if (out->flow) flow_csr.resize((size_t)m);
  } catch (...) {
    return -3;
  }
  int64_t* user_flow = out->flow;
  out->flow = user_flow ? flow_csr.data() : nullptr;
  const int rc = network_simplex(n_nodes, row_ptr.data(), col.data(), cst.data(), supply, pivot_cap, out);
  out->flow = user_flow;
  if (rc == 0 && user_flow)
    for (int64_t q = 0; q < m; ++q) user_flow[perm[(size_t)q]] = flow_csr[(size_t)q];
  return rc;
}

// The method's network without the cell arcs u -> v that cost at
// least both cells' diagonal arcs together (cost(u, v) >= d(u) + d(v), with
// d = j - i the diagonal cost in the same units).  Leaving them out keeps the
// optimal cost (the argument of diagonal-dominance pruning, arc by arc):
// some optimal flow sends everything from B's diagonal node to A's directly
// over the zero-cost arc, so that arc carries as much as all paths from A
// mass to B mass together; a path through a dropped arc is replaced by its
// source's arc to A's diagonal node and its sink's arc from B's (both exist,
// the source holding A mass and the sink B mass), taking as much off the
// zero-cost arc, and d is 1-Lipschitz along cell arcs (|d(u) - d(v)| <=
// |di| + |dj| <= cost), so the replacement costs no more.  Paths from B's
// diagonal node, or into A's, are shortened the same way.  Rows stay sorted.
//
// The Euclidean network's costs are the real distances rounded up to
// integers through double arithmetic (relative error eta <= 2^-52 before the
// rounding up), so each rounded cost exceeds the real one by less than
// 1 + eta * cost and may fall short of it by eta * cost.  Carried through the
// argument above (a path between cells has fewer than n_cells arcs, and every
// cell's diagonal cost is the cost of one of its arcs, so all of them are at
// most the largest cost), a dropped arc must then cost at least
// d(u) + d(v) + M with M = 3 + 2^-50 * (n_cells + 3) * (largest cost); d is
// the rounded cost of the arc to the diagonal, formed as the network forms it.
namespace {
template <typename C>
void drop_dominated(int64_t nc, const int64_t* row_ptr, const uint32_t* col, const C* cost, const int32_t* ci,
                    const int32_t* cj, int cost_shift, SolveRows<C>& out) {
  const int64_t nrow = nc + 2, m = row_ptr[nrow];
  out.row_ptr.assign((size_t)nrow + 1, 0);
  out.col.clear();
  out.cost.clear();
  // most cell arcs go (all but 8% of a 400 + 400-point pair's); the vectors
  // grow if more stay
  out.col.reserve((size_t)(m / 8 + 4 * nrow));
  out.cost.reserve((size_t)(m / 8 + 4 * nrow));
  std::vector<int64_t> d((size_t)nc);
  int64_t margin = 0;
  if (cost_shift >= 0) {
    int64_t cmax = 0;
    for (int64_t a = 0; a < m; ++a) cmax = std::max<int64_t>(cmax, (int64_t)cost[a]);
    margin = 3 + (int64_t)std::ceil(std::ldexp((double)(nc + 3) * (double)cmax, -50));
    for (int64_t u = 0; u < nc; ++u)
      d[(size_t)u] = (int64_t)std::ceil(
          std::ldexp((double)((int64_t)cj[u] - (int64_t)ci[u]) * 0x1.6a09e667f3bcdp-1, cost_shift));
  } else {
    for (int64_t u = 0; u < nc; ++u) d[(size_t)u] = (int64_t)cj[u] - (int64_t)ci[u];
  }
  for (int64_t u = 0; u < nrow; ++u) {
    for (int64_t a = row_ptr[u]; a < row_ptr[u + 1]; ++a) {
      const uint32_t v = col[a];
      if (u < nc && (int64_t)v < nc && (int64_t)cost[a] >= d[(size_t)u] + d[(size_t)v] + margin) continue;
      out.col.push_back(v);
      out.cost.push_back(cost[a]);
    }
    out.row_ptr[(size_t)u + 1] = (int64_t)out.col.size();
  }
}
}  // namespace

void drop_dominated_arcs(int64_t n_cells, const int64_t* row_ptr, const uint32_t* col, const int32_t* cost,
                         const int32_t* ci, const int32_t* cj, int cost_shift, SolveRows<int32_t>& out) {
  drop_dominated(n_cells, row_ptr, col, cost, ci, cj, cost_shift, out);
}
void drop_dominated_arcs(int64_t n_cells, const int64_t* row_ptr, const uint32_t* col, const int64_t* cost,
                         const int32_t* ci, const int32_t* cj, int cost_shift, SolveRows<int64_t>& out) {
  drop_dominated(n_cells, row_ptr, col, cost, ci, cj, cost_shift, out);
}

}  // namespace w1

// Plain CPU oracle of the approximate 1-Wasserstein pipeline for persistence
// diagrams (Dey & Zhang, "Approximating 1-Wasserstein Distance between
// Persistence Diagrams by Graph Sparsification").
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
// reference that the GPU library is checked against.  Only the test suite, the
// smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
// code, header, table or helper with the GPU library, and the GPU library
// never calls it.
//
// Everything is single-threaded FP64 / int64 with the steps in the paper's
// order.  The ground metric is L-infinity (the integer-grid reading of the
// method, costs in units of g/2) or, with ORC_L2, the paper's own Euclidean
// metric (costs rounded up to integers in units of g 2^-K); where the paper
// is silent or ambiguous the reading taken is stated next to the step.  Every function with a pin in the test suite says so in
// its comment; nothing here is "parity unpinned".
//
// Steps
//   O0  validate, drop points on the diagonal              (Sec. 4.2)
//   O1  0-condensation of A u B with net multiplicities    (Sec. 4.3, overlap
//       rule of Sec. 5.3 applied at delta = 0)
//   O2  RWMD lower bound L = max(L_A, L_B)                 (Alg. 1, Sec. 5.1)
//   O3  eps split, s and the power-of-two grid g            (Prop. delta-
//       condensation, Thm. WSPD network, Cor. approximation bound)
//   O4  delta-condensation onto the grid                    (Alg. 2)
//   O5  Morton order of the cells
//   O6  binary radix (compressed quad) tree with tight boxes (Sec. 5.3,
//       split-tree paragraph)
//   O7  s-WSPD by the descendant-pair recursion            (Alg. 5 / Alg. 6)
//   O8  biarcs + diagonal arcs + supplies, and the network in
//       (tail, head)-sorted compressed sparse row form     (Sec. 5.3, Alg. 7,
//                                                           Appendix, network
//                                                           representation)
//   O9  exact min-cost flow (successive shortest paths)     (Def. transshipment)
//   O10 W1 = (g/2)(F* + n), W1_paper = (g/2) F*
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <queue>
#include <vector>

namespace {

enum Status { ORC_OK = 0, ORC_EINVAL = -1, ORC_ERANGE = -2, ORC_ENOFLOW = -7 };

struct Loc {
  double b, d;
  int64_t w;  // net multiplicity: count in A minus count in B
};

struct Cell {
  uint64_t key;
  int64_t i, j;       // shifted grid coordinates i' , j'
  int64_t cA, cB;     // multiplicities from A and from B
};

struct Node {
  int64_t lo, hi;     // range of cells (Morton order), inclusive
  int64_t left, right;  // child node ids, -1 for a leaf
  int64_t split;      // last index of the left child's range (internal only)
  int64_t mini, minj, maxi, maxj;
  int64_t diam;       // L-infinity diameter of the box = longest side
};

struct Arc {
  int64_t u, v, c;
};

struct Oracle {
  int status = ORC_OK;
  // O0/O1
  int64_t nA = 0, nB = 0, n = 0;
  std::vector<Loc> locs;
  // O2
  std::vector<double> t, term;
  double LA = 0, LB = 0, L = 0;
  int64_t SA = 0, SB = 0;
  int FA = 0, FB = 0;
  // O3
  double eps = 0, eps_c = 0;
  int s = 0;
  int e = 0;
  // O4/O5
  std::vector<Cell> cells;
  int64_t m0 = 0;
  // O6
  std::vector<Node> nodes;  // leaves 0..N-1 are the cells, internal nodes follow
  int64_t root = -1;
  // O7
  bool count_only = false;
  bool keep_nodes = false;
  bool prune = false;       // diagonal-dominance pruning (O7')
  bool l2 = false;          // Euclidean ground metric (the paper's own)
  int K = 0;                // l2: costs are integers in units of g 2^-K
  int64_t n_pairs = 0;
  uint64_t chk1 = 0, chk2 = 0;
  std::vector<int64_t> pu, pv, pc, pnu, pnv;
  // O9/O10
  int64_t flow_cost = -1;
  double W1 = 0, W1_paper = 0;
  // wall time of each step (seconds; bookkeeping for the CPU baseline, not
  // part of the method): O0+O1, O2, O3+O4+O5, O6, O7, O8, O9
  double stage_s[7] = {0, 0, 0, 0, 0, 0, 0};
};

// Seconds since t0, and t0 moved to now (stage timing bookkeeping).
double lap(std::chrono::steady_clock::time_point& t0) {
  auto t1 = std::chrono::steady_clock::now();
  double d = std::chrono::duration<double>(t1 - t0).count();
  t0 = t1;
  return d;
}

// ---------------------------------------------------------------- helpers --

int bitlen(uint64_t k) {
  int b = 0;
  while (k) {
    ++b;
    k >>= 1;
  }
  return b;
}

// Round-toward-zero conversion of a non-negative int64 below 2^62.
double to_double_rz(int64_t S) {
  double d = (double)S;
  if ((int64_t)d > S) d = std::nextafter(d, 0.0);
  return d;
}

// Order-independent pair checksum (test bookkeeping, not part of the method).
uint64_t pair_mix(uint64_t u, uint64_t v, uint64_t c) {
  uint64_t x = ((u + 1) * 0x9E3779B97F4A7C15ull + (v + 1)) * 0xC2B2AE3D27D4EB4Full + c;
  return x * 0x165667B19E3779F9ull;
}

// --------------------------------------------------------------- O0 + O1 --
// A persistence diagram is a multiset of off-diagonal points plus the
// diagonal (Sec. 4.2).  Points with death == birth are on the diagonal and
// carry no cost; non-finite values or death < birth are invalid input.
// W1 depends only on the signed difference of the two multisets (it is a
// Kantorovich distance on the plane with the diagonal collapsed to a point),
// so co-located A and B points cancel: this is the paper's rule for
// overlapping condensed nodes (merge, add supplies; Sec. 5.3) applied already
// at delta = 0.  The result is the 0-condensation of Sec. 4.3 of the net
// diagrams.  Pins: Hungarian exact W1 is invariant under adding common
// points; sum of net multiplicities; closed forms.
int condense0(Oracle& o, const double* A, int64_t nA, const double* B, int64_t nB) {
  struct P {
    double b, d;
    int64_t side;
  };
  std::vector<P> pts;
  pts.reserve((size_t)(nA + nB));
  for (int side = 0; side < 2; ++side) {
    const double* X = side == 0 ? A : B;
    int64_t nx = side == 0 ? nA : nB;
    for (int64_t k = 0; k < nx; ++k) {
      double b = X[2 * k] + 0.0, d = X[2 * k + 1] + 0.0;  // +0.0 folds -0.0 into +0.0
      if (!std::isfinite(b) || !std::isfinite(d) || d < b) return ORC_EINVAL;
      if (d == b) continue;
      pts.push_back({b, d, side});
    }
  }
  std::sort(pts.begin(), pts.end(), [](const P& x, const P& y) {
    if (x.b != y.b) return x.b < y.b;
    return x.d < y.d;
  });
  o.locs.clear();
  size_t k = 0;
  while (k < pts.size()) {
    size_t r = k;
    int64_t w = 0;
    while (r < pts.size() && pts[r].b == pts[k].b && pts[r].d == pts[k].d) {
      w += pts[r].side == 0 ? 1 : -1;
      ++r;
    }
    if (w != 0) o.locs.push_back({pts[k].b, pts[k].d, w});
    k = r;
  }
  o.nA = o.nB = 0;
  for (const Loc& l : o.locs) {
    if (l.w > 0) o.nA += l.w;
    else o.nB += -l.w;
  }
  o.n = o.nA + o.nB;
  return ORC_OK;
}

// -------------------------------------------------------------------- O2 --
// RWMD (Alg. 1 and the text before it): relax the conservation constraint of
// one side; each unit of supply at u then goes to its cheapest neighbour.
// In G(A,B) the neighbours of an A node are the B nodes and the diagonal node
// (the text takes the argmin over every arc, including the one to the
// diagonal; Alg. 1 as printed omits it, which would not give a lower bound).
// The cost to the diagonal in L-infinity is (d - b)/2.
// The sum is formed in exact int64 fixed point with every term rounded down,
// so it is independent of summation order and never exceeds the real sum.
// Pins: RWMD <= exact W1 over many seeds; single-point closed form; golden
// hand-computed example.
double fixed_point_sum(const std::vector<double>& terms, int64_t* S_out, int* F_out) {
  double M = 0.0;
  for (double x : terms) M = std::max(M, x);
  *S_out = 0;
  *F_out = 0;
  if (terms.empty() || M == 0.0) return 0.0;
  int E = 0;
  std::frexp(M, &E);  // M < 2^E
  int F = 62 - E - bitlen((uint64_t)terms.size());
  int64_t S = 0;
  for (double x : terms) S += (int64_t)std::floor(std::ldexp(x, F));
  *S_out = S;
  *F_out = F;
  return std::ldexp(to_double_rz(S), -F);
}

// The nearest location of the other diagram is found by scanning that
// diagram in birth order outwards from the query's birth, stopping once the
// birth gap alone reaches the best cost found (the L-infinity distance is at
// least the birth gap), so the minimum is exact.
double cheapest_arc(const std::vector<Loc>& other, double b, double d) {
  double best = 0.5 * (d - b);  // arc to the diagonal node
  size_t k = (size_t)(std::lower_bound(other.begin(), other.end(), b,
                                       [](const Loc& l, double x) { return l.b < x; }) - other.begin());
  for (size_t r = k; r < other.size() && other[r].b - b < best; ++r)
    best = std::min(best, std::max(std::fabs(b - other[r].b), std::fabs(d - other[r].d)));
  for (size_t r = k; r-- > 0 && b - other[r].b < best;)
    best = std::min(best, std::max(std::fabs(b - other[r].b), std::fabs(d - other[r].d)));
  return best;
}

// Euclidean ground metric (the paper's own, Sec. 4.2 problem statement):
// the distance of (b, d) to the diagonal is (d - b)/sqrt(2), here
// (d - b) * R with R the double nearest to 1/sqrt(2) (just above it).  The
// nearest location of the other diagram minimises
// q = (b - bv)^2 + (d - dv)^2 (each operation one IEEE double operation, in
// this order), and t = min(sqrt(q_min), (d - b) R) with the correctly rounded
// square root.  The scan in birth order stops once the squared birth gap
// exceeds the smallest q found: q is at least that square (every operation
// is monotone), so no later location can lower q_min.
const double R_SQRT1_2 = 0x1.6a09e667f3bcdp-1;

double cheapest_arc_l2(const std::vector<Loc>& other, double b, double d) {
  double q = std::numeric_limits<double>::infinity();
  size_t k = (size_t)(std::lower_bound(other.begin(), other.end(), b,
                                       [](const Loc& l, double x) { return l.b < x; }) - other.begin());
  for (size_t r = k; r < other.size(); ++r) {
    const double gb = b - other[r].b, gd = d - other[r].d;
    if (gb * gb > q) break;
    q = std::min(q, gb * gb + gd * gd);
  }
  for (size_t r = k; r-- > 0;) {
    const double gb = b - other[r].b, gd = d - other[r].d;
    if (gb * gb > q) break;
    q = std::min(q, gb * gb + gd * gd);
  }
  return std::min(std::sqrt(q), (d - b) * R_SQRT1_2);
}

void rwmd(Oracle& o) {
  const size_t m = o.locs.size();
  o.t.assign(m, 0.0);
  o.term.assign(m, 0.0);
  std::vector<Loc> sideA, sideB;  // locs are sorted by (b, d), so these are too
  for (const Loc& l : o.locs) (l.w > 0 ? sideA : sideB).push_back(l);
  std::vector<double> termA, termB;
  for (size_t u = 0; u < m; ++u) {
    const Loc& a = o.locs[u];
    const double best = o.l2 ? cheapest_arc_l2(a.w > 0 ? sideB : sideA, a.b, a.d)
                             : cheapest_arc(a.w > 0 ? sideB : sideA, a.b, a.d);
    o.t[u] = best;
    o.term[u] = (double)(a.w > 0 ? a.w : -a.w) * best;
    if (a.w > 0) termA.push_back(o.term[u]);
    else termB.push_back(o.term[u]);
  }
  o.LA = fixed_point_sum(termA, &o.SA, &o.FA);
  o.LB = fixed_point_sum(termB, &o.SB, &o.FB);
  o.L = std::max(o.LA, o.LB);
}

// -------------------------------------------------------------------- O3 --
// Error budget (L-infinity).  Snapping every point to the centre of its grid
// cell of side g moves it by at most g/2 per coordinate, and the cost to the
// diagonal is 1-Lipschitz, so W1 of the snapped diagrams is within n*g/2 of
// W1 (proof of Prop. delta-condensation, with the L-infinity ball instead of
// the sqrt(2) L2 ball).  Choosing g <= 2*eps_c*L/n with L <= W1 makes that
// error at most eps_c*W1.  The s-WSPD with the L-infinity box test below is a
// t-spanner with t = (s+2)/(s-2) (same induction as the paper's spanner
// statement, with diameters measured in L-infinity).  With
// W1_out = (g/2)(F* + n):  W1 <= W1_out <= (t + (t+1) eps_c) W1.
// s is the smallest integer with t + (t+1) eps_c <= 1 + eps; eps_c = kappa*eps.
// The grid side is rounded down to a power of two so that snapping is an
// exact scaling.  Pins: (eps -> s) golden table; bracket tests.
int choose_s(double eps, double eps_c) {
  double tau = (eps - 2.0 * eps_c) / (1.0 + eps_c);
  int s = (int)std::ceil(2.0 + 4.0 / tau);
  if (s < 3) s = 3;
  for (;;) {
    double t = (double)(s + 2) / (double)(s - 2);
    if (t + (t + 1.0) * eps_c <= 1.0 + eps) break;
    ++s;
  }
  return s;
}

// Euclidean metric: a point moves by at most half a cell diagonal, g/sqrt(2),
// and the distance to the diagonal is 1-Lipschitz, so W1 of the snapped
// diagrams is within n g/sqrt(2) of W1; g <= sqrt(2) eps_c L / n keeps that
// below eps_c W1 (Prop. delta-condensation's sqrt(2)).
int grid_exponent(double eps_c, double L, int64_t n, bool l2) {
  double gmax = ((2.0 * eps_c) * L) / (double)n;
  if (l2) gmax = gmax * R_SQRT1_2;
  double gsafe = gmax * (1.0 - 0x1p-40);
  int E = 0;
  std::frexp(gsafe, &E);  // 2^(E-1) <= gsafe < 2^E
  return E - 1;
}

// ---------------------------------------------------------------- O4 + O5 --
// delta-condensation (Alg. 2) with k = 1 and no random jitter: cell
// (floor(b/g), floor(d/g)), node at the cell centre, supplies aggregated.
// A and B points landing in one cell become one node with the supplies added
// (Sec. 5.3).  Coordinates are shifted by one common m0 so both axes stay
// aligned with the diagonal.  Cells are ordered by the Morton interleave of
// (i', j') (i' bits at even positions, j' bits at odd positions).
// Pins: sum of multiplicities, scaling by 2^k and translation invariance,
// node-drop identity.
uint64_t morton(int64_t i, int64_t j) {
  uint64_t k = 0;
  for (int bit = 0; bit < 30; ++bit) {
    k |= (uint64_t)((i >> bit) & 1) << (2 * bit);
    k |= (uint64_t)((j >> bit) & 1) << (2 * bit + 1);
  }
  return k;
}

int grid_condense(Oracle& o) {
  std::vector<Cell> raw;
  raw.reserve(o.locs.size());
  std::vector<int64_t> I(o.locs.size()), J(o.locs.size());
  int64_t m0 = std::numeric_limits<int64_t>::max();
  for (size_t k = 0; k < o.locs.size(); ++k) {
    double x = std::ldexp(o.locs[k].b, -o.e);
    double y = std::ldexp(o.locs[k].d, -o.e);
    if (!(std::fabs(x) < 0x1p62 && std::fabs(y) < 0x1p62)) return ORC_ERANGE;
    I[k] = (int64_t)std::floor(x);
    J[k] = (int64_t)std::floor(y);
    m0 = std::min(m0, std::min(I[k], J[k]));
  }
  for (size_t k = 0; k < o.locs.size(); ++k) {
    int64_t i = I[k] - m0, j = J[k] - m0;
    if (i >= (int64_t(1) << 30) || j >= (int64_t(1) << 30)) return ORC_ERANGE;
    int64_t w = o.locs[k].w;
    raw.push_back({morton(i, j), i, j, w > 0 ? w : 0, w < 0 ? -w : 0});
  }
  o.m0 = m0;
  std::sort(raw.begin(), raw.end(), [](const Cell& x, const Cell& y) { return x.key < y.key; });
  o.cells.clear();
  for (const Cell& c : raw) {
    if (!o.cells.empty() && o.cells.back().key == c.key) {
      o.cells.back().cA += c.cA;
      o.cells.back().cB += c.cB;
    } else {
      o.cells.push_back(c);
    }
  }
  return ORC_OK;
}

// -------------------------------------------------------------------- O6 --
// Hierarchy for the WSPD: the paper uses a split tree (bounding box, halve the
// longest side).  Any hierarchy whose leaves are the single points yields a
// valid WSPD, and the method's spanner argument only needs a WSPD.  Here the
// hierarchy is the binary radix tree of the sorted Morton keys (a compressed
// quadtree with the x/y halvings as separate levels): a node covering cells
// [lo, hi] splits where the highest bit in which key[lo] and key[hi] differ
// changes from 0 to 1.  As in the paper's implementation, a node keeps only a
// representative (its first cell) and a tight bounding box.
// Pins: tree invariants (two children, ranges partition, highest differing
// bit, tight boxes by brute force).
int64_t build_tree(Oracle& o, int64_t lo, int64_t hi) {
  if (lo == hi) return lo;  // leaf = cell id
  uint64_t x = o.cells[lo].key ^ o.cells[hi].key;
  int bit = 63;
  while (!((x >> bit) & 1)) --bit;
  int64_t m = lo;
  while (m + 1 <= hi && !((o.cells[m + 1].key >> bit) & 1)) ++m;
  int64_t id = (int64_t)o.nodes.size();
  o.nodes.push_back(Node{});
  int64_t l = build_tree(o, lo, m);
  int64_t r = build_tree(o, m + 1, hi);
  Node nd;
  nd.lo = lo;
  nd.hi = hi;
  nd.left = l;
  nd.right = r;
  nd.split = m;
  nd.mini = std::min(o.nodes[l].mini, o.nodes[r].mini);
  nd.minj = std::min(o.nodes[l].minj, o.nodes[r].minj);
  nd.maxi = std::max(o.nodes[l].maxi, o.nodes[r].maxi);
  nd.maxj = std::max(o.nodes[l].maxj, o.nodes[r].maxj);
  nd.diam = std::max(nd.maxi - nd.mini, nd.maxj - nd.minj);
  o.nodes[id] = nd;
  return id;
}

void tree(Oracle& o) {
  const int64_t N = (int64_t)o.cells.size();
  o.nodes.clear();
  for (int64_t k = 0; k < N; ++k) {
    const Cell& c = o.cells[k];
    o.nodes.push_back(Node{k, k, -1, -1, -1, c.i, c.j, c.i, c.j, 0});
  }
  o.root = N > 0 ? build_tree(o, 0, N - 1) : -1;
}

// -------------------------------------------------------------------- O7 --
// s-WSPD (Alg. 5 / Alg. 6): for each internal node w, search its two
// children; a pair of nodes that is s-well-separated is output with the
// nodes' representatives, otherwise the node with the longer bounding-box
// side is split (ties split the second node).  Well-separated (L-infinity
// reading of the ball test): the box gap is at least s times the larger box
// diameter.  Pins: brute-force coverage (every pair of distinct cells in
// exactly one output pair), separation of every pair, spanner stretch by
// all-pairs shortest paths.
// Euclidean costs (O8 with the l2 metric), integers in units of g 2^-K: the
// distance of two cell centres, ceil(sqrt(di^2 + dj^2) 2^K), and of a cell
// centre to the diagonal, ceil((j - i) R 2^K), each from IEEE double
// operations in this order (the integer sum converted to double, correctly
// rounded square root, exact scaling by 2^K).  Rounding up keeps every cost
// at least the exact distance (up to one rounding of the square root), so
// the network's optimum still bounds W1 of the condensed diagrams from above.
int64_t cost_l2(int64_t di, int64_t dj, int K) {
  return (int64_t)std::ceil(std::ldexp(std::sqrt((double)(di * di + dj * dj)), K));
}
int64_t diag_cost_l2(int64_t di_dj, int K) {
  return (int64_t)std::ceil(std::ldexp((double)di_dj * R_SQRT1_2, K));
}

void emit(Oracle& o, int64_t U, int64_t V) {
  const Node& a = o.nodes[U];
  const Node& b = o.nodes[V];
  int64_t u = a.lo, v = b.lo;
  int64_t c = o.l2 ? cost_l2(o.cells[u].i - o.cells[v].i, o.cells[u].j - o.cells[v].j, o.K)
                   : 2 * std::max(std::llabs(o.cells[u].i - o.cells[v].i), std::llabs(o.cells[u].j - o.cells[v].j));
  ++o.n_pairs;
  // record checksum: a Euclidean pair record carries no cost (its costs come
  // from the cells when the network rows are built), so c = 0 enters it
  uint64_t h = pair_mix((uint64_t)u, (uint64_t)v, o.l2 ? 0 : (uint64_t)c);
  o.chk1 += h;
  o.chk2 += h * h;
  if (o.count_only) return;
  o.pu.push_back(u);
  o.pv.push_back(v);
  o.pc.push_back(c);
  if (o.keep_nodes) {
    o.pnu.push_back(U);
    o.pnv.push_back(V);
  }
}

// O7' (optional, not in the paper): diagonal-dominance pruning.  Costs are
// in units of g/2: a cell's arc to the diagonal costs j - i, a WSPD arc
// between cells p and q costs 2 max(|di|, |dj|) >= 2 dist(U, V) for p in U,
// q in V, and j - i <= maxj - mini over a box.  When
//   2 dist(U, V) >= (U.maxj - U.mini) + (V.maxj - V.mini)
// every arc the pair (U, V) or any of its descendant pairs would add costs at
// least the two representatives' diagonal costs together, c(p,q) >= dd(p) +
// dd(q).  Such arcs can be left out without changing the optimal flow cost
// F*: take an optimal flow, decompose it into paths, and send every path that
// uses such an arc from its source cell straight to the A-diagonal node and
// from the B-diagonal node straight to its sink cell (lowering the flow on the
// zero-cost B->A diagonal arc by as much, which carries at least the total
// cell-to-cell flow).  The diagonal cost is 1-Lipschitz along cell arcs
// (|d(j-i)| <= 2 max(|di|,|dj|)), so neither replacement costs more.  The
// test is monotone (children have smaller boxes and larger gaps), so the
// whole recursion below a dominated pair is skipped, and the pairs kept are
// exactly the s-WSPD pairs whose own boxes are not dominated.
// Pins: F* equal with and without pruning over many seeds; the pruned pair
// set equals the unpruned one filtered by the box test.
bool dominated(const Node& a, const Node& b) {
  int64_t gi = std::max(a.mini - b.maxi, b.mini - a.maxi);
  int64_t gj = std::max(a.minj - b.maxj, b.minj - a.maxj);
  int64_t dist = std::max<int64_t>(0, std::max(gi, gj));
  return 2 * dist >= (a.maxj - a.mini) + (b.maxj - b.mini);
}

// Euclidean reading of the separation (Sec. 5.3: balls of the larger
// diameter at distance at least s times that diameter): the boxes' Euclidean
// gap is at least s times the larger box diagonal, tested exactly on squares
// in 128-bit integers; the node with the longer diagonal is split (ties
// split the second node).  The spanner stretch (s+2)/(s-2) holds with
// Euclidean diameters by the same induction.
void visit_l2(Oracle& o, int64_t U, int64_t V) {
  const Node& a = o.nodes[U];
  const Node& b = o.nodes[V];
  const int64_t gi = std::max<int64_t>(0, std::max(a.mini - b.maxi, b.mini - a.maxi));
  const int64_t gj = std::max<int64_t>(0, std::max(a.minj - b.maxj, b.minj - a.maxj));
  const int64_t da = (a.maxi - a.mini) * (a.maxi - a.mini) + (a.maxj - a.minj) * (a.maxj - a.minj);
  const int64_t db = (b.maxi - b.mini) * (b.maxi - b.mini) + (b.maxj - b.minj) * (b.maxj - b.minj);
  const __int128 dist2 = (__int128)gi * gi + (__int128)gj * gj;
  if (dist2 >= (__int128)o.s * o.s * std::max(da, db)) {
    emit(o, U, V);
    return;
  }
  if (da > db) {
    visit_l2(o, a.left, V);
    visit_l2(o, a.right, V);
  } else {
    visit_l2(o, U, b.left);
    visit_l2(o, U, b.right);
  }
}

void visit(Oracle& o, int64_t U, int64_t V) {
  if (o.l2) {
    visit_l2(o, U, V);
    return;
  }
  const Node& a = o.nodes[U];
  const Node& b = o.nodes[V];
  if (o.prune && dominated(a, b)) return;
  int64_t gi = std::max(a.mini - b.maxi, b.mini - a.maxi);
  int64_t gj = std::max(a.minj - b.maxj, b.minj - a.maxj);
  int64_t dist = std::max<int64_t>(0, std::max(gi, gj));
  int64_t dmax = std::max(a.diam, b.diam);
  if (dist >= (int64_t)o.s * dmax) {
    emit(o, U, V);
    return;
  }
  if (a.diam > b.diam) {
    visit(o, a.left, V);
    visit(o, a.right, V);
  } else {
    visit(o, U, b.left);
    visit(o, U, b.right);
  }
}

void wspd(Oracle& o) {
  o.n_pairs = 0;
  o.chk1 = o.chk2 = 0;
  o.pu.clear();
  o.pv.clear();
  o.pc.clear();
  o.pnu.clear();
  o.pnv.clear();
  const int64_t N = (int64_t)o.cells.size();
  for (int64_t w = N; w < (int64_t)o.nodes.size(); ++w) visit(o, o.nodes[w].left, o.nodes[w].right);
}

// -------------------------------------------------------------------- O9 --
// Uncapacitated min-cost flow: minimise sum c*f subject to
// out(v) - in(v) = supply(v) and f >= 0 (Def. transshipment; the printed
// conservation rows are garbled for transit nodes, the standard balance is
// used).  Solved exactly by successive shortest paths with Dijkstra on
// reduced costs (Johnson potentials), super source and sink.  Returns the
// optimal cost; flow and potentials (a dual certificate) on request.
// Pins: equals 2x the Hungarian exact W1 on the 0-condensed network of
// integer diagrams (Prop. matching <=> flow), equals networkx network simplex,
// LP optimality certificate.
struct Edge {
  int64_t to, cap, cost;
};

int64_t ssp(int64_t nn, const std::vector<Arc>& arcs, const std::vector<int64_t>& supply,
            std::vector<int64_t>* flow_out, std::vector<int64_t>* pot_out, int* status) {
  const int64_t S = nn, T = nn + 1, V = nn + 2;
  int64_t total = 0;
  for (int64_t x : supply)
    if (x > 0) total += x;
  std::vector<Edge> E;
  std::vector<std::vector<int64_t>> adj((size_t)V);
  auto add = [&](int64_t a, int64_t b, int64_t cap, int64_t cost) {
    adj[(size_t)a].push_back((int64_t)E.size());
    E.push_back({b, cap, cost});
    adj[(size_t)b].push_back((int64_t)E.size());
    E.push_back({a, 0, -cost});
  };
  const int64_t INF_CAP = total + 1;
  for (const Arc& a : arcs) add(a.u, a.v, INF_CAP, a.c);
  for (int64_t v = 0; v < nn; ++v) {
    if (supply[(size_t)v] > 0) add(S, v, supply[(size_t)v], 0);
    if (supply[(size_t)v] < 0) add(v, T, -supply[(size_t)v], 0);
  }
  const int64_t INF = std::numeric_limits<int64_t>::max() / 4;
  std::vector<int64_t> h((size_t)V, 0), dist((size_t)V), prev_e((size_t)V);
  std::vector<char> done((size_t)V);
  int64_t sent = 0;
  while (sent < total) {
    std::fill(dist.begin(), dist.end(), INF);
    std::fill(done.begin(), done.end(), 0);
    std::fill(prev_e.begin(), prev_e.end(), -1);
    typedef std::pair<int64_t, int64_t> QE;
    std::priority_queue<QE, std::vector<QE>, std::greater<QE>> pq;
    dist[(size_t)S] = 0;
    pq.push({0, S});
    while (!pq.empty()) {
      QE top = pq.top();
      pq.pop();
      int64_t x = top.second;
      if (done[(size_t)x] || top.first != dist[(size_t)x]) continue;
      done[(size_t)x] = 1;
      if (x == T) break;
      for (int64_t ei : adj[(size_t)x]) {
        const Edge& ed = E[(size_t)ei];
        if (ed.cap <= 0) continue;
        int64_t nd = dist[(size_t)x] + ed.cost + h[(size_t)x] - h[(size_t)ed.to];
        if (nd < dist[(size_t)ed.to]) {
          dist[(size_t)ed.to] = nd;
          prev_e[(size_t)ed.to] = ei;
          pq.push({nd, ed.to});
        }
      }
    }
    if (!done[(size_t)T]) {
      *status = ORC_ENOFLOW;
      return -1;
    }
    const int64_t dT = dist[(size_t)T];
    for (int64_t x = 0; x < V; ++x) h[(size_t)x] += std::min(dist[(size_t)x], dT);
    int64_t push = INF;
    for (int64_t x = T; x != S;) {
      const Edge& ed = E[(size_t)prev_e[(size_t)x]];
      push = std::min(push, ed.cap);
      x = E[(size_t)(prev_e[(size_t)x] ^ 1)].to;
    }
    for (int64_t x = T; x != S;) {
      int64_t ei = prev_e[(size_t)x];
      E[(size_t)ei].cap -= push;
      E[(size_t)(ei ^ 1)].cap += push;
      x = E[(size_t)(ei ^ 1)].to;
    }
    sent += push;
  }
  int64_t cost = 0;
  if (flow_out) flow_out->assign(arcs.size(), 0);
  for (size_t k = 0; k < arcs.size(); ++k) {
    int64_t f = E[2 * k + 1].cap;  // flow = capacity of the reverse edge
    cost += f * arcs[k].c;
    if (flow_out) (*flow_out)[k] = f;
  }
  if (pot_out) {
    pot_out->assign((size_t)nn, 0);
    for (int64_t x = 0; x < nn; ++x) (*pot_out)[(size_t)x] = -h[(size_t)x];
  }
  *status = ORC_OK;
  return cost;
}

// -------------------------------------------------------------------- O8 --
// Sparse transshipment network WS_s^PD (Sec. 5.3, Alg. 7): nodes are the
// cells (ids 0..N-1 in Morton order), the diagonal node of A (id N) and of B
// (id N+1).  Every WSPD pair gives a biarc (both directions) with the
// L-infinity distance of the representatives; an A cell has an arc to the A
// diagonal node and the B diagonal node has an arc to a B cell, both with the
// cell's distance to the diagonal; the B diagonal node sends to the A
// diagonal node at cost 0 (projection-projection edges, Sec. 4.3).  Costs are
// integers in units of g/2.  Supplies: cell cA - cB, A diagonal -nA, B
// diagonal +nB.
void network(const Oracle& o, std::vector<Arc>* arcs, std::vector<int64_t>* supply) {
  const int64_t N = (int64_t)o.cells.size();
  arcs->clear();
  for (size_t k = 0; k < o.pu.size(); ++k) {
    arcs->push_back({o.pu[k], o.pv[k], o.pc[k]});
    arcs->push_back({o.pv[k], o.pu[k], o.pc[k]});
  }
  for (int64_t c = 0; c < N; ++c) {
    int64_t dd = o.cells[(size_t)c].j - o.cells[(size_t)c].i;
    if (o.l2) dd = diag_cost_l2(dd, o.K);
    if (o.cells[(size_t)c].cA > 0) arcs->push_back({c, N, dd});
    if (o.cells[(size_t)c].cB > 0) arcs->push_back({N + 1, c, dd});
  }
  arcs->push_back({N + 1, N, 0});
  supply->assign((size_t)(N + 2), 0);
  for (int64_t c = 0; c < N; ++c) (*supply)[(size_t)c] = o.cells[(size_t)c].cA - o.cells[(size_t)c].cB;
  (*supply)[(size_t)N] = -o.nA;
  (*supply)[(size_t)(N + 1)] = o.nB;
}

// Compressed sparse row form of the same network (O8, Appendix
// "Representing the Transshipment Network"): the arcs sorted by tail, ties by
// head, so the arcs of node v are row_ptr[v] .. row_ptr[v+1]-1.  A plain
// std::sort of the arc list, then the row pointers from the tails.  The arc
// pairs are distinct (a repeated (tail, head) would mean a cell pair covered
// by two WSPD pairs), so the sorted order is unique.  Pins: sortedness and
// distinct arcs, the arc-count identity, costs recomputed from the cells,
// equality with the unsorted arc list as a multiset.
void csr(const Oracle& o, std::vector<int64_t>* row_ptr, std::vector<Arc>* arcs) {
  std::vector<int64_t> supply;
  network(o, arcs, &supply);
  std::sort(arcs->begin(), arcs->end(), [](const Arc& x, const Arc& y) {
    if (x.u != y.u) return x.u < y.u;
    return x.v < y.v;
  });
  const int64_t nn = (int64_t)o.cells.size() + 2;
  row_ptr->assign((size_t)(nn + 1), 0);
  for (const Arc& a : *arcs) ++(*row_ptr)[(size_t)(a.u + 1)];
  for (int64_t v = 0; v < nn; ++v) (*row_ptr)[(size_t)(v + 1)] += (*row_ptr)[(size_t)v];
}

}  // namespace

// ===================================================================== ABI ==
extern "C" {

enum {
  ORC_STOP_AFTER_TREE = 1,
  ORC_COUNT_ONLY = 2,
  ORC_NO_FLOW = 4,
  ORC_KEEP_PAIR_NODES = 8,
  ORC_SKIP_RWMD = 16,   // take L from the caller (for timing later stages alone)
  ORC_PRUNE = 32,       // diagonal-dominance pruning of the WSPD pairs (O7')
  ORC_L2 = 64,          // Euclidean ground metric
  ORC_PAPER_GRID = 128, // with s_override: the grid of Alg. 2 / Alg. 3 (eps_c from s)
};

void* orc_new(void) { return new Oracle(); }
void orc_free(void* p) { delete (Oracle*)p; }

int orc_run(void* p, const double* A, int64_t nA, const double* B, int64_t nB, double eps, double kappa,
            int s_override, int flags, double given_L) {
  Oracle& o = *(Oracle*)p;
  o = Oracle();
  if (!(eps > 0.0 && eps <= 1.0) || !(kappa > 0.0 && kappa < 0.5) || nA < 0 || nB < 0) return o.status = ORC_EINVAL;
  o.count_only = (flags & ORC_COUNT_ONLY) != 0;
  o.keep_nodes = (flags & ORC_KEEP_PAIR_NODES) != 0;
  o.prune = (flags & ORC_PRUNE) != 0;
  o.l2 = (flags & ORC_L2) != 0;
  if (o.l2 && o.prune) return o.status = ORC_EINVAL;  // pruning is exact for integer L-infinity costs only
  auto t0 = std::chrono::steady_clock::now();
  int st = condense0(o, A, nA, B, nB);
  o.stage_s[0] = lap(t0);
  if (st) return o.status = st;
  o.eps = eps;
  o.eps_c = kappa * eps;
  if (flags & ORC_PAPER_GRID) {
    // the paper's own parameter choice for a given sparsity s (Alg. 2, Alg. 3):
    // the condensation error is 8/(s - 4) for s >= 12 and 1 below that, and
    // it sets the grid through the same bound g <= 2 eps_c L / n as above
    if (s_override <= 0) return o.status = ORC_EINVAL;
    o.eps_c = s_override >= 12 ? 8.0 / (double)(s_override - 4) : 1.0;
  }
  o.s = s_override > 0 ? s_override : choose_s(eps, o.eps_c);
  if (o.n == 0) {  // identical diagrams (up to diagonal points): W1 = 0
    o.flow_cost = 0;
    return o.status = ORC_OK;
  }
  if (flags & ORC_SKIP_RWMD) {
    o.L = given_L;
  } else {
    rwmd(o);
  }
  o.stage_s[1] = lap(t0);
  if (!(o.L > 0.0)) return o.status = ORC_ERANGE;
  o.e = grid_exponent(o.eps_c, o.L, o.n, o.l2);
  st = grid_condense(o);
  o.stage_s[2] = lap(t0);
  if (st) return o.status = st;
  if (o.l2) {
    // cost scale 2^K: every cost is below 2^(bitlen(X) + 1 + K) and F* at
    // most n times the largest diagonal cost (X: the largest shifted
    // coordinate), so K = 59 - bitlen(n) - bitlen(X) keeps F* and any
    // big-M cost of (max cost + 1)(node count + 1) below 2^60
    int64_t X = 1;
    for (const Cell& c : o.cells) X = std::max(X, std::max(c.i, c.j));
    o.K = std::min(30, 59 - bitlen((uint64_t)o.n) - bitlen((uint64_t)X));
    if (o.K < 0) return o.status = ORC_ERANGE;
  }
  tree(o);
  o.stage_s[3] = lap(t0);
  if (flags & ORC_STOP_AFTER_TREE) return o.status = ORC_OK;
  wspd(o);
  o.stage_s[4] = lap(t0);
  if (o.count_only || (flags & ORC_NO_FLOW)) return o.status = ORC_OK;
  std::vector<Arc> arcs;
  std::vector<int64_t> supply;
  network(o, &arcs, &supply);
  o.stage_s[5] = lap(t0);
  int fst = 0;
  o.flow_cost = ssp((int64_t)o.cells.size() + 2, arcs, supply, nullptr, nullptr, &fst);
  o.stage_s[6] = lap(t0);
  if (fst) return o.status = fst;
  if (o.l2) {  // W1 = g (F* 2^-K + n / sqrt(2)): the condensation's n g / sqrt(2) added back
    o.W1_paper = std::ldexp((double)o.flow_cost, o.e - o.K);
    o.W1 = o.W1_paper + (double)o.n * std::ldexp(R_SQRT1_2, o.e);
  } else {
    o.W1 = std::ldexp((double)(o.flow_cost + o.n), o.e - 1);
    o.W1_paper = std::ldexp((double)o.flow_cost, o.e - 1);
  }
  return o.status = ORC_OK;
}

// Scalars ------------------------------------------------------------------
enum {
  K_STATUS, K_NA, K_NB, K_N, K_NLOC, K_S, K_E, K_M0, K_NCELLS, K_NNODES, K_ROOT, K_NPAIRS, K_FLOW,
  K_SA, K_SB, K_FA, K_FB, K_CHK1, K_CHK2, K_COSTK
};
int64_t orc_i64(void* p, int key) {
  Oracle& o = *(Oracle*)p;
  switch (key) {
    case K_STATUS: return o.status;
    case K_NA: return o.nA;
    case K_NB: return o.nB;
    case K_N: return o.n;
    case K_NLOC: return (int64_t)o.locs.size();
    case K_S: return o.s;
    case K_E: return o.e;
    case K_M0: return o.m0;
    case K_NCELLS: return (int64_t)o.cells.size();
    case K_NNODES: return (int64_t)o.nodes.size();
    case K_ROOT: return o.root;
    case K_NPAIRS: return o.n_pairs;
    case K_FLOW: return o.flow_cost;
    case K_SA: return o.SA;
    case K_SB: return o.SB;
    case K_FA: return o.FA;
    case K_FB: return o.FB;
    case K_CHK1: return (int64_t)o.chk1;
    case K_CHK2: return (int64_t)o.chk2;
    case K_COSTK: return o.K;
  }
  return 0;
}

enum { D_L, D_LA, D_LB, D_W1, D_W1P, D_G, D_EPSC };
double orc_f64(void* p, int key) {
  Oracle& o = *(Oracle*)p;
  switch (key) {
    case D_L: return o.L;
    case D_LA: return o.LA;
    case D_LB: return o.LB;
    case D_W1: return o.W1;
    case D_W1P: return o.W1_paper;
    case D_G: return std::ldexp(1.0, o.e);
    case D_EPSC: return o.eps_c;
  }
  return 0.0;
}

// Wall time of each step of the last run: O0+O1, O2, O3-O5, O6, O7, O8, O9.
void orc_stage_seconds(void* p, double* out7) {
  Oracle& o = *(Oracle*)p;
  for (int k = 0; k < 7; ++k) out7[k] = o.stage_s[k];
}

// Arrays (caller allocates with the sizes above) ------------------------------
void orc_locs(void* p, double* b, double* d, int64_t* w, double* t, double* term) {
  Oracle& o = *(Oracle*)p;
  for (size_t k = 0; k < o.locs.size(); ++k) {
    b[k] = o.locs[k].b;
    d[k] = o.locs[k].d;
    w[k] = o.locs[k].w;
    if (t) t[k] = k < o.t.size() ? o.t[k] : 0.0;
    if (term) term[k] = k < o.term.size() ? o.term[k] : 0.0;
  }
}

void orc_cells(void* p, int64_t* i, int64_t* j, int64_t* cA, int64_t* cB, uint64_t* key) {
  Oracle& o = *(Oracle*)p;
  for (size_t k = 0; k < o.cells.size(); ++k) {
    i[k] = o.cells[k].i;
    j[k] = o.cells[k].j;
    cA[k] = o.cells[k].cA;
    cB[k] = o.cells[k].cB;
    key[k] = o.cells[k].key;
  }
}

// Node k: lo, hi, left, right, split, mini, minj, maxi, maxj, diam (10 int64).
void orc_nodes(void* p, int64_t* out10) {
  Oracle& o = *(Oracle*)p;
  for (size_t k = 0; k < o.nodes.size(); ++k) {
    const Node& n = o.nodes[k];
    int64_t* r = out10 + 10 * k;
    r[0] = n.lo; r[1] = n.hi; r[2] = n.left; r[3] = n.right; r[4] = n.split;
    r[5] = n.mini; r[6] = n.minj; r[7] = n.maxi; r[8] = n.maxj; r[9] = n.diam;
  }
}

void orc_pairs(void* p, int64_t* u, int64_t* v, int64_t* c, int64_t* nu, int64_t* nv) {
  Oracle& o = *(Oracle*)p;
  for (size_t k = 0; k < o.pu.size(); ++k) {
    u[k] = o.pu[k];
    v[k] = o.pv[k];
    c[k] = o.pc[k];
    if (nu && k < o.pnu.size()) nu[k] = o.pnu[k];
    if (nv && k < o.pnv.size()) nv[k] = o.pnv[k];
  }
}

// Network as arc arrays: returns arc count when called with null buffers.
int64_t orc_network(void* p, int64_t* src, int64_t* dst, int64_t* cost, int64_t* supply) {
  Oracle& o = *(Oracle*)p;
  std::vector<Arc> arcs;
  std::vector<int64_t> sup;
  network(o, &arcs, &sup);
  if (src) {
    for (size_t k = 0; k < arcs.size(); ++k) {
      src[k] = arcs[k].u;
      dst[k] = arcs[k].v;
      cost[k] = arcs[k].c;
    }
    for (size_t k = 0; k < sup.size(); ++k) supply[k] = sup[k];
  }
  return (int64_t)arcs.size();
}

// Network in CSR form (n_cells + 3 row pointers, arcs sorted by (tail,
// head)): returns the arc count when called with null buffers.
int64_t orc_csr(void* p, int64_t* row_ptr, int64_t* col, int64_t* cost) {
  Oracle& o = *(Oracle*)p;
  std::vector<int64_t> rp;
  std::vector<Arc> arcs;
  csr(o, &rp, &arcs);
  if (row_ptr) {
    for (size_t k = 0; k < rp.size(); ++k) row_ptr[k] = rp[k];
    for (size_t k = 0; k < arcs.size(); ++k) {
      col[k] = arcs[k].v;
      cost[k] = arcs[k].c;
    }
  }
  return (int64_t)arcs.size();
}

// Stand-alone exact min-cost flow on any network with non-negative integer
// costs; returns the optimal cost or -1 if the supplies cannot be routed.
int64_t orc_mcf(int64_t nn, int64_t m, const int64_t* src, const int64_t* dst, const int64_t* cost,
                const int64_t* supply, int64_t* flow_out, int64_t* pot_out) {
  std::vector<Arc> arcs((size_t)m);
  for (int64_t k = 0; k < m; ++k) arcs[(size_t)k] = {src[k], dst[k], cost[k]};
  std::vector<int64_t> sup(supply, supply + nn);
  std::vector<int64_t> flow, pot;
  int st = 0;
  int64_t c = ssp(nn, arcs, sup, &flow, &pot, &st);
  if (st) return -1;
  if (flow_out) std::memcpy(flow_out, flow.data(), sizeof(int64_t) * (size_t)m);
  if (pot_out) std::memcpy(pot_out, pot.data(), sizeof(int64_t) * (size_t)nn);
  return c;
}

int orc_choose_s(double eps, double kappa) { return choose_s(eps, kappa * eps); }
int orc_grid_exponent(double eps_c, double L, int64_t n, int l2) { return grid_exponent(eps_c, L, n, l2 != 0); }

}  // extern "C"

// Host code under AddressSanitizer and UndefinedBehaviorSanitizer (built
// with g++ by tests/test_sanitizers.py; no GPU): the library's network
// simplex on random networks, in its three entry forms, with and without
// pivot caps and on invalid input, and the oracle pipeline in every mode on
// small random diagrams, reading back every array it exposes.  Results are
// checked only loosely here (flow conservation, optimality certificates, the
// simplex against the oracle's successive shortest paths); the point is
// that no access goes out of bounds and no arithmetic is undefined.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2110_14734_amd/csrc/flow.h"

extern "C" {
void* orc_new(void);
void orc_free(void* p);
int orc_run(void* p, const double* A, int64_t nA, const double* B, int64_t nB, double eps, double kappa,
            int s_override, int flags, double given_L);
int64_t orc_i64(void* p, int key);
double orc_f64(void* p, int key);
void orc_stage_seconds(void* p, double* out7);
void orc_locs(void* p, double* b, double* d, int64_t* w, double* t, double* term);
void orc_cells(void* p, int64_t* i, int64_t* j, int64_t* cA, int64_t* cB, uint64_t* key);
void orc_nodes(void* p, int64_t* out10);
void orc_pairs(void* p, int64_t* u, int64_t* v, int64_t* c, int64_t* nu, int64_t* nv);
int64_t orc_network(void* p, int64_t* src, int64_t* dst, int64_t* cost, int64_t* supply);
int64_t orc_csr(void* p, int64_t* row_ptr, int64_t* col, int64_t* cost);
int64_t orc_mcf(int64_t nn, int64_t m, const int64_t* src, const int64_t* dst, const int64_t* cost,
                const int64_t* supply, int64_t* flow_out, int64_t* pot_out);
}

static int fails = 0;
#define EXPECT(c)                                          \
  do {                                                     \
    if (!(c)) {                                            \
      std::printf("FAILED: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                             \
    }                                                      \
  } while (0)

// keys of orc_i64
enum { K_STATUS, K_NA, K_NB, K_N, K_NLOC, K_S, K_E, K_M0, K_NCELLS, K_NNODES, K_ROOT, K_NPAIRS, K_FLOW };
constexpr int K_COSTK = 19;  // the Euclidean cost shift

static void flows(std::mt19937_64& rng) {
  for (int trial = 0; trial < 60; ++trial) {
    const int64_t n = 3 + (int64_t)(rng() % 40);
    std::vector<uint32_t> src, dst;
    std::vector<int32_t> cost;
    for (int64_t v = 0; v < n; ++v) {  // a cycle keeps every supply feasible
      src.push_back((uint32_t)v);
      dst.push_back((uint32_t)((v + 1) % n));
      cost.push_back((int32_t)(rng() % 20));
    }
    const int64_t extra = (int64_t)(rng() % (size_t)(6 * n));
    for (int64_t k = 0; k < extra; ++k) {
      const uint32_t a = (uint32_t)(rng() % (size_t)n), b = (uint32_t)(rng() % (size_t)n);
      if (a == b) continue;
      src.push_back(a);
      dst.push_back(b);
      cost.push_back((int32_t)(trial % 3 == 0 ? rng() % 2 : rng() % 30));
    }
    const int64_t m = (int64_t)src.size();
    std::vector<int64_t> sup((size_t)n);
    int64_t tot = 0;
    for (int64_t v = 0; v + 1 < n; ++v) {
      sup[(size_t)v] = (int64_t)(rng() % 13) - 6;
      tot += sup[(size_t)v];
    }
    sup[(size_t)(n - 1)] = -tot;
    // arc-list form, with flow and potentials
    std::vector<int64_t> flow((size_t)m), pot((size_t)n);
    w1::FlowResult r{};
    r.flow = flow.data();
    r.pot = pot.data();
    EXPECT(w1::network_simplex_arcs(n, m, src.data(), dst.data(), cost.data(), sup.data(), 0, &r) == 0);
    EXPECT(r.status == 0 && r.feasible == 1);
    std::vector<int64_t> bal((size_t)n, 0);
    for (int64_t k = 0; k < m; ++k) {
      EXPECT(flow[(size_t)k] >= 0);
      bal[src[(size_t)k]] += flow[(size_t)k];
      bal[dst[(size_t)k]] -= flow[(size_t)k];
      const int64_t red = cost[(size_t)k] + pot[src[(size_t)k]] - pot[dst[(size_t)k]];
      EXPECT(red >= 0 && (flow[(size_t)k] == 0 || red == 0));
    }
    for (int64_t v = 0; v < n; ++v) EXPECT(bal[(size_t)v] == sup[(size_t)v]);
    std::vector<int64_t> s64(src.begin(), src.end()), d64(dst.begin(), dst.end()), c64(cost.begin(), cost.end());
    EXPECT(orc_mcf(n, m, s64.data(), d64.data(), c64.data(), sup.data(), nullptr, nullptr) == r.cost);
    // CSR form (sorted by tail, then head), 32- and 64-bit costs
    std::vector<int64_t> order((size_t)m);
    for (int64_t k = 0; k < m; ++k) order[(size_t)k] = k;
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
      return src[(size_t)a] != src[(size_t)b] ? src[(size_t)a] < src[(size_t)b] : dst[(size_t)a] < dst[(size_t)b];
    });
    std::vector<int64_t> rp((size_t)n + 1, 0);
    std::vector<uint32_t> col((size_t)m);
    std::vector<int32_t> cc((size_t)m);
    std::vector<int64_t> cc64((size_t)m);
    for (int64_t k = 0; k < m; ++k) {
      const int64_t a = order[(size_t)k];
      rp[src[(size_t)a] + 1]++;
      col[(size_t)k] = dst[(size_t)a];
      cc[(size_t)k] = cost[(size_t)a];
      cc64[(size_t)k] = cost[(size_t)a];
    }
    for (int64_t v = 0; v < n; ++v) rp[(size_t)v + 1] += rp[(size_t)v];
    w1::FlowResult r2{}, r3{};
    EXPECT(w1::network_simplex(n, rp.data(), col.data(), cc.data(), sup.data(), 0, &r2) == 0);
    EXPECT(w1::network_simplex64(n, rp.data(), col.data(), cc64.data(), sup.data(), 0, &r3) == 0);
    EXPECT(r2.cost == r.cost && r3.cost == r.cost);
    // a pivot cap stops early without reading or writing out of bounds
    for (int64_t cap = 1; cap < 6; ++cap) {
      w1::FlowResult rc{};
      std::vector<int64_t> f2((size_t)m);
      rc.flow = f2.data();
      EXPECT(w1::network_simplex(n, rp.data(), col.data(), cc.data(), sup.data(), cap, &rc) == 0);
      EXPECT(rc.pivots <= cap);
    }
    // unbalanced supplies are rejected
    std::vector<int64_t> bad = sup;
    bad[0] += 1;
    w1::FlowResult rb{};
    EXPECT(w1::network_simplex_arcs(n, m, src.data(), dst.data(), cost.data(), bad.data(), 0, &rb) != 0);
  }
}

static void oracle_modes(std::mt19937_64& rng) {
  std::uniform_real_distribution<double> U(0.0, 1.0);
  std::exponential_distribution<double> E(20.0);
  const int flags_list[] = {0, 32, 64, 2, 4, 8, 8 | 32, 8 | 64, 128, 128 | 64, 16};
  for (int trial = 0; trial < 40; ++trial) {
    const int64_t nA = (int64_t)(rng() % 60), nB = (int64_t)(rng() % 50);
    std::vector<double> A((size_t)(2 * nA)), B((size_t)(2 * nB));
    for (int64_t k = 0; k < nA; ++k) {
      A[(size_t)(2 * k)] = U(rng);
      A[(size_t)(2 * k + 1)] = A[(size_t)(2 * k)] + (trial % 5 == 0 ? 0.0 : E(rng));
    }
    for (int64_t k = 0; k < nB; ++k) {
      B[(size_t)(2 * k)] = U(rng);
      B[(size_t)(2 * k + 1)] = B[(size_t)(2 * k)] + E(rng);
    }
    if (nA > 3 && nB > 3) {  // shared points cancel
      B[0] = A[0];
      B[1] = A[1];
    }
    for (int flags : flags_list) {
      const int s = (flags & 128) ? 1 + (int)(rng() % 20) : (trial % 4 == 0 ? 2 : 0);
      void* o = orc_new();
      const int st = orc_run(o, A.data(), nA, B.data(), nB, 0.2, 0.1, s, flags, (flags & 16) ? 0.5 : 0.0);
      if (st == 0 && orc_i64(o, K_N) > 0) {
        const int64_t nl = orc_i64(o, K_NLOC), nc = orc_i64(o, K_NCELLS), nn = orc_i64(o, K_NNODES);
        std::vector<double> b((size_t)nl), d((size_t)nl), t((size_t)nl), term((size_t)nl);
        std::vector<int64_t> w((size_t)nl);
        orc_locs(o, b.data(), d.data(), w.data(), t.data(), term.data());
        std::vector<int64_t> ci((size_t)nc), cj((size_t)nc), ca((size_t)nc), cb((size_t)nc);
        std::vector<uint64_t> key((size_t)nc);
        orc_cells(o, ci.data(), cj.data(), ca.data(), cb.data(), key.data());
        std::vector<int64_t> nodes((size_t)(10 * nn));
        orc_nodes(o, nodes.data());
        double stage[7];
        orc_stage_seconds(o, stage);
        if (!(flags & (1 | 2)) && nc > 0) {  // pairs and networks exist
          const int64_t P = orc_i64(o, K_NPAIRS);
          std::vector<int64_t> u((size_t)P), v((size_t)P), c((size_t)P), nu((size_t)P), nv((size_t)P);
          orc_pairs(o, u.data(), v.data(), c.data(), (flags & 8) ? nu.data() : nullptr,
                    (flags & 8) ? nv.data() : nullptr);
          const int64_t m = orc_network(o, nullptr, nullptr, nullptr, nullptr);
          std::vector<int64_t> src((size_t)m), dst((size_t)m), cost((size_t)m), sup((size_t)(nc + 2));
          EXPECT(orc_network(o, src.data(), dst.data(), cost.data(), sup.data()) == m);
          const int64_t mc = orc_csr(o, nullptr, nullptr, nullptr);
          std::vector<int64_t> rp((size_t)(nc + 3)), col((size_t)mc), cc((size_t)mc);
          EXPECT(orc_csr(o, rp.data(), col.data(), cc.data()) == mc && mc == m);
        }
      }
      orc_free(o);
    }
  }
}

// The warm start from the flow through the diagonal gives the optimum of the
// artificial start on the method's own networks (every metric and mode),
// with optimality certificates, and never stalls with supply unrouted.
static void warm_starts(std::mt19937_64& rng) {
  std::uniform_real_distribution<double> U(0.0, 1.0);
  std::exponential_distribution<double> E(15.0);
  int64_t piv_cold = 0, piv_warm = 0, arcs_all = 0, arcs_kept = 0;
  const int flags_list[] = {4, 4 | 32, 4 | 64};
  for (int trial = 0; trial < 24; ++trial) {
    const int64_t nA = 1 + (int64_t)(rng() % 120), nB = (int64_t)(rng() % 100);
    std::vector<double> A((size_t)(2 * nA)), B((size_t)(2 * nB));
    for (int64_t k = 0; k < nA; ++k) {
      A[(size_t)(2 * k)] = U(rng);
      A[(size_t)(2 * k + 1)] = A[(size_t)(2 * k)] + E(rng);
    }
    for (int64_t k = 0; k < nB; ++k) {
      B[(size_t)(2 * k)] = U(rng);
      B[(size_t)(2 * k + 1)] = B[(size_t)(2 * k)] + E(rng);
    }
    if (nA > 5 && nB > 5)
      for (int k = 0; k < 4; ++k) {  // shared cells (mixed supply) and cancellations
        B[(size_t)(2 * k)] = A[(size_t)(2 * k)];
        B[(size_t)(2 * k + 1)] = A[(size_t)(2 * k + 1)] + (k & 1 ? 1e-9 : 0.0);
      }
    for (int flags : flags_list) {
      void* o = orc_new();
      const int st = orc_run(o, A.data(), nA, B.data(), nB, trial % 2 ? 0.1 : 0.3, 0.1, trial % 5 == 0 ? 2 : 0,
                             flags, 0.0);
      if (st == 0 && orc_i64(o, K_N) > 0) {
        const int64_t nc = orc_i64(o, K_NCELLS);
        const int64_t m = orc_csr(o, nullptr, nullptr, nullptr);
        std::vector<int64_t> rp((size_t)(nc + 3)), c64((size_t)m), cc((size_t)m);
        EXPECT(orc_csr(o, rp.data(), c64.data(), cc.data()) == m);
        std::vector<int64_t> src((size_t)m), dst((size_t)m), cost((size_t)m), sup((size_t)(nc + 2));
        orc_network(o, src.data(), dst.data(), cost.data(), sup.data());
        std::vector<uint32_t> col(c64.begin(), c64.end());
        const int64_t nn = nc + 2;
        std::vector<int64_t> flow((size_t)m), pot((size_t)nn);
        w1::FlowResult cold{}, warm{};
        warm.flow = flow.data();
        warm.pot = pot.data();
        if (flags & 64) {
          EXPECT(w1::network_simplex64(nn, rp.data(), col.data(), cc.data(), sup.data(), 0, &cold) == 0);
          EXPECT(w1::network_simplex64_diag(nn, rp.data(), col.data(), cc.data(), sup.data(), 0, &warm) == 0);
        } else {
          std::vector<int32_t> c32(cc.begin(), cc.end());
          EXPECT(w1::network_simplex(nn, rp.data(), col.data(), c32.data(), sup.data(), 0, &cold) == 0);
          EXPECT(w1::network_simplex_diag(nn, rp.data(), col.data(), c32.data(), sup.data(), 0, &warm) == 0);
          // a stalled warm solve still routes every supply (it starts feasible)
          w1::FlowResult cap{};
          EXPECT(w1::network_simplex_diag(nn, rp.data(), col.data(), c32.data(), sup.data(), 3, &cap) == 0);
          EXPECT(cap.feasible == 1 && cap.cost >= cold.cost);
        }
        EXPECT(warm.status == 0 && cold.status == 0 && warm.cost == cold.cost);
        // the library's solve without the dominated cell arcs: the same optimum
        std::vector<int64_t> ci64((size_t)nc), cj64((size_t)nc), ca64((size_t)nc), cb64((size_t)nc);
        std::vector<uint64_t> key((size_t)nc);
        orc_cells(o, ci64.data(), cj64.data(), ca64.data(), cb64.data(), key.data());
        std::vector<int32_t> ci(ci64.begin(), ci64.end()), cj(cj64.begin(), cj64.end());
        w1::FlowResult red{};
        int64_t kept = 0;
        if (flags & 64) {
          w1::SolveRows<int64_t> sr;
          w1::drop_dominated_arcs(nc, rp.data(), col.data(), cc.data(), ci.data(), cj.data(), (int)orc_i64(o, K_COSTK),
                                  sr);
          EXPECT(w1::network_simplex64_diag(nn, sr.row_ptr.data(), sr.col.data(), sr.cost.data(), sup.data(), 0, &red) ==
                 0);
          kept = (int64_t)sr.col.size();
        } else {
          std::vector<int32_t> c32(cc.begin(), cc.end());
          w1::SolveRows<int32_t> sr;
          w1::drop_dominated_arcs(nc, rp.data(), col.data(), c32.data(), ci.data(), cj.data(), -1, sr);
          EXPECT(w1::network_simplex_diag(nn, sr.row_ptr.data(), sr.col.data(), sr.cost.data(), sup.data(), 0, &red) == 0);
          kept = (int64_t)sr.col.size();
        }
        EXPECT(red.status == 0 && red.cost == cold.cost && kept <= m);
        arcs_all += m;
        arcs_kept += kept;
        std::vector<int64_t> bal((size_t)nn, 0);
        for (int64_t v = 0; v < nn; ++v)
          for (int64_t a = rp[(size_t)v]; a < rp[(size_t)v + 1]; ++a) {
            EXPECT(flow[(size_t)a] >= 0);
            bal[(size_t)v] += flow[(size_t)a];
            bal[(size_t)col[(size_t)a]] -= flow[(size_t)a];
            const int64_t red = cc[(size_t)a] + pot[(size_t)v] - pot[(size_t)col[(size_t)a]];
            EXPECT(red >= 0 && (flow[(size_t)a] == 0 || red == 0));
          }
        for (int64_t v = 0; v < nn; ++v) EXPECT(bal[(size_t)v] == sup[(size_t)v]);
        piv_cold += cold.pivots;
        piv_warm += warm.pivots;
      }
      orc_free(o);
    }
  }
  std::printf("pivots: artificial start %lld, diagonal start %lld\n", (long long)piv_cold, (long long)piv_warm);
  std::printf("arcs: %lld, kept without the dominated cell arcs %lld\n", (long long)arcs_all, (long long)arcs_kept);
  EXPECT(arcs_kept < arcs_all);
  {
    // edge cases of the filter: no cells (only the two diagonal nodes), and
    // a hand network where one cell arc costs exactly d(u) + d(v) (dropped),
    // one less (kept), and arcs touching a diagonal node (always kept)
    const int64_t rp0[3] = {0, 0, 0};
    w1::SolveRows<int32_t> e;
    w1::drop_dominated_arcs(0, rp0, nullptr, (const int32_t*)nullptr, nullptr, nullptr, -1, e);
    EXPECT(e.row_ptr.size() == 3 && e.row_ptr[2] == 0 && e.col.empty() && e.cost.empty());
    const int64_t rp[5] = {0, 2, 3, 3, 4};
    const uint32_t cl[4] = {1, 2, 0, 0};
    const int32_t cs[4] = {6, 4, 5, 4};
    const int32_t ci[2] = {0, 1}, cj[2] = {4, 3};  // d = 4 and 2
    w1::SolveRows<int32_t> h;
    w1::drop_dominated_arcs(2, rp, cl, cs, ci, cj, -1, h);
    EXPECT(h.row_ptr.size() == 5 && h.row_ptr[1] == 1 && h.row_ptr[2] == 2 && h.row_ptr[3] == 2 && h.row_ptr[4] == 3);
    EXPECT(h.col.size() == 3 && h.col[0] == 2 && h.col[1] == 0 && h.col[2] == 0);
    EXPECT(h.cost[0] == 4 && h.cost[1] == 5 && h.cost[2] == 4);
  }
}

int main() {
  std::mt19937_64 rng(12345);
  flows(rng);
  oracle_modes(rng);
  warm_starts(rng);
  if (fails) return 1;
  std::printf("sanitized host checks ok\n");
  return 0;
}

"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values
derived by hand (tests/golden), closed forms, brute force on tiny inputs,
independent solvers (scipy Hungarian, networkx network simplex), LP duality
certificates, invariances and the approximation theorems.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import pdsynth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ------------------------------------------------------------- exact W1 --
def test_exact_w1_matches_bruteforce(orc):
    rng = np.random.default_rng(5)
    for trial in range(40):
        na, nb = rng.integers(0, 4, 2)
        A = pdsynth.exp_pd(int(na), 1000 + trial, mean_pers=0.3)
        B = pdsynth.exp_pd(int(nb), 2000 + trial, mean_pers=0.3)
        assert orc.exact_w1(A, B) == pytest.approx(orc.brute_w1(A, B), rel=1e-12, abs=1e-12)


def test_exact_w1_closed_forms(orc):
    p = np.array([[0.25, 1.75]])
    q = np.array([[0.5, 1.5]])
    assert orc.exact_w1(p, np.zeros((0, 2))) == 0.75  # (d-b)/2
    # one point each: min(direct, both to the diagonal)
    assert orc.exact_w1(p, q) == min(0.25, 0.75 + 0.5)
    far = np.array([[10.0, 10.5]])
    assert orc.exact_w1(p, far) == 0.75 + 0.25
    A = pdsynth.exp_pd(30, 3)
    assert orc.exact_w1(A, A) == 0.0
    B = pdsynth.exp_pd(25, 4)
    assert orc.exact_w1(A, B) == pytest.approx(orc.exact_w1(B, A), rel=1e-14)


def test_exact_w1_emd_reduction(orc):
    # Translating equal-size diagrams far from the diagonal makes every point
    # cheaper to match than to send to the diagonal, so W1 equals the plain
    # optimal assignment (EMD) of the two point sets (Sec. 6, conditional
    # lower bound reduction).
    from scipy.optimize import linear_sum_assignment

    rng = np.random.default_rng(11)
    for trial in range(5):
        P = rng.random((12, 2))
        Q = rng.random((12, 2))
        M = 100.0
        A = np.stack([P[:, 0] - M, P[:, 1] + M], 1)
        B = np.stack([Q[:, 0] - M, Q[:, 1] + M], 1)
        C = np.maximum(np.abs(P[:, None, 0] - Q[None, :, 0]), np.abs(P[:, None, 1] - Q[None, :, 1]))
        r, c = linear_sum_assignment(C)
        assert orc.exact_w1(A, B) == pytest.approx(C[r, c].sum(), rel=1e-12)


def test_exact_w1_net_invariance(orc):
    A = pdsynth.exp_pd(20, 7)
    B = pdsynth.exp_pd(18, 8)
    C = pdsynth.exp_pd(10, 9)
    assert orc.exact_w1(np.concatenate([A, C]), np.concatenate([B, C])) == pytest.approx(orc.exact_w1(A, B), rel=1e-12)


# ------------------------------------------------------------ min-cost flow --
def _certificate(n, src, dst, cost, supply, flow, pot):
    bal = np.zeros(n, np.int64)
    np.add.at(bal, src, flow)
    np.add.at(bal, dst, -flow)
    assert np.array_equal(bal, supply), "flow conservation"
    assert (flow >= 0).all()
    red = cost - pot[src] + pot[dst]
    assert (red >= 0).all(), "dual feasibility"
    assert (red[flow > 0] == 0).all(), "complementary slackness"
    assert int((cost * flow).sum()) == int((supply * pot).sum()), "strong duality"


def test_mcf_against_networkx_and_certificate(orc):
    import networkx as nx

    rng = np.random.default_rng(3)
    for trial in range(15):
        n = int(rng.integers(5, 40))
        m = int(rng.integers(n, 6 * n))
        src = rng.integers(0, n, m)
        dst = rng.integers(0, n, m)
        keep = src != dst
        src, dst = src[keep], dst[keep]
        # a spanning cycle keeps every instance feasible
        src = np.concatenate([src, np.arange(n)])
        dst = np.concatenate([dst, (np.arange(n) + 1) % n])
        cost = rng.integers(0, 50, src.shape[0])
        supply = rng.integers(-5, 6, n)
        supply[-1] -= supply.sum()
        c, flow, pot = orc.mcf(n, src, dst, cost, supply, want_certificate=True)
        _certificate(n, src, dst, cost, supply, flow, pot)
        G = nx.MultiDiGraph()
        for v in range(n):
            G.add_node(v, demand=-int(supply[v]))
        for k in range(src.shape[0]):
            G.add_edge(int(src[k]), int(dst[k]), weight=int(cost[k]))
        assert c == nx.network_simplex(G)[0]


def _g_ab(A, B):
    """Dense 0-condensed network G(A, B) of Sec. 4.3 with costs doubled
    (integer diagrams make every doubled cost an integer)."""
    A = np.asarray(A, np.float64)
    B = np.asarray(B, np.float64)
    ua, ca = np.unique(A, axis=0, return_counts=True)
    ub, cb = np.unique(B, axis=0, return_counts=True)
    na, nb = ua.shape[0], ub.shape[0]
    abar, bbar = na + nb, na + nb + 1
    src, dst, cost = [], [], []
    for x in range(na):
        for y in range(nb):
            src.append(x); dst.append(na + y)
            cost.append(int(2 * max(abs(ua[x, 0] - ub[y, 0]), abs(ua[x, 1] - ub[y, 1]))))
        src.append(x); dst.append(abar); cost.append(int(ua[x, 1] - ua[x, 0]))
    for y in range(nb):
        src.append(bbar); dst.append(na + y); cost.append(int(ub[y, 1] - ub[y, 0]))
    src.append(bbar); dst.append(abar); cost.append(0)
    supply = np.concatenate([ca, -cb, [-ca.sum(), cb.sum()]]).astype(np.int64)
    return na + nb + 2, np.array(src), np.array(dst), np.array(cost), supply


def test_matching_equals_flow(orc):
    # Prop. (matching <=> flow): the min-cost flow on the 0-condensed network
    # G(A, B) equals the min-weight perfect matching on Bi(A, B).
    for seed in range(8):
        A = pdsynth.integer_pd(25, 100 + seed, hi=8)
        B = pdsynth.integer_pd(20, 200 + seed, hi=8)
        n, src, dst, cost, supply = _g_ab(A, B)
        assert orc.mcf(n, src, dst, cost, supply) == round(2 * orc.exact_w1(A, B))


# -------------------------------------------------------------------- RWMD --
def test_rwmd_golden(orc):
    g = gold("rwmd_small.json")
    r = orc.run(np.array(g["A"], float), np.array(g["B"], float), eps=0.1)
    assert r.LA == g["L_A"] and r.LB == g["L_B"] and r.L == g["L"]
    w = r.locs["w"]
    assert list(r.locs["t"][w > 0]) == g["t_A"]
    assert list(r.locs["t"][w < 0]) == g["t_B"]
    assert orc.exact_w1(g["A"], g["B"]) == g["exact_w1"]


def test_rwmd_single_point_closed_form(orc):
    r = orc.run(np.array([[0.5, 2.0]]), np.zeros((0, 2)), eps=0.1)
    assert r.L == 0.75 and r.LB == 0.0


def test_rwmd_fixed_point_rounds_down(orc):
    A = pdsynth.exp_pd(300, 21)
    B = pdsynth.exp_pd(280, 22)
    r = orc.run(A, B, eps=0.1, flags=orc.ORC_STOP_AFTER_TREE)
    w, term = r.locs["w"], r.locs["term"]
    for side, Lx, F in ((w > 0, r.LA, r.FA), (w < 0, r.LB, r.FB)):
        exact = sum(Fraction(x) for x in term[side])
        k = int(side.sum())
        assert Fraction(Lx) <= exact
        assert exact - Fraction(Lx) <= Fraction(k + 1, 2 ** F) + exact * Fraction(1, 2 ** 52)
    # A sum whose fixed-point total is exactly representable, so the final
    # conversion cannot hide a term rounded the wrong way: one unit diagonal
    # term and 200 terms of 2^-60 (each far below one fixed-point unit of
    # 2^-53).  Every small term drops, and L_A = 1 exactly, below the real sum.
    tiny = [[j * 2.0 ** -50, j * 2.0 ** -50 + 2.0 ** -59] for j in range(1, 201)]
    r = orc.run(np.array([[0.0, 2.0]] + tiny), np.zeros((0, 2)), eps=0.1, flags=orc.ORC_STOP_AFTER_TREE)
    assert r.FA == 53 and r.LA == 1.0 and Fraction(r.LA) < 1 + Fraction(200, 2 ** 60)


def test_rwmd_lower_bound_and_net(orc):
    for seed in range(30):
        A = pdsynth.exp_pd(12, 300 + seed, mean_pers=0.2)
        B = pdsynth.exp_pd(9, 400 + seed, mean_pers=0.2)
        r = orc.run(A, B, eps=0.1, flags=orc.ORC_STOP_AFTER_TREE)
        assert r.L <= orc.exact_w1(A, B) + 1e-15
    # co-located A and B points cancel (W1 depends on the net multiset only)
    A = pdsynth.exp_pd(40, 1)
    B = pdsynth.exp_pd(30, 2)
    C = A[:10]
    r1 = orc.run(A, B, flags=orc.ORC_STOP_AFTER_TREE)
    r2 = orc.run(np.concatenate([A, C, C]), np.concatenate([B, C, C]), flags=orc.ORC_STOP_AFTER_TREE)
    assert r1.L == r2.L and r1.n == r2.n


def _brute_nn_t(b, d, w):
    """RWMD per-location cost by exhaustive search: the cheapest arc out of
    each location is to the nearest location of the other diagram (all of
    them, O(n^2)) or to the diagonal, (d - b)/2 (Alg. 1 with the diagonal
    arc of the text)."""
    t = 0.5 * (d - b)
    for side in (w > 0, w < 0):
        other = ~side & (w != 0)
        if not other.any():
            continue
        D = np.maximum(np.abs(b[side, None] - b[None, other]), np.abs(d[side, None] - d[None, other]))
        t[side] = np.minimum(D.min(axis=1), t[side])
    return t


@pytest.mark.parametrize("case", ["mixture", "integer_ties", "dense_cluster"])
def test_rwmd_nearest_neighbour_bruteforce(orc, case):
    # The oracle's nearest-neighbour search is a pruned sweep in birth order;
    # an exhaustive O(n^2) scan must give bit-identical costs: every entry is
    # the same IEEE max/abs/halving of the same FP64 inputs.
    if case == "mixture":
        A, B = pdsynth.mixture_pd(2500, 31), pdsynth.mixture_pd(2200, 32)
    elif case == "integer_ties":  # many equidistant candidates and diagonal ties
        A, B = pdsynth.integer_pd(1800, 33, hi=60), pdsynth.integer_pd(1700, 34, hi=60)
    else:  # thousands of points in a tiny box next to a sparse background
        rng = np.random.default_rng(35)
        cl = lambda n: np.stack([0.5 + 1e-6 * rng.random(n), 0.7 + 1e-6 * rng.random(n)], axis=1)
        A = np.concatenate([cl(1500), pdsynth.exp_pd(300, 36)])
        B = np.concatenate([cl(1400), pdsynth.exp_pd(250, 37)])
    r = orc.run(A, B, eps=0.1, flags=orc.ORC_STOP_AFTER_TREE)
    b, d, w = r.locs["b"], r.locs["d"], r.locs["w"]
    assert (w > 0).sum() > 100 and (w < 0).sum() > 100
    t = _brute_nn_t(b, d, w)
    assert np.array_equal(r.locs["t"], t)
    assert np.array_equal(r.locs["term"], np.abs(w) * t)


# ------------------------------------------------------------------ params --
def test_params_golden(orc):
    g = gold("params.json")
    for eps, s in g["s_table"].items():
        assert orc.choose_s(float(eps)) == s
    c = g["grid_case"]
    assert orc.grid_exponent(c["eps_c"], c["L"], c["n"]) == c["e"]


def test_params_minimal_s(orc):
    for eps in np.linspace(0.01, 0.9, 40):
        s = orc.choose_s(eps)
        ec = 0.1 * eps
        t = (s + 2) / (s - 2)
        assert t + (t + 1) * ec <= 1 + eps
        if s > 3:
            t1 = (s + 1) / (s - 3)
            assert t1 + (t1 + 1) * ec > 1 + eps


# -------------------------------------------------------------------- grid --
def test_grid_counts_and_node_drop(orc):
    A = pdsynth.pareto_pd(3000, 5)
    B = pdsynth.pareto_pd(2500, 6)
    r = orc.run(A, B, eps=0.5, flags=orc.ORC_STOP_AFTER_TREE)
    assert r.cells["cA"].sum() == r.nA and r.cells["cB"].sum() == r.nB
    # node-drop identity: the cells are exactly the distinct floor cells
    pts = np.concatenate([r.locs["b"], r.locs["d"]]).reshape(2, -1).T
    cellset = np.unique(np.floor(np.ldexp(pts, -r.e)).astype(np.int64), axis=0)
    assert cellset.shape[0] == r.cells["i"].shape[0]
    assert (r.cells["j"] >= r.cells["i"]).all()
    assert (np.diff(r.cells["key"].astype(np.float64)) > 0).all()


def test_scale_and_translation_invariance(orc):
    A = pdsynth.integer_pd(60, 1, hi=40) * 2.0 ** -8
    B = pdsynth.integer_pd(50, 2, hi=40) * 2.0 ** -8
    r = orc.run(A, B, eps=0.2)
    for k in (-3, 5):
        rk = orc.run(A * 2.0 ** k, B * 2.0 ** k, eps=0.2)
        assert rk.e == r.e + k and rk.W1 == r.W1 * 2.0 ** k and rk.flow == r.flow
        for f in ("i", "j", "cA", "cB"):
            assert np.array_equal(rk.cells[f], r.cells[f])
        assert np.array_equal(rk.pairs["u"], r.pairs["u"]) and np.array_equal(rk.pairs["v"], r.pairs["v"])
    shift = 37 * 2.0 ** r.e
    rt = orc.run(A + shift, B + shift, eps=0.2)
    assert rt.W1 == r.W1 and rt.flow == r.flow
    for f in ("i", "j", "cA", "cB"):
        assert np.array_equal(rt.cells[f], r.cells[f])


# -------------------------------------------------------------------- tree --
def test_tree_invariants(orc):
    A = pdsynth.mixture_pd(700, 3)
    B = pdsynth.mixture_pd(650, 4)
    r = orc.run(A, B, eps=0.2, flags=orc.ORC_STOP_AFTER_TREE)
    N = r.cells["i"].shape[0]
    nodes, key = r.nodes, r.cells["key"]
    assert nodes.shape[0] == 2 * N - 1
    seen = np.zeros(2 * N - 1, np.int64)
    for k in range(N, 2 * N - 1):
        lo, hi, l, rr, m = nodes[k, :5]
        seen[l] += 1
        seen[rr] += 1
        assert nodes[l, 0] == lo and nodes[l, 1] == m and nodes[rr, 0] == m + 1 and nodes[rr, 1] == hi
        x = int(key[lo]) ^ int(key[hi])
        bit = x.bit_length() - 1
        assert all(((int(key[q]) >> bit) & 1) == (q > m) for q in range(lo, hi + 1))
        ii, jj = r.cells["i"][lo:hi + 1], r.cells["j"][lo:hi + 1]
        assert tuple(nodes[k, 5:9]) == (ii.min(), jj.min(), ii.max(), jj.max())
        assert nodes[k, 9] == max(ii.max() - ii.min(), jj.max() - jj.min())
    assert seen[r.root] == 0 and (np.delete(seen, r.root) == 1).all()


# -------------------------------------------------------------------- WSPD --
@pytest.mark.parametrize("s_override", [1, 2, 3, 5, 12, 53])
def test_wspd_bruteforce_coverage(orc, s_override):
    for seed in range(3):
        A = pdsynth.exp_pd(24, 50 + seed, mean_pers=0.3)
        B = pdsynth.exp_pd(22, 60 + seed, mean_pers=0.3)
        r = orc.run(A, B, eps=0.2, s_override=s_override, flags=orc.ORC_KEEP_PAIR_NODES | orc.ORC_NO_FLOW)
        assert r.cells["i"].shape[0] >= 30
        orc.wspd_coverage(r)


def _check_csr(orc, r, net):
    """Checks of the network in compressed sparse row form against the cells
    and the WSPD pairs of the same run (Sec. 5.3 network, Alg. 7 diagonal
    arcs, Appendix network representation)."""
    N = r.cells["i"].shape[0]
    rp, col, cost = net["row_ptr"], net["col"], net["cost"]
    ci, cj, cA, cB = r.cells["i"], r.cells["j"], r.cells["cA"], r.cells["cB"]
    assert net["n_cells"] == N and rp.shape == (N + 3,)
    assert rp[0] == 0 and (np.diff(rp) >= 0).all() and rp[-1] == col.size == cost.size
    tail = np.repeat(np.arange(N + 2), np.diff(rp))
    # sorted by (tail, head) with no repeated arc
    key = tail * (N + 2) + col
    assert (np.diff(key) > 0).all()
    # arc-count identity: both directions of each pair, one diagonal arc per
    # A cell and per B cell, and the B-diagonal -> A-diagonal arc
    assert col.size == 2 * r.n_pairs + (cA > 0).sum() + (cB > 0).sum() + 1
    # cell-cell arcs are exactly the two orientations of the WSPD pairs, with
    # cost 2 max(|di|, |dj|) in units of g/2 recomputed from the cells
    cc = (tail < N) & (col < N)
    pairs = set(zip(r.pairs["u"].tolist(), r.pairs["v"].tolist()))
    assert set(zip(tail[cc].tolist(), col[cc].tolist())) == pairs | {(v, u) for u, v in pairs}
    assert cc.sum() == 2 * len(pairs)
    t, h = tail[cc], col[cc]
    assert (cost[cc] == 2 * np.maximum(np.abs(ci[t] - ci[h]), np.abs(cj[t] - cj[h]))).all()
    # diagonal arcs by membership; cost = distance to the diagonal, j - i
    toA = (tail < N) & (col == N)
    assert np.array_equal(tail[toA], np.flatnonzero(cA > 0))
    assert (cost[toA] == cj[tail[toA]] - ci[tail[toA]]).all()
    assert rp[N + 1] == rp[N]  # the A-diagonal node sends nothing
    bb = col[rp[N + 1]:rp[N + 2]]
    assert np.array_equal(bb, np.append(np.flatnonzero(cB > 0), N))
    assert (cost[rp[N + 1]:rp[N + 2] - 1] == cj[bb[:-1]] - ci[bb[:-1]]).all() and cost[rp[N + 2] - 1] == 0
    assert np.array_equal(net["supply"], np.concatenate([cA - cB, [-r.nA, r.nB]]))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_csr_network(orc, seed):
    # small: the pairs themselves are pinned by brute-force coverage
    A = pdsynth.exp_pd(24, 500 + seed, mean_pers=0.3)
    B = pdsynth.exp_pd(22, 600 + seed, mean_pers=0.3)
    r = orc.run(A, B, eps=0.2, flags=orc.ORC_KEEP_PAIR_NODES | orc.ORC_NO_FLOW)
    orc.wspd_coverage(r)
    _check_csr(orc, r, orc.csr(A, B, eps=0.2))
    # medium, FP32 mixture with overlapping A/B cells
    A, B = pdsynth.mixture_pd(900, 700 + seed), pdsynth.mixture_pd(800, 710 + seed)
    r = orc.run(A, B, eps=0.1, flags=orc.ORC_NO_FLOW)
    _check_csr(orc, r, orc.csr(A, B, eps=0.1))
    # the sorted network has the optimum of the arc list it sorts
    A, B = pdsynth.exp_pd(150, 720 + seed), pdsynth.exp_pd(140, 730 + seed)
    net = orc.csr(A, B, eps=0.1)
    rp = net["row_ptr"]
    tail = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    full = orc.run(A, B, eps=0.1)
    assert orc.mcf(rp.size - 1, tail, net["col"], net["cost"], net["supply"]) == full.flow


def test_csr_network_edges(orc):
    # identical diagrams: nothing to ship
    A = pdsynth.exp_pd(30, 1)
    net = orc.csr(A, A.copy(), eps=0.1)
    assert net["n_cells"] == 0 and net["col"].size == 0 and list(net["row_ptr"]) == [0, 0, 0]
    # one point against nothing: one cell, its A-diagonal arc and B->A
    net = orc.csr(np.array([[0.25, 1.75]]), np.zeros((0, 2)), eps=0.1)
    assert list(net["row_ptr"]) == [0, 1, 1, 2]
    assert list(net["col"]) == [1, 1] and net["cost"][1] == 0


@pytest.mark.parametrize("s_override", [1, 2, 3])
def test_small_s_still_upper_bound(orc, s_override):
    # With no stretch bound (s <= 2) the sparse network still only holds
    # real arcs between cell representatives, so its optimum is at least the
    # complete network's and the output stays above the exact W1 (Sec. 5.5
    # and the condensation bound of Sec. 5.1).
    for seed in range(4):
        A = pdsynth.exp_pd(40, 80 + seed, mean_pers=0.2)
        B = pdsynth.exp_pd(36, 90 + seed, mean_pers=0.2)
        r = orc.run(A, B, eps=0.2, s_override=s_override)
        assert r.status == 0 and r.s == s_override
        assert r.W1 >= orc.exact_w1(A, B) * (1 - 1e-12)
        # A pair separated at s is separated at any smaller s, so the same
        # traversal stops no later: the pair count cannot drop as s grows.
        r2 = orc.run(A, B, eps=0.2, s_override=s_override + 1, flags=orc.ORC_NO_FLOW)
        assert 0 < r.n_pairs <= r2.n_pairs


@pytest.mark.parametrize("s_override", [4, 9, 28])
def test_wspd_spanner_stretch(orc, s_override):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import shortest_path

    A = pdsynth.exp_pd(80, 70, mean_pers=0.2)
    B = pdsynth.exp_pd(70, 71, mean_pers=0.2)
    r = orc.run(A, B, eps=0.2, s_override=s_override, flags=orc.ORC_NO_FLOW)
    N = r.cells["i"].shape[0]
    u, v, c = r.pairs["u"], r.pairs["v"], r.pairs["c"]
    G = coo_matrix((c.astype(float), (u, v)), shape=(N, N)).tocsr()
    D = shortest_path(G, directed=False)
    ci, cj = r.cells["i"], r.cells["j"]
    direct = 2 * np.maximum(np.abs(ci[:, None] - ci[None, :]), np.abs(cj[:, None] - cj[None, :]))
    t = (s_override + 2) / (s_override - 2)
    off = ~np.eye(N, dtype=bool)
    assert (D[off] <= t * direct[off] + 1e-9).all()
    assert (D[off] >= direct[off] - 1e-9).all()


# --------------------------------------------------------------- theorems --
def _dense_gdelta_flow(orc, r):
    """Min-cost flow on the bipartite condensed network G_delta (A cells and
    B cells as separate nodes, all A-B arcs), costs in units of g/2."""
    ci, cj, ca, cb = r.cells["i"], r.cells["j"], r.cells["cA"], r.cells["cB"]
    ia, ib = np.nonzero(ca)[0], np.nonzero(cb)[0]
    na, nb = ia.shape[0], ib.shape[0]
    abar, bbar = na + nb, na + nb + 1
    X, Y = np.meshgrid(np.arange(na), np.arange(nb), indexing="ij")
    src = [X.ravel()]
    dst = [na + Y.ravel()]
    cost = [2 * np.maximum(np.abs(ci[ia][X] - ci[ib][Y]), np.abs(cj[ia][X] - cj[ib][Y])).ravel()]
    src += [np.arange(na), np.full(nb, bbar), [bbar]]
    dst += [np.full(na, abar), na + np.arange(nb), [abar]]
    cost += [cj[ia] - ci[ia], cj[ib] - ci[ib], [0]]
    supply = np.concatenate([ca[ia], -cb[ib], [-ca.sum(), cb.sum()]])
    return orc.mcf(na + nb + 2, np.concatenate(src), np.concatenate(dst), np.concatenate(cost), supply)


def test_sparse_network_theorem(orc):
    # Thm. (WSPD network): f* <= fbar* <= t f* with t the spanner stretch.
    for seed, s in ((0, 4), (1, 6), (2, 12)):
        A = pdsynth.exp_pd(70, 500 + seed, mean_pers=0.2)
        B = pdsynth.exp_pd(60, 600 + seed, mean_pers=0.2)
        r = orc.run(A, B, eps=0.2, s_override=s)
        fd = _dense_gdelta_flow(orc, r)
        t = (s + 2) / (s - 2)
        assert fd <= r.flow <= t * fd + 1e-9


@pytest.mark.parametrize("eps", [0.2, 0.1, 0.05])
def test_bracket_small(orc, eps):
    # RWMD <= exact <= W1 <= (1+eps) exact; the paper's value lies within
    # [(1 - eps_c), (1 + eps)] of exact.
    for seed in range(12):
        A = pdsynth.exp_pd(45, 2 * seed)
        B = pdsynth.exp_pd(40, 2 * seed + 1)
        r = orc.run(A, B, eps=eps)
        ex = orc.exact_w1(A, B)
        assert r.L <= ex <= r.W1 <= (1 + eps) * ex
        assert (1 - r.eps_c) * ex <= r.W1_paper <= (1 + eps) * ex


def test_bracket_config1(orc):
    for k in range(2):
        A = pdsynth.exp_pd(400, 2 * k)
        B = pdsynth.exp_pd(400, 2 * k + 1)
        r = orc.run(A, B, eps=0.1)
        ex = orc.exact_w1(A, B)
        assert r.L <= ex <= r.W1 <= 1.1 * ex


def test_symmetry_and_net_invariance(orc):
    A = pdsynth.exp_pd(60, 31)
    B = pdsynth.exp_pd(55, 32)
    r = orc.run(A, B, eps=0.2)
    rs = orc.run(B, A, eps=0.2)
    assert rs.W1 == r.W1 and rs.flow == r.flow and rs.L == r.L
    C = pdsynth.exp_pd(20, 33)
    rc = orc.run(np.concatenate([A, C]), np.concatenate([C, B]), eps=0.2)
    assert rc.W1 == r.W1
    rz = orc.run(A, A.copy(), eps=0.2)
    assert rz.status == 0 and rz.W1 == 0.0 and rz.n == 0


def test_one_sided_and_invalid(orc):
    A = pdsynth.exp_pd(50, 41)
    r = orc.run(A, np.zeros((0, 2)), eps=0.1)
    exact = float(np.sum(0.5 * (A[:, 1] - A[:, 0])))
    assert r.L <= exact <= r.W1 <= 1.1 * exact
    assert orc.run(np.array([[1.0, 0.5]]), A).status == -1  # death < birth
    assert orc.run(np.array([[np.nan, 0.5]]), A).status == -1
    diag = np.array([[0.3, 0.3], [0.7, 0.7]])
    assert orc.run(np.concatenate([A, diag]), np.zeros((0, 2))).W1 == r.W1


# ------------------------------------------------- diagonal-dominance pruning --
def _dominated(nodes, U, V):
    """Box test of O7': 2 dist(U, V) >= (U.maxj - U.mini) + (V.maxj - V.mini),
    all in grid cells (node rows: lo, hi, left, right, split, mini, minj,
    maxi, maxj, diam)."""
    a, b = nodes[U], nodes[V]
    gi = max(a[5] - b[7], b[5] - a[7])
    gj = max(a[6] - b[8], b[6] - a[8])
    dist = max(0, gi, gj)
    return 2 * dist >= (a[8] - a[5]) + (b[8] - b[5])


@pytest.mark.parametrize("kind", ["exp", "mixture", "pareto", "integer", "one_sided"])
def test_prune_keeps_optimum(orc, kind):
    # Leaving out the diagonal-dominated pairs never changes F* (the rerouting
    # argument of O7'), so W1 and W1_paper are identical; the network shrinks.
    for seed in range(6):
        if kind == "exp":
            A, B = pdsynth.exp_pd(60 + 7 * seed, 900 + seed), pdsynth.exp_pd(50 + 5 * seed, 950 + seed)
        elif kind == "mixture":
            A, B = pdsynth.mixture_pd(300, 910 + seed), pdsynth.mixture_pd(280, 960 + seed)
        elif kind == "pareto":
            A, B = pdsynth.pareto_pd(200, 920 + seed), pdsynth.pareto_pd(220, 970 + seed)
        elif kind == "integer":
            A, B = pdsynth.integer_pd(40, 930 + seed), pdsynth.integer_pd(35, 980 + seed)
        else:
            A, B = pdsynth.exp_pd(70, 940 + seed), np.zeros((0, 2))
        for eps, s in ((0.1, 0), (0.2, 0), (0.2, 3)):
            full = orc.run(A, B, eps=eps, s_override=s, fetch=False)
            pr = orc.run(A, B, eps=eps, s_override=s, flags=orc.ORC_PRUNE, fetch=False)
            assert full.status == 0 and pr.status == 0
            assert pr.flow == full.flow and pr.W1 == full.W1 and pr.W1_paper == full.W1_paper
            assert pr.n_pairs <= full.n_pairs


@pytest.mark.parametrize("kind", ["exp", "mixture", "pareto", "integer", "one_sided"])
def test_arc_dominance_keeps_optimum(orc, kind):
    # Arc by arc: a cell arc u -> v with cost >= d(u) + d(v) (d = j - i, the
    # diagonal arc's cost) is never needed -- some optimal flow sends all of
    # B's diagonal node's surplus to A's directly, and a path through such an
    # arc is rerouted over its ends' diagonal arcs at no extra cost.  The
    # library's host flow solves the L-infinity network without these arcs;
    # here the oracle's own flow solves both networks and F* must agree.
    dropped = 0
    for seed in range(4):
        if kind == "exp":
            A, B = pdsynth.exp_pd(60 + 9 * seed, 1100 + seed), pdsynth.exp_pd(55 + 6 * seed, 1150 + seed)
        elif kind == "mixture":
            A, B = pdsynth.mixture_pd(250, 1110 + seed), pdsynth.mixture_pd(230, 1160 + seed)
        elif kind == "pareto":
            A, B = pdsynth.pareto_pd(180, 1120 + seed), pdsynth.pareto_pd(200, 1170 + seed)
        elif kind == "integer":
            A, B = pdsynth.integer_pd(40, 1130 + seed), pdsynth.integer_pd(35, 1180 + seed)
        else:
            A, B = pdsynth.exp_pd(70, 1140 + seed), np.zeros((0, 2))
        for eps, s, prune in ((0.1, 0, False), (0.2, 3, False), (0.2, 0, True)):
            r = orc.run(A, B, eps=eps, s_override=s, flags=orc.ORC_PRUNE if prune else 0)
            src, dst, cost, sup = orc.network(A, B, eps=eps, s_override=s, prune=prune)
            N = sup.shape[0] - 2
            d = (r.cells["j"] - r.cells["i"]).astype(np.int64)
            assert d.shape[0] == N
            cell = (src < N) & (dst < N)
            dom = np.zeros(src.shape[0], bool)
            dom[cell] = cost[cell] >= d[src[cell]] + d[dst[cell]]
            keep = ~dom
            f_full = orc.mcf(N + 2, src, dst, cost, sup)
            f_kept = orc.mcf(N + 2, src[keep], dst[keep], cost[keep], sup)
            assert f_full == f_kept == r.flow, (kind, seed, eps, s, prune)
            dropped += int(dom.sum())
    if kind != "one_sided":
        assert dropped > 0


@pytest.mark.parametrize("kind", ["exp", "mixture", "pareto"])
def test_arc_dominance_keeps_optimum_l2(orc, kind):
    # The same on the Euclidean network, whose costs are real distances
    # rounded up through double arithmetic: an arc is dropped when it costs at
    # least d(u) + d(v) + M, M = 3 + 2^-50 (n_cells + 3) max cost, d the
    # diagonal arc's rounded cost (the rounding slack carried through the
    # rerouting argument).  F* from the oracle's own flow must not change.
    import math

    dropped = 0
    for seed in range(3):
        if kind == "exp":
            A, B = pdsynth.exp_pd(60 + 9 * seed, 1200 + seed), pdsynth.exp_pd(55 + 6 * seed, 1250 + seed)
        elif kind == "mixture":
            A, B = pdsynth.mixture_pd(200, 1210 + seed), pdsynth.mixture_pd(190, 1260 + seed)
        else:
            A, B = pdsynth.pareto_pd(150, 1220 + seed), pdsynth.pareto_pd(160, 1270 + seed)
        for eps, s in ((0.1, 0), (0.2, 3)):
            r = orc.run(A, B, eps=eps, s_override=s, flags=orc.ORC_L2)
            src, dst, cost, sup = orc.network(A, B, eps=eps, s_override=s, l2=True)
            N = sup.shape[0] - 2
            K, R = r.K, float.fromhex("0x1.6a09e667f3bcdp-1")
            d = np.array([math.ceil(math.ldexp(float(int(j) - int(i)) * R, K))
                          for i, j in zip(r.cells["i"], r.cells["j"])], np.int64)
            M = 3 + math.ceil(math.ldexp(float(N + 3) * float(cost.max()), -50))
            cell = (src < N) & (dst < N)
            dom = np.zeros(src.shape[0], bool)
            dom[cell] = cost[cell] >= d[src[cell]] + d[dst[cell]] + M
            keep = ~dom
            assert orc.mcf(N + 2, src[keep], dst[keep], cost[keep], sup) == orc.mcf(N + 2, src, dst, cost, sup) == r.flow
            dropped += int(dom.sum())
    assert dropped > 0


def test_prune_pair_set_is_filtered_wspd(orc):
    # The recursion below a dominated pair is cut, and the test is monotone,
    # so the pruned pairs are exactly the s-WSPD pairs whose own boxes pass.
    for seed in range(4):
        A = pdsynth.exp_pd(90, 990 + seed, mean_pers=0.15)
        B = pdsynth.exp_pd(80, 995 + seed, mean_pers=0.15)
        fl = orc.ORC_KEEP_PAIR_NODES | orc.ORC_NO_FLOW
        full = orc.run(A, B, eps=0.2, flags=fl)
        pr = orc.run(A, B, eps=0.2, flags=fl | orc.ORC_PRUNE)
        keep = [k for k in range(full.n_pairs)
                if not _dominated(full.nodes, full.pairs["nu"][k], full.pairs["nv"][k])]
        want = sorted(zip(full.pairs["u"][keep].tolist(), full.pairs["v"][keep].tolist(),
                          full.pairs["c"][keep].tolist()))
        got = sorted(zip(pr.pairs["u"].tolist(), pr.pairs["v"].tolist(), pr.pairs["c"].tolist()))
        assert got == want and 0 < len(got) < full.n_pairs
        # every arc left out costs at least its two diagonal arcs together
        ci, cj = full.cells["i"], full.cells["j"]
        drop = np.setdiff1d(np.arange(full.n_pairs), keep)
        u, v, c = full.pairs["u"][drop], full.pairs["v"][drop], full.pairs["c"][drop]
        assert (c >= (cj[u] - ci[u]) + (cj[v] - ci[v])).all()


def test_prune_closed_forms(orc):
    # One point each, far apart relative to their persistence: the optimum
    # sends both to the diagonal, the only WSPD pair is dominated and left
    # out, and W1 is unchanged.  Close together: the pair stays.
    p = np.array([[0.0, 0.25]])
    for q, kept in ((np.array([[4.0, 4.5]]), 0), (np.array([[0.01, 0.27]]), 1)):
        full = orc.run(p, q, eps=0.1)
        pr = orc.run(p, q, eps=0.1, flags=orc.ORC_PRUNE)
        assert full.n_pairs == 1 and pr.n_pairs == kept
        assert pr.W1 == full.W1
        ex = orc.exact_w1(p, q)
        assert full.L <= ex <= pr.W1 <= 1.1 * ex


# ------------------------------------------------------ Euclidean metric --
R_SQRT1_2 = float.fromhex("0x1.6a09e667f3bcdp-1")


def test_l2_exact_w1_pins(orc):
    # closed forms: one point, (d - b)/sqrt(2); one point each, the cheaper
    # of matching them and sending both to the diagonal
    p, q = np.array([[0.25, 1.75]]), np.array([[0.5, 1.5]])
    assert orc.exact_w1(p, np.zeros((0, 2)), l2=True) == pytest.approx(1.5 / np.sqrt(2), rel=1e-15)
    assert orc.exact_w1(p, q, l2=True) == pytest.approx(min(np.hypot(0.25, 0.25), (1.5 + 1.0) / np.sqrt(2)), rel=1e-15)
    far = np.array([[10.0, 10.5]])
    assert orc.exact_w1(p, far, l2=True) == pytest.approx((1.5 + 0.5) / np.sqrt(2), rel=1e-15)
    rng = np.random.default_rng(15)
    for trial in range(30):
        na, nb = rng.integers(0, 4, 2)
        A = pdsynth.exp_pd(int(na), 3000 + trial, mean_pers=0.3)
        B = pdsynth.exp_pd(int(nb), 4000 + trial, mean_pers=0.3)
        assert orc.exact_w1(A, B, l2=True) == pytest.approx(orc.brute_w1(A, B, l2=True), rel=1e-12, abs=1e-12)
    # L-infinity <= Euclidean <= sqrt(2) L-infinity for the ground costs, and
    # the diagonal costs differ by the factor sqrt(2)/2 ... 1: W1 keeps order
    A, B = pdsynth.exp_pd(40, 5), pdsynth.exp_pd(35, 6)
    assert orc.exact_w1(A, B) <= orc.exact_w1(A, B, l2=True) * (1 + 1e-12)


@pytest.mark.parametrize("case", ["exp", "cluster", "ties"])
def test_l2_rwmd_nearest_neighbour_bruteforce(orc, case):
    # every location's cost t = min(sqrt(q_min), (d - b) R) against an
    # exhaustive scan with the same IEEE operations, bit for bit
    if case == "exp":
        A, B = pdsynth.exp_pd(700, 31), pdsynth.exp_pd(650, 32)
    elif case == "cluster":
        rng = np.random.default_rng(4)
        b = 0.5 + 1e-3 * rng.random(600)
        A = np.stack([b[:300], b[:300] + 0.2 + 1e-3 * rng.random(300)], 1)
        B = np.stack([b[300:], b[300:] + 0.2 + 1e-3 * rng.random(300)], 1)
    else:
        g = np.arange(12) * 0.25
        P = np.array([(x, y) for x in g for y in g if y > x])
        A, B = P[::2], P[1::2] + np.array([0.0, 0.125])
    r = orc.run(A, B, eps=0.1, flags=orc.ORC_L2 | orc.ORC_NO_FLOW)
    lb, ld, lw = r.locs["b"], r.locs["d"], r.locs["w"]
    for side in (1, -1):
        me, other = np.flatnonzero(np.sign(lw) == side), np.flatnonzero(np.sign(lw) == -side)
        gb = lb[me][:, None] - lb[other][None, :]
        gd = ld[me][:, None] - ld[other][None, :]
        q = gb * gb + gd * gd
        qmin = q.min(axis=1) if other.size else np.full(me.size, np.inf)
        t = np.minimum(np.sqrt(qmin), (ld[me] - lb[me]) * R_SQRT1_2)
        assert np.array_equal(t, r.locs["t"][me])


@pytest.mark.parametrize("eps", [0.2, 0.1, 0.05])
def test_l2_bracket(orc, eps):
    # RWMD <= exact <= W1 <= (1 + eps) exact with the Euclidean metric; the
    # paper's value within [(1 - eps_c), (1 + eps)] of exact
    for seed in range(10):
        A = pdsynth.exp_pd(45, 100 + 2 * seed)
        B = pdsynth.exp_pd(40, 101 + 2 * seed)
        r = orc.run(A, B, eps=eps, flags=orc.ORC_L2)
        ex = orc.exact_w1(A, B, l2=True)
        assert r.status == 0
        assert r.L <= ex * (1 + 1e-12) and ex <= r.W1 <= (1 + eps) * ex
        assert (1 - r.eps_c) * ex <= r.W1_paper <= (1 + eps) * ex
    A, B = pdsynth.exp_pd(400, 0), pdsynth.exp_pd(400, 1)
    r = orc.run(A, B, eps=eps, flags=orc.ORC_L2)
    ex = orc.exact_w1(A, B, l2=True)
    assert r.L <= ex <= r.W1 <= (1 + eps) * ex


@pytest.mark.parametrize("s_override", [1, 3, 12, 53])
def test_l2_wspd_coverage(orc, s_override):
    for seed in range(2):
        A = pdsynth.exp_pd(24, 150 + seed, mean_pers=0.3)
        B = pdsynth.exp_pd(22, 160 + seed, mean_pers=0.3)
        r = orc.run(A, B, eps=0.2, s_override=s_override,
                    flags=orc.ORC_L2 | orc.ORC_KEEP_PAIR_NODES | orc.ORC_NO_FLOW)
        assert r.cells["i"].shape[0] >= 30
        orc.wspd_coverage(r, l2=True)


@pytest.mark.parametrize("s_override", [4, 9, 28])
def test_l2_spanner_stretch(orc, s_override):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import shortest_path

    A = pdsynth.exp_pd(80, 170, mean_pers=0.2)
    B = pdsynth.exp_pd(70, 171, mean_pers=0.2)
    r = orc.run(A, B, eps=0.2, s_override=s_override, flags=orc.ORC_L2 | orc.ORC_NO_FLOW)
    N = r.cells["i"].shape[0]
    ci, cj = r.cells["i"].astype(float), r.cells["j"].astype(float)
    u, v = r.pairs["u"], r.pairs["v"]
    G = coo_matrix((np.hypot(ci[u] - ci[v], cj[u] - cj[v]), (u, v)), shape=(N, N)).tocsr()
    D = shortest_path(G, directed=False)
    direct = np.hypot(ci[:, None] - ci[None, :], cj[:, None] - cj[None, :])
    t = (s_override + 2) / (s_override - 2)
    off = ~np.eye(N, dtype=bool)
    assert (D[off] <= t * direct[off] * (1 + 1e-12)).all()


def test_l2_costs_rounded_up(orc):
    # every cost is ceil(2^K x distance) computed in doubles: not below the
    # exact distance by more than a rounding of the square root, and less
    # than one unit above it (50-digit decimal arithmetic as the judge)
    from decimal import Decimal, getcontext

    getcontext().prec = 50
    A, B = pdsynth.mixture_pd(300, 180), pdsynth.mixture_pd(280, 181)
    r = orc.run(A, B, eps=0.1, flags=orc.ORC_L2 | orc.ORC_NO_FLOW)
    net = orc.csr(A, B, eps=0.1, l2=True)
    K = r.K
    assert 0 <= K <= 30
    N = r.cells["i"].shape[0]
    ci, cj = r.cells["i"], r.cells["j"]
    rp, col, cost = net["row_ptr"], net["col"], net["cost"]
    tail = np.repeat(np.arange(N + 2), np.diff(rp))
    scale = Decimal(2) ** K
    lo, hi = Decimal(1) - Decimal(2) ** -50, Decimal(1) + Decimal(2) ** -50
    for t, h, c in zip(tail.tolist(), col.tolist(), cost.tolist()):
        if t < N and h < N:
            x = Decimal(int(ci[t] - ci[h]) ** 2 + int(cj[t] - cj[h]) ** 2).sqrt() * scale
        elif t < N:
            x = Decimal(int(cj[t] - ci[t])) / Decimal(2).sqrt() * scale
        elif h < N:
            x = Decimal(int(cj[h] - ci[h])) / Decimal(2).sqrt() * scale
        else:
            x = Decimal(0)
        assert Decimal(c) >= x * lo and Decimal(c) - 1 < x * hi, (t, h, c, x)


def test_l2_invariances(orc):
    A, B = pdsynth.exp_pd(60, 190), pdsynth.exp_pd(55, 191)
    r = orc.run(A, B, eps=0.2, flags=orc.ORC_L2)
    rs = orc.run(B, A, eps=0.2, flags=orc.ORC_L2)
    assert rs.W1 == r.W1 and rs.flow == r.flow and rs.L == r.L
    r2 = orc.run(2 * A, 2 * B, eps=0.2, flags=orc.ORC_L2)
    assert r2.flow == r.flow and r2.K == r.K and r2.W1 == 2 * r.W1 and r2.L == 2 * r.L
    # pruning is defined for the L-infinity network only
    assert orc.run(A, B, eps=0.2, flags=orc.ORC_L2 | orc.ORC_PRUNE).status == -1


def test_l2_sparse_network_theorem(orc):
    # f* of the dense condensed network <= f* of the sparse one <= t f*(dense),
    # costs rounded up alike (units of g 2^-K, so the rounding adds under one
    # unit per arc: a relative 1e-6 allowance)
    for seed, s in ((0, 4), (1, 12)):
        A = pdsynth.exp_pd(60, 520 + seed, mean_pers=0.2)
        B = pdsynth.exp_pd(50, 620 + seed, mean_pers=0.2)
        r = orc.run(A, B, eps=0.2, s_override=s, flags=orc.ORC_L2)
        K = r.K
        ci, cj, ca, cb = r.cells["i"], r.cells["j"], r.cells["cA"], r.cells["cB"]
        ia, ib = np.nonzero(ca)[0], np.nonzero(cb)[0]
        na, nb = ia.shape[0], ib.shape[0]
        X, Y = np.meshgrid(np.arange(na), np.arange(nb), indexing="ij")
        d = np.sqrt(((ci[ia][X] - ci[ib][Y]) ** 2 + (cj[ia][X] - cj[ib][Y]) ** 2).astype(np.float64))
        cAB = np.ceil(np.ldexp(d, K)).astype(np.int64).ravel()
        dd = lambda k: np.ceil(np.ldexp((cj[k] - ci[k]).astype(np.float64) * R_SQRT1_2, K)).astype(np.int64)
        src = np.concatenate([X.ravel(), np.arange(na), np.full(nb, na + nb + 1), [na + nb + 1]])
        dst = np.concatenate([na + Y.ravel(), np.full(na, na + nb), na + np.arange(nb), [na + nb]])
        cost = np.concatenate([cAB, dd(ia), dd(ib), [0]])
        supply = np.concatenate([ca[ia], -cb[ib], [-ca.sum(), cb.sum()]])
        fd = orc.mcf(na + nb + 2, src, dst, cost, supply)
        t = (s + 2) / (s - 2)
        assert fd <= r.flow <= t * fd * (1 + 1e-6)


def test_l2_grid_exponent(orc):
    # g = 2^e with e = floor(log2(sqrt(2) eps_c L / n)) (the condensation moves
    # a point by at most half a cell diagonal, g / sqrt(2)), computed here in
    # 50-digit decimal arithmetic away from powers of two
    from decimal import Decimal, getcontext

    getcontext().prec = 50
    rng = np.random.default_rng(3)
    two = Decimal(2)
    seen_diff = 0
    for _ in range(200):
        eps_c = float(rng.choice([0.02, 0.01, 0.005, 0.001]))
        L = float(np.exp(rng.uniform(np.log(1e-3), np.log(1e4))))
        n = int(rng.integers(1, 10**6))
        x = two * Decimal(eps_c) * Decimal(L) / Decimal(n) / two.sqrt()
        e = int(np.floor(float(x.ln() / two.ln())))
        frac = x / two ** e
        if not (Decimal("1.000001") < frac < Decimal("1.999999")):
            continue
        assert orc.grid_exponent(eps_c, L, n, l2=True) == e
        seen_diff += orc.grid_exponent(eps_c, L, n) != e
    assert seen_diff > 20  # the sqrt(2) moves the exponent for a good share of the cases


def test_l2_condensation_corner(orc):
    # One point at the far corner of its cell (birth at the low edge, death
    # at the high edge): snapping it to the cell centre lowers its distance
    # to the diagonal by almost the full g / sqrt(2), so W1 >= exact needs
    # the whole n g / sqrt(2) added back after the flow.
    g = 2.0**-10
    tiny = g / 1024
    p = np.array([[7 * g + tiny, 148 * g - tiny]])
    r = orc.run(p, np.zeros((0, 2)), eps=0.1, flags=orc.ORC_L2)
    assert r.status == 0 and r.g == g and r.n_pairs == 0
    ex = orc.exact_w1(p, np.zeros((0, 2)), l2=True)
    # L is (d - b) R, R the double nearest 1/sqrt(2): equal to exact up to
    # the rounding of that product
    assert r.L <= ex * (1 + 2.0**-50) and ex <= r.W1 <= 1.1 * ex
    assert ex - r.W1_paper > 0.7 * g  # most of the half diagonal


# ------------------------------------------------------- record checksum --
def _mix(u, v, c):
    # the record hash as the library header defines it, in Python integers
    M = 2**64
    x = (((u + 1) * 0x9E3779B97F4A7C15 + (v + 1)) * 0xC2B2AE3D27D4EB4F + c) % M
    return (x * 0x165667B19E3779F9) % M


@pytest.mark.parametrize("l2", [False, True])
def test_pair_checksum_definition(orc, l2):
    # The count-only checksum equals the definition summed over the pair list
    # the oracle emits (whose coverage and separation other pins fix); a
    # Euclidean record carries no cost, so c = 0 there.
    A = pdsynth.exp_pd(70, 1201)
    B = pdsynth.exp_pd(60, 1202)
    fl = orc.ORC_L2 if l2 else 0
    full = orc.run(A, B, eps=0.2, flags=fl | orc.ORC_NO_FLOW)
    cnt = orc.run(A, B, eps=0.2, flags=fl | orc.ORC_COUNT_ONLY, fetch=False)
    assert cnt.n_pairs == full.n_pairs > 100
    h1 = h2 = 0
    for u, v, c in zip(full.pairs["u"].tolist(), full.pairs["v"].tolist(), full.pairs["c"].tolist()):
        h = _mix(u, v, 0 if l2 else c)
        h1 = (h1 + h) % 2**64
        h2 = (h2 + h * h) % 2**64
    assert cnt.checksum == full.checksum == (h1, h2)


# ------------------------------------------------- the paper's own grid --
def test_paper_grid_closed_forms(orc):
    # Alg. 2 / Alg. 3 take eps_c = 8/(s - 4) for s >= 12 and 1 below.  One
    # point (0.5, 2) against the empty diagram: L = 0.75 and n = 1, so the
    # grid side is the largest power of two not above 1.5 eps_c (L-infinity)
    # or 1.5 eps_c / sqrt(2) (Euclidean).  Values worked out by hand:
    # s = 12 -> eps_c 1 -> 1.5 -> g = 1;  s = 20 -> 0.5 -> 0.75 -> 1/2;
    # s = 53 -> 8/49 -> 0.2449 -> 1/8;  s = 5 and s = 1 -> 1 -> g = 1.
    # Euclidean: 1.06 -> 1, 0.53 -> 1/2, 0.173 -> 1/8, 1.06 -> 1.
    A, E = np.array([[0.5, 2.0]]), np.zeros((0, 2))
    for s, e_inf, e_l2, ec in ((12, 0, 0, 1.0), (20, -1, -1, 0.5), (53, -3, -3, 8 / 49), (5, 0, 0, 1.0),
                               (1, 0, 0, 1.0)):
        r = orc.run(A, E, eps=0.1, s_override=s, flags=orc.ORC_PAPER_GRID)
        assert r.status == 0 and r.L == 0.75 and r.s == s
        assert r.e == e_inf and r.eps_c == ec
        r2 = orc.run(A, E, eps=0.1, s_override=s, flags=orc.ORC_PAPER_GRID | orc.ORC_L2)
        assert r2.status == 0 and r2.e == e_l2
    # the flag needs a sparsity parameter
    assert orc.run(A, E, eps=0.1, flags=orc.ORC_PAPER_GRID).status != 0


@pytest.mark.parametrize("s", [12, 20, 5])
def test_paper_grid_bracket(orc, s):
    # exact W1 <= w1 <= (t + (t + 1) eps_c) exact W1 with t = (s + 2)/(s - 2),
    # the L-infinity stretch, and the paper's eps_c for this s
    ec = 8 / (s - 4) if s >= 12 else 1.0
    t = (s + 2) / (s - 2)
    for seed in range(8):
        A = pdsynth.exp_pd(60, 1300 + 2 * seed)
        B = pdsynth.exp_pd(55, 1301 + 2 * seed)
        r = orc.run(A, B, eps=0.1, s_override=s, flags=orc.ORC_PAPER_GRID)
        ex = orc.exact_w1(A, B)
        assert r.status == 0 and r.eps_c == ec
        assert ex * (1 - 1e-12) <= r.W1 <= (t + (t + 1) * ec) * ex * (1 + 1e-12)

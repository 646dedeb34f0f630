"""GPU parity: every stage of the HIP pipeline against the CPU oracle on the
same seeded inputs.  Integer and index outputs must match bit for bit; the
FP64 RWMD terms and L must match exactly too (same IEEE operations, exact
fixed-point sum), and W1 = (g/2)(F* + n) must be identical because F* is an
integer optimum on the identical network."""
import os
import sys

import numpy as np
import pytest

import cases
import pdsynth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2110_14734_amd as w1

    return w1.Context(0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_tree(r):
    N = r.cells["i"].shape[0]
    nodes = r.nodes[N:]
    key = np.lexsort((nodes[:, 1], nodes[:, 0]))
    nodes = nodes[key]
    return nodes[:, 0], nodes[:, 1], nodes[:, 4], nodes[:, 5:9]


def _gpu_tree(g):
    st = g.stages
    lo, hi, left = st["node_lo"].astype(np.int64), st["node_hi"].astype(np.int64), st["node_left"].astype(np.int64)
    split = np.where(left >= 0, hi[np.maximum(left, 0)], ~left)
    key = np.lexsort((hi, lo))
    return lo[key], hi[key], split[key], st["node_box"].astype(np.int64)[key]


def check_csr(net, o):
    """The library's network rows equal the oracle's sorted rows exactly."""
    assert np.array_equal(net["row_ptr"], o["row_ptr"])
    assert np.array_equal(net["col"].astype(np.int64), o["col"])
    assert np.array_equal(net["cost"].astype(np.int64), o["cost"])
    assert np.array_equal(net["supply"], o["supply"])


NET_KEYS = ("cell_i", "cell_j", "cell_ca", "cell_cb", "supply", "row_ptr", "col", "cost")


def same_network(a, b):
    return all(np.array_equal(a.network.get(f, np.zeros(0)), b.network.get(f, np.zeros(0))) for f in NET_KEYS)


def _stored_flows():
    import json

    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_flows.json")) as f:
        return json.load(f)


STORED = _stored_flows()


def compare(orc, ctx, A, B, eps=0.1, s_override=0, flow=True, tree=True, prune=False, stored=None, l2=False,
            paper_grid=False):
    """Stage-by-stage parity with the oracle.  `stored` names the oracle's
    optimal flow written by tests/golden/make_oracle_flows.py; the oracle
    then runs without its (slow) flow solve.  Pruning leaves F* unchanged,
    so a pruned case compares with the unpruned stored optimum."""
    import paper_2110_14734_amd as w1

    flags = w1.KEEP_NETWORK | w1.KEEP_STAGES | (0 if flow else w1.NO_FLOW) | (w1.PRUNE if prune else 0)
    flags |= (w1.METRIC_L2 if l2 else 0) | (w1.PAPER_GRID if paper_grid else 0)
    g = ctx.approx(A, B, eps=eps, s_override=s_override, flags=flags)
    oflow = flow and stored is None
    oflags = (0 if oflow else orc.ORC_NO_FLOW) | (orc.ORC_PRUNE if prune else 0) | (orc.ORC_L2 if l2 else 0)
    oflags |= orc.ORC_PAPER_GRID if paper_grid else 0
    r = orc.run(A, B, eps=eps, s_override=s_override, flags=oflags)
    assert r.status == 0 and g.status == 0
    # a0: net 0-condensation
    assert (g.n_a, g.n_b, g.n_points) == (r.nA, r.nB, r.n)
    assert g.n_locations == r.locs["b"].shape[0]
    if r.n == 0:
        assert g.w1 == 0.0 and g.n_cells == 0 and g.n_pairs == 0
        return g, r
    st = g.stages
    assert np.array_equal(st["loc_b"], r.locs["b"]) and np.array_equal(st["loc_d"], r.locs["d"])
    assert np.array_equal(st["loc_w"], r.locs["w"])
    # a1: RWMD per location and the exact fixed-point sums
    assert np.array_equal(st["loc_t"], r.locs["t"])
    assert (st["rwmd_sum_a"], st["rwmd_sum_b"]) == (r.SA, r.SB)
    assert (st["rwmd_shift_a"], st["rwmd_shift_b"]) == (r.FA, r.FB)
    assert g.lower_bound == r.L
    # a2: grid and cells
    assert (g.grid_exp, g.s) == (r.e, r.s)
    net = g.network
    assert g.n_cells == r.cells["i"].shape[0]
    assert np.array_equal(net["cell_i"], r.cells["i"]) and np.array_equal(net["cell_j"], r.cells["j"])
    assert np.array_equal(net["cell_ca"], r.cells["cA"]) and np.array_equal(net["cell_cb"], r.cells["cB"])
    # a3: tree (as a set of nodes: range, split, box)
    if tree and g.n_cells >= 2:
        for x, y in zip(_gpu_tree(g), _oracle_tree(r)):
            assert np.array_equal(x, y)
    # a4 + a5: the WSPD pairs and the network, compared as the sorted rows
    # element by element (no host-side sorting of the library's output)
    assert g.n_pairs == r.n_pairs
    if l2:
        assert g.metric_l2 and g.cost_shift == r.K
    check_csr(net, orc.csr(A, B, eps=eps, s_override=s_override, prune=prune, l2=l2, paper_grid=paper_grid))
    # flow and W1
    if flow and stored is None:
        assert g.flow_cost == r.flow
        assert g.w1 == r.W1 and g.w1_paper == r.W1_paper
    elif flow:
        ref = STORED[stored]
        assert g.flow_cost == ref["flow"]
        assert g.w1 == float.fromhex(ref["W1"]) and g.w1_paper == float.fromhex(ref["W1_paper"])
    return g, r


CASES = cases.STAGE_CASES


@pytest.mark.parametrize("name,make,eps", CASES, ids=[c[0] for c in CASES])
def test_stage_parity(orc, ctx, name, make, eps):
    _say(f"[gpu] stage parity {name}")
    A, B = make()
    compare(orc, ctx, A, B, eps=eps, stored=name)


@pytest.mark.parametrize("name,make,eps", CASES, ids=[c[0] for c in CASES])
def test_prune_parity(orc, ctx, name, make, eps):
    """Diagonal-dominance pruning: the kept pairs and the network equal the
    oracle's pruned network row for row, and F* (hence W1) equals the
    unpruned optimum."""
    _say(f"[gpu] prune parity {name}")
    A, B = make()
    g, r = compare(orc, ctx, A, B, eps=eps, prune=True, stored=name)
    full = ctx.approx(A, B, eps=eps)
    assert g.flow_cost == full.flow_cost and g.w1 == full.w1 and g.n_pairs <= full.n_pairs


@pytest.mark.parametrize("name,make,eps", CASES, ids=[c[0] for c in CASES])
def test_l2_parity(orc, ctx, name, make, eps):
    """Euclidean ground metric: every stage bit for bit with the oracle --
    RWMD costs and L, grid, cells, tree, the sorted network with its 64-bit
    costs -- and F* and W1 equal to the oracle's stored optimum."""
    _say(f"[gpu] Euclidean parity {name}")
    A, B = make()
    compare(orc, ctx, A, B, eps=eps, stored=name + "_l2", l2=True)


def test_l2_batch_small_s_and_errors(orc, ctx):
    """Euclidean metric in the batched form and at small s: per-pair counts,
    networks and W1 equal the single calls and the oracle; pruning is
    rejected."""
    import paper_2110_14734_amd as w1

    _say("[gpu] Euclidean batch")
    As, Bs = cases.batch_pairs()
    batch = ctx.approx_batch(As, Bs, eps=0.2, flags=w1.KEEP_NETWORK | w1.METRIC_L2)
    for i in range(len(As)):
        single = ctx.approx(As[i], Bs[i], eps=0.2, flags=w1.KEEP_NETWORK | w1.METRIC_L2)
        assert same_network(batch[i], single) and batch[i].w1 == single.w1
        r = orc.run(As[i], Bs[i], eps=0.2, flags=orc.ORC_L2 | orc.ORC_NO_FLOW)
        assert batch[i].n_pairs == r.n_pairs and batch[i].lower_bound == r.L
        if r.n:
            check_csr(batch[i].network, orc.csr(As[i], Bs[i], eps=0.2, l2=True))
    A, B = cases.small_s_pair()
    for s in (1, 3):
        compare(orc, ctx, A, B, eps=0.1, s_override=s, flow=False, l2=True)
    with pytest.raises(w1.W1Error) as e:
        ctx.approx(A, B, eps=0.1, flags=w1.METRIC_L2 | w1.PRUNE)
    assert e.value.code == w1.W1_EINVAL
    # the RWMD bound alone in the Euclidean metric
    L = ctx.rwmd(As[:4], Bs[:4], flags=w1.METRIC_L2)
    for i in range(4):
        assert L[i] == orc.run(As[i], Bs[i], eps=0.2, flags=orc.ORC_L2 | orc.ORC_NO_FLOW).L


def test_l2_bracket_against_exact(orc, ctx):
    """Euclidean (1 + eps) bracket against Hungarian matching with Euclidean
    costs, end to end, on 20 pairs of 120 + 110 points (exact W1 computed
    here: 230 x 230 assignments)."""
    _say("[gpu] Euclidean bracket")
    As = [pdsynth.exp_pd(120, 7000 + 2 * k) for k in range(20)]
    Bs = [pdsynth.exp_pd(110, 7001 + 2 * k) for k in range(20)]
    import paper_2110_14734_amd as w1

    res = ctx.approx_batch(As, Bs, eps=0.1, flags=w1.METRIC_L2)
    for A, B, g in zip(As, Bs, res):
        ex = orc.exact_w1(A, B, l2=True)
        assert g.lower_bound <= ex * (1 + 2.0**-50) and ex <= g.w1 <= 1.1 * ex


def test_prune_batch_and_count_only(orc, ctx):
    """Pruning in the batched form: every pair's network equals the oracle's
    pruned rows, the count-only pass counts the same kept pairs, and the
    optimum equals the unpruned batch's."""
    _say("[gpu] prune batch")
    import paper_2110_14734_amd as w1

    sizes = pdsynth.batch_sizes(16, 31, lo=20, hi=2500)
    As = [pdsynth.mixture_pd(int(sizes[i]), 5000 + 2 * i) for i in range(8)]
    Bs = [pdsynth.mixture_pd(int(sizes[8 + i]), 5001 + 2 * i) for i in range(8)]
    As[2] = np.zeros((0, 2), np.float32)
    pr = ctx.approx_batch(As, Bs, eps=0.1, flags=w1.KEEP_NETWORK | w1.PRUNE)
    full = ctx.approx_batch(As, Bs, eps=0.1)
    cnt = ctx.approx_batch(As, Bs, eps=0.1, flags=w1.COUNT_ONLY | w1.PRUNE)
    for i in range(8):
        r = orc.run(As[i], Bs[i], eps=0.1, flags=orc.ORC_PRUNE | orc.ORC_NO_FLOW)
        assert pr[i].n_pairs == r.n_pairs == cnt[i].n_pairs
        assert pr[i].flow_cost == full[i].flow_cost and pr[i].w1 == full[i].w1
        if r.n:
            check_csr(pr[i].network, orc.csr(As[i], Bs[i], eps=0.1, prune=True))


@pytest.mark.parametrize("s_override", [1, 2, 3, 6, 12])
def test_paper_mode_small_s(orc, ctx, s_override):
    _say(f"[gpu] s_override {s_override}")
    A, B = cases.small_s_pair()
    compare(orc, ctx, A, B, eps=0.1, s_override=s_override, stored=f"small_s{s_override}")


@pytest.mark.parametrize("s_override,l2", [(12, False), (20, False), (3, False), (20, True)])
def test_paper_grid(orc, ctx, s_override, l2):
    """The paper's own grid for a given s (eps_c = 8/(s - 4), or 1 below
    s = 12): every stage, the network and W1 equal the oracle's; the flag
    without s_override is rejected."""
    import paper_2110_14734_amd as w1

    _say(f"[gpu] paper grid s={s_override} l2={l2}")
    A, B = pdsynth.exp_pd(300, 40), pdsynth.exp_pd(280, 41)
    g, r = compare(orc, ctx, A, B, eps=0.1, s_override=s_override, l2=l2, paper_grid=True)
    assert r.eps_c == (8 / (s_override - 4) if s_override >= 12 else 1.0)
    with pytest.raises(w1.W1Error) as e:
        ctx.approx(A, B, eps=0.1, flags=w1.PAPER_GRID)
    assert e.value.code == w1.W1_EINVAL


def test_fused_expansion(orc, ctx):
    """The work list expanded in one workgroup, round by round, and in one
    workgroup that runs out of room (then round by round from the roots)
    gives the same WSPD pairs, network and W1, for single pairs (also at
    s = 1 and 3, Euclidean, pruned, on the paper's grid) and for a batch
    expanded in one workgroup; one fused case against the oracle too."""
    import paper_2110_14734_amd as w1

    _say("[gpu] fused work-list expansion")
    t0 = ctx.tuning
    configs = ((dict(fused_expand_cells=0), 0), (dict(fused_expand_cells=65536), 1),
               (dict(fused_expand_cells=65536, fused_expand_items=64), -1))
    A, B = pdsynth.exp_pd(300, 40), pdsynth.exp_pd(280, 41)
    single = [(A, B, dict(eps=0.1)), (A, B, dict(eps=0.1, s_override=1)), (A, B, dict(eps=0.1, s_override=3)),
              (A, B, dict(eps=0.1, flags=w1.METRIC_L2)), (A, B, dict(eps=0.1, flags=w1.PRUNE)),
              (A, B, dict(eps=0.1, s_override=20, flags=w1.PAPER_GRID))]
    for name, make, eps in cases.STAGE_CASES:
        X, Y = make()
        single.append((X, Y, dict(eps=eps)))
    try:
        for case, (X, Y, kw) in enumerate(single):
            kw = dict(kw)
            fl = kw.pop("flags", 0) | w1.KEEP_NETWORK | w1.NO_FLOW
            out = []
            for cfg, want in configs:
                ctx.tuning = dict(t0, **cfg)
                g = ctx.approx(X, Y, flags=fl, **kw)
                if g.n_cells >= 2:
                    got = ctx.kernel_times()["fused_expand"]
                    # the default room may run out on the larger stage cases
                    assert got == want or (want == 1 and case >= 6 and got == -1)
                out.append(g)
            for g in out[1:]:
                assert (g.n_pairs, g.lower_bound, g.n_arcs) == (out[0].n_pairs, out[0].lower_bound, out[0].n_arcs)
                assert same_network(g, out[0])
        As, Bs = cases.batch_pairs()
        res = []
        for cfg, want in ((dict(fused_expand_cells=0), 0),
                          (dict(fused_expand_cells=65536, fused_expand_items=1 << 23), 1)):
            ctx.tuning = dict(t0, **cfg)
            res.append(ctx.approx_batch(As, Bs, eps=0.2, flags=w1.KEEP_NETWORK | w1.NO_FLOW))
            assert ctx.kernel_times()["fused_expand"] == want
        for a, b in zip(*res):
            assert a.n_pairs == b.n_pairs and same_network(a, b)
        ctx.tuning = dict(t0, fused_expand_cells=65536)
        compare(orc, ctx, *cases.STAGE_CASES[2][1](), eps=cases.STAGE_CASES[2][2], flow=False)
        assert ctx.kernel_times()["fused_expand"] == 1
        for bad in (dict(fused_expand_cells=-1), dict(fused_expand_cells=65537), dict(fused_expand_items=-1)):
            with pytest.raises(w1.W1Error):
                ctx.tuning = dict(t0, **bad)
    finally:
        ctx.tuning = t0


def test_edge_cases(orc, ctx):
    _say("[gpu] edge cases")
    import paper_2110_14734_amd as w1

    E = np.zeros((0, 2))
    A = pdsynth.exp_pd(50, 14)
    # empty / empty, identical, one-sided, single point, diagonal points
    for X, Y in ((E, E), (A, A.copy()), (A, E), (E, A), (A[:1], E), (A[:1], A[1:2])):
        compare(orc, ctx, X, Y, eps=0.1)
    diag = np.array([[0.3, 0.3], [0.5, 0.5]])
    g1 = ctx.approx(np.concatenate([A, diag]), A[:20], eps=0.1)
    g2 = ctx.approx(A, A[:20], eps=0.1)
    assert g1.w1 == g2.w1
    # co-located A/B points cancel
    C = A[:7]
    g3 = ctx.approx(np.concatenate([A, C]), np.concatenate([C, A[:20]]), eps=0.1)
    assert g3.w1 == g2.w1 and g3.n_points == g2.n_points
    # invalid points: error for that pair only
    bad = np.array([[1.0, 0.5]])
    with pytest.raises(w1.W1Error) as e:
        ctx.approx(bad, A)
    assert e.value.code == w1.W1_EINVAL
    res = ctx.approx_batch([bad, A], [A, A[:10]], eps=0.1, check=False)
    assert res[0].status == w1.W1_EINVAL and res[1].status == 0
    assert res[1].w1 == ctx.approx(A, A[:10], eps=0.1).w1
    nan = np.array([[np.nan, 1.0]])
    assert ctx.approx_batch([nan], [A], check=False)[0].status == w1.W1_EINVAL


def _exact_gold():
    import json

    with open(os.path.join(os.path.dirname(__file__), "golden", "exact_w1.json")) as f:
        return json.load(f)


def test_bracket_against_exact(ctx):
    """RWMD <= exact W1 <= w1 <= (1 + eps) exact W1 on 100 pairs of 400 + 400
    points at eps 0.1, end to end (host flow included); exact W1 by Hungarian
    matching, stored by tests/golden/make_exact_brackets.py (oracle only)."""
    _say("[gpu] bracket vs Hungarian, 100 pairs of 400+400 points")
    ex = [float.fromhex(x) for x in _exact_gold()["c1"]["w1"]]
    As = [pdsynth.exp_pd(400, 2 * k) for k in range(len(ex))]
    Bs = [pdsynth.exp_pd(400, 2 * k + 1) for k in range(len(ex))]
    res = ctx.approx_batch(As, Bs, eps=0.1)
    for k, (g, e) in enumerate(zip(res, ex)):
        assert g.status == 0 and g.flow_solved == 1, k
        assert g.lower_bound <= e <= g.w1 <= 1.1 * e, (k, g.lower_bound, e, g.w1)
        assert (1 - 0.01) * e <= g.w1_paper <= 1.1 * e, k


def test_bracket_batched_small_pairs(ctx):
    """The same bracket on every pair of the batched workload (4096 pairs,
    100 to 50k points per diagram, FP32) with n_A + n_B <= 3000: 1081 pairs,
    solved end to end in one batch call at eps 0.1."""
    _say("[gpu] bracket vs Hungarian, batched workload pairs with n_A + n_B <= 3000")
    gold = _exact_gold()["c3_small"]
    idx, ex = gold["index"], [float.fromhex(x) for x in gold["w1"]]
    sizes = pdsynth.batch_sizes(2 * 4096, 3)
    na, nb = sizes[0::2], sizes[1::2]
    As = [pdsynth.exp_pd(int(na[i]), 10 + 2 * i, dtype=np.float32) for i in idx]
    Bs = [pdsynth.exp_pd(int(nb[i]), 11 + 2 * i, dtype=np.float32) for i in idx]
    res = ctx.approx_batch(As, Bs, eps=0.1)
    for i, g, e in zip(idx, res, ex):
        assert g.status == 0 and g.flow_solved == 1, i
        assert g.lower_bound <= e <= g.w1 <= 1.1 * e, (i, g.lower_bound, e, g.w1)


def test_batch_equals_single_and_oracle(orc, ctx):
    _say("[gpu] batch vs single")
    import paper_2110_14734_amd as w1

    As, Bs = cases.batch_pairs()
    flags = w1.KEEP_NETWORK
    batch = ctx.approx_batch(As, Bs, eps=0.2, flags=flags)
    for i in range(12):
        single = ctx.approx(As[i], Bs[i], eps=0.2, flags=flags)
        r = orc.run(As[i], Bs[i], eps=0.2, flags=orc.ORC_NO_FLOW)
        ref = STORED[f"batch{i}"]
        for x in (batch[i], single):
            assert x.w1 == float.fromhex(ref["W1"]) and x.flow_cost == ref["flow"] and x.n_pairs == r.n_pairs
            assert x.lower_bound == r.L
        assert same_network(batch[i], single)
        if r.n:
            check_csr(batch[i].network, orc.csr(As[i], Bs[i], eps=0.2))


def test_determinism_and_count_only(ctx):
    _say("[gpu] determinism")
    import paper_2110_14734_amd as w1

    A, B = pdsynth.mixture_pd(20000, 20), pdsynth.mixture_pd(19000, 21)
    g1 = ctx.approx(A, B, eps=0.2, flags=w1.KEEP_NETWORK | w1.NO_FLOW)
    g2 = ctx.approx(A, B, eps=0.2, flags=w1.KEEP_NETWORK | w1.NO_FLOW)
    assert same_network(g1, g2)
    g3 = ctx.approx(A, B, eps=0.2, flags=w1.COUNT_ONLY)
    assert g3.n_pairs == g1.n_pairs and g3.lower_bound == g1.lower_bound


def test_device_inputs_and_stream(orc, ctx):
    """torch device tensors on a side stream give the same result as host
    arrays (oracle compared without its flow: its successive-shortest-path
    solve is far too slow for the 1e7 arcs of this pair)."""
    _say("[gpu] torch device inputs")
    import torch

    import paper_2110_14734_amd as w1

    A, B = pdsynth.mixture_pd(5000, 22), pdsynth.mixture_pd(4800, 23)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    g_host = ctx.approx(A, B, eps=0.2)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g_dev = ctx.approx(tA, tB, eps=0.2, flags=w1.KEEP_NETWORK)
    assert g_dev.w1 == g_host.w1 and g_dev.flow_cost == g_host.flow_cost
    r = orc.run(A, B, eps=0.2, flags=orc.ORC_NO_FLOW)
    assert g_dev.lower_bound == r.L and g_dev.n_pairs == r.n_pairs
    check_csr(g_dev.network, orc.csr(A, B, eps=0.2))
    assert g_host.lower_bound <= g_host.w1


GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _digest(a, dtype):
    import hashlib

    dt = np.dtype(dtype)
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dt).astype(dt.newbyteorder("<")).tobytes()).hexdigest()


def _hip_runtime():
    """The HIP runtime already mapped into this process (the one the library
    and torch share), for plain device-to-host copies."""
    import ctypes

    paths = sorted({ln.split()[-1] for ln in open("/proc/self/maps") if "libamdhip64" in ln})
    assert len(paths) == 1, paths
    h = ctypes.CDLL(paths[0])
    h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return h


def _d2h(hip, ptr, n, dtype, out=None):
    out = np.empty(n, dtype) if out is None else out[:n]
    if n:
        assert hip.hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2) == 0  # hipMemcpyDeviceToHost
    return out


def check_device_network(ctx, k, chk, n_pairs, checker, chunk_arcs=1 << 28):
    """Checks pair k's device-resident network row block by row block: heads
    strictly increasing, costs recomputed from the cells, diagonal rows by
    membership, and both orientations of the cell arcs against the oracle's
    pair count and pair checksum."""
    import ctypes

    d = ctx.device_network(k)
    n, m = d["n_cells"], d["n_arcs"]
    hip, L = _hip_runtime(), checker
    rp = _d2h(hip, d["row_ptr"], n + 3, np.int64)
    ij = _d2h(hip, d["cell_ij"], 2 * n, np.int32).reshape(-1, 2)
    ci, cj = np.ascontiguousarray(ij[:, 0]), np.ascontiguousarray(ij[:, 1])
    ca, cb = _d2h(hip, d["cell_ca"], n, np.int32), _d2h(hip, d["cell_cb"], n, np.int32)
    assert rp[0] == 0 and rp[-1] == m and (np.diff(rp) >= 0).all()
    col_buf = np.empty(min(m, chunk_arcs + n + 2), np.uint32)
    cost_buf = np.empty_like(col_buf, dtype=np.int32)
    sums = np.zeros(4, np.uint64)
    counts = np.zeros(2, np.int64)
    first = ctypes.c_int64(-1)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    r0 = 0
    while r0 < n + 2:
        r1 = int(np.searchsorted(rp, rp[r0] + chunk_arcs, side="right")) - 1
        r1 = min(max(r1, r0 + 1), n + 2)
        a0, a1 = int(rp[r0]), int(rp[r1])
        assert a1 - a0 <= col_buf.shape[0]
        col = _d2h(hip, d["col"] + 4 * a0, a1 - a0, np.uint32, col_buf)
        cost = _d2h(hip, d["cost"] + 4 * a0, a1 - a0, np.int32, cost_buf)
        bad = L.csr_check_rows(n, r0, r1, p(rp), a0, a1 - a0, p(col), p(cost), p(ci), p(cj), p(ca), p(cb),
                               p(sums), p(counts), ctypes.byref(first))
        assert bad == 0, f"{bad} bad rows in [{r0}, {r1}), first {first.value}"
        r0 = r1
    assert counts[0] == n_pairs and counts[1] == n_pairs
    assert (int(sums[0]), int(sums[1])) == tuple(chk) and (int(sums[2]), int(sums[3])) == tuple(chk)
    return m


@pytest.mark.parametrize("eps,prune", [(0.1, False), (0.05, False), (0.1, True)])
def test_full_size_config2(ctx, csr_checker, eps, prune):
    """200k + 200k FP32 points (mixture) at the benchmark's eps 0.1 and at
    0.05, checked against the oracle's stored results (written by
    tests/golden/make_full_size.py, which calls only the oracle): every
    location and its RWMD cost, L and its fixed-point sums, every cell, the
    pair count, and the device-built network row by row -- sorted heads,
    costs from the cells, diagonal rows, and both orientations of the cell
    arcs against the oracle's pair checksum.  With pruning, the kept pairs
    against the oracle's pruned count and checksum."""
    import json

    import paper_2110_14734_amd as w1

    with open(os.path.join(GOLD, "c2_full.json")) as f:
        gold = json.load(f)["eps"][str(eps)]
    _say(f"[gpu] full-size mixture 200k+200k eps {eps} prune {prune}")
    A, B = pdsynth.mixture_pd(200_000, 0), pdsynth.mixture_pd(200_000, 1)
    g = ctx.approx(A, B, eps=eps, flags=w1.KEEP_STAGES | w1.NO_FLOW | (w1.PRUNE if prune else 0))
    pairs = gold["pruned"] if prune else gold
    assert (g.n_a, g.n_b, g.n_points, g.s, g.grid_exp) == (gold["nA"], gold["nB"], gold["n"], gold["s"], gold["e"])
    assert g.lower_bound == float.fromhex(gold["L"])
    st = g.stages
    assert (st["rwmd_sum_a"], st["rwmd_sum_b"], st["rwmd_shift_a"], st["rwmd_shift_b"]) == (
        gold["SA"], gold["SB"], gold["FA"], gold["FB"])
    h = gold["sha256"]
    assert g.n_locations == gold["n_locations"]
    for key, dt in (("loc_b", np.float64), ("loc_d", np.float64), ("loc_w", np.int64), ("loc_t", np.float64)):
        assert _digest(st[key], dt) == h[key], key
    assert g.n_cells == gold["n_cells"] and g.n_pairs == pairs["n_pairs"]
    d = ctx.device_network(0)
    hip = _hip_runtime()
    ij = _d2h(hip, d["cell_ij"], 2 * g.n_cells, np.int32).reshape(-1, 2)
    assert _digest(ij[:, 0], np.int64) == h["cell_i"] and _digest(ij[:, 1], np.int64) == h["cell_j"]
    assert _digest(_d2h(hip, d["cell_ca"], g.n_cells, np.int32), np.int64) == h["cell_ca"]
    assert _digest(_d2h(hip, d["cell_cb"], g.n_cells, np.int32), np.int64) == h["cell_cb"]
    _say(f"[gpu]   network: {g.n_arcs} arcs, checking rows")
    m = check_device_network(ctx, 0, pairs["checksum"], pairs["n_pairs"], csr_checker)
    assert m == g.n_arcs


@pytest.mark.parametrize("win", [64, 100])
def test_row_sort_windows(orc, ctx, win):
    """Rows sorted window by window (a bitmap window of 2048 or 3200 cells,
    far smaller than the pairs; a window of 100 words ends inside a group)
    give the oracle's network, row by row."""
    _say(f"[gpu] row sort in windows of {win} words")
    t0 = ctx.tuning
    try:
        ctx.tuning = dict(t0, sort_window_words=win)
        for name, make, eps in cases.STAGE_CASES[:4]:
            A, B = make()
            compare(orc, ctx, A, B, eps=eps, flow=False)
    finally:
        ctx.tuning = t0


def _net_digest(ctx, chunk=1 << 28):
    """Order-sensitive digest of pair 0's device network (heads, costs, row
    pointers), computed on the device."""
    import ctypes

    import torch

    d = ctx.device_network(0)
    hip = _hip_runtime()
    m = d["n_arcs"]
    buf = torch.empty(min(m, chunk), dtype=torch.int32, device="cuda")
    h = []
    for name in ("col", "cost"):
        acc = 0
        for a0 in range(0, m, chunk):
            n = min(chunk, m - a0)
            torch.cuda.synchronize()
            assert hip.hipMemcpy(ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(d[name] + 4 * a0), 4 * n, 3) == 0
            x = buf[:n].to(torch.int64) + 1
            w = torch.arange(a0, a0 + n, device="cuda", dtype=torch.int64) % 1000003 + 1
            acc = (acc + int((x * w).sum().item())) % (1 << 61)
        h.append(acc)
    rp = _d2h(hip, d["row_ptr"], d["n_cells"] + 3, np.int64)
    return tuple(h) + (int(rp.sum()), int(rp[-1]))


@pytest.mark.skip(reason="blocked emission is off by default and not yet validated on the GPU: its first runs "
                         "faulted (a block pointer lost between chunks, then a missing barrier before the bucket "
                         "scatter's counters), both fixed from reading the code but not run again")
def test_blocked_emission(ctx):
    """A single large pair's network is the same whether its pair records go
    into blocks sized by a count over every 16th chunk (the default), into
    the counted layout (blocked_emit 0), or into too few blocks, so that the
    pass is redone counted (emit_block_limit)."""
    import torch

    import paper_2110_14734_amd as w1

    _say("[gpu] blocked emission: default, off, forced fallback")
    A, B = pdsynth.mixture_pd(200_000, 0), pdsynth.mixture_pd(200_000, 1)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    t0 = ctx.tuning
    out = []
    try:
        for cfg, blocked in ((dict(blocked_emit=1), True), (dict(blocked_emit=0), False),
                             (dict(blocked_emit=1, emit_block_limit=64), False)):
            ctx.tuning = dict(t0, **cfg)
            g = ctx.approx(tA, tB, eps=0.1, flags=w1.NO_FLOW)
            kt = ctx.kernel_times()
            assert (kt["emit_blocks"] > 0) == blocked, cfg
            assert kt["pairs"] == g.n_pairs
            out.append((g.n_pairs, g.n_arcs, _net_digest(ctx)))
        with pytest.raises(w1.W1Error):
            ctx.tuning = dict(t0, blocked_emit=2)
    finally:
        ctx.tuning = t0
    assert out[0] == out[1] == out[2]
    assert out[0][0] == 1_823_249_560


def test_tuning_and_launch_groups(orc, ctx):
    """Other tunings and launch groups of a few points give the same pair
    sets, counts and W1; invalid tunings are rejected."""
    import paper_2110_14734_amd as w1

    _say("[gpu] tuning and launch groups")
    sizes = pdsynth.batch_sizes(12, 5, lo=50, hi=1500)
    As = [pdsynth.exp_pd(int(sizes[i]), 3000 + 2 * i, dtype=np.float32) for i in range(6)]
    Bs = [pdsynth.exp_pd(int(sizes[6 + i]), 3001 + 2 * i, dtype=np.float32) for i in range(6)]
    ref = ctx.approx_batch(As, Bs, eps=0.2, flags=w1.KEEP_NETWORK)
    t0 = ctx.tuning
    try:
        ctx.tuning = dict(stack_depth=12, work_cap=64, chunk_items=16, blocks_per_cu=2,
                          max_points_per_launch=2000)
        got = ctx.approx_batch(As, Bs, eps=0.2, flags=w1.KEEP_NETWORK)
        for a, b in zip(ref, got):
            assert (a.w1, a.n_pairs, a.n_cells, a.flow_cost) == (b.w1, b.n_pairs, b.n_cells, b.flow_cost)
            assert same_network(a, b)
        # the large-item setting used for counting at large separations
        ctx.tuning = dict(stack_depth=32, work_cap=65536, chunk_items=64, blocks_per_cu=2,
                          max_points_per_launch=1 << 22)
        big = ctx.approx_batch(As, Bs, eps=0.2, flags=w1.COUNT_ONLY)
        assert [x.n_pairs for x in big] == [x.n_pairs for x in ref]
        C, D = pdsynth.pareto_pd(20000, 8), pdsynth.pareto_pd(20000, 9)
        r0 = orc.run(C, D, eps=0.05, flags=orc.ORC_COUNT_ONLY)
        g0 = ctx.approx(C, D, eps=0.05, flags=w1.COUNT_ONLY)
        assert (g0.n_pairs, g0.n_cells, g0.n_points) == (r0.n_pairs, len(r0.cells["i"]), r0.n)
        for bad in (dict(stack_depth=4), dict(stack_depth=40), dict(blocks_per_cu=0), dict(work_cap=0),
                    dict(max_points_per_launch=0), dict(compact_records=2), dict(compact_records=-1)):
            with pytest.raises(w1.W1Error):
                ctx.tuning = dict(t0, **bad)
    finally:
        ctx.tuning = t0
    assert ctx.tuning == t0


def test_compact_records_and_wide_extent(orc, ctx):
    """The packed split records (28-bit child boxes) and the full child
    records give the same network; a pair whose grid extent exceeds 2^28
    cells, where the packed records cannot be used, still matches the oracle
    stage by stage."""
    import paper_2110_14734_amd as w1

    _say("[gpu] compact and full traversal records")
    sizes = pdsynth.batch_sizes(8, 7, lo=100, hi=3000)
    As = [pdsynth.mixture_pd(int(sizes[i]), 4000 + 2 * i) for i in range(4)]
    Bs = [pdsynth.mixture_pd(int(sizes[4 + i]), 4001 + 2 * i) for i in range(4)]
    t0 = ctx.tuning
    assert t0["compact_records"] == 1
    try:
        ref = ctx.approx_batch(As, Bs, eps=0.1, flags=w1.KEEP_NETWORK)
        ctx.tuning = dict(t0, compact_records=0)
        full = ctx.approx_batch(As, Bs, eps=0.1, flags=w1.KEEP_NETWORK)
        for a, b in zip(ref, full):
            assert (a.w1, a.n_pairs, a.flow_cost) == (b.w1, b.n_pairs, b.flow_cost)
            assert same_network(a, b)
    finally:
        ctx.tuning = t0
    # a cluster near the origin and two points near 19000: the grid is
    # 2^-15, so cell coordinates reach about 6.2e8 > 2^28
    rng = np.random.default_rng(5)
    b0 = rng.uniform(0.0, 1.0, 40)
    A = np.concatenate([np.stack([b0, b0 + rng.uniform(0.5, 1.0, 40)], 1), [[19000.0, 19001.0], [19003.0, 19005.0]]])
    B = A.copy()
    B[:, 1] += rng.uniform(0.0, 0.01, len(B))
    g = ctx.approx(A, B, eps=0.1)
    extent = (B[:, 1].max() - A[:, 0].min()) / g.grid
    assert 2.0**28 < extent < 2.0**30, (g.grid_exp, extent)
    compare(orc, ctx, A, B, eps=0.1)


def test_rwmd_dense_cluster(orc, ctx):
    """A cluster far denser than the RWMD bucket grid assumes: the 3x3 block
    of buckets around it holds thousands of candidates, more than the LDS
    stage takes, so its queries run the full ring search; every stage still
    matches the oracle."""
    _say("[gpu] RWMD dense cluster")
    rng = np.random.default_rng(21)

    def cluster(n, seed_shift):
        b = 0.5 + 0.005 * rng.random(n)
        d = 0.6 + 0.005 * rng.random(n)
        out = np.array([[0.0, 1.0], [0.9, 1.0], [0.1 + 0.01 * seed_shift, 0.7]])
        return np.concatenate([np.stack([b, d], 1), out])

    A, B = cluster(3000, 0), cluster(3000, 1)
    g, _ = compare(orc, ctx, A, B, eps=0.2, flow=False)
    assert g.n_locations > 6000


def _stream_gold():
    import json

    with open(os.path.join(os.path.dirname(__file__), "golden", "stream_checksums.json")) as f:
        return json.load(f)


def test_slotted_and_counted_layouts(orc, ctx):
    """Short work lists are emitted into per-chunk slots without a count
    pass (long ones are counted first: the full-size tests).  A 400 +
    400-point pair takes the slotted layout (no count-pass time), and its
    sorted rows and F* equal the oracle's, with and without pruning."""
    _say("[gpu] slotted emission")
    A, B = pdsynth.exp_pd(400, 0), pdsynth.exp_pd(400, 1)
    import paper_2110_14734_amd as w1

    for prune in (False, True):
        g = ctx.approx(A, B, eps=0.1, flags=w1.KEEP_NETWORK | (w1.PRUNE if prune else 0))
        # no count pass: the two events around where it would run are a few
        # microseconds apart (a count pass over this work list takes ~0.2 ms)
        assert ctx.kernel_times()["count_ms"] < 0.05
        net = orc.csr(A, B, eps=0.1, prune=prune)
        assert np.array_equal(g.network["row_ptr"], net["row_ptr"])
        assert np.array_equal(g.network["col"].astype(np.int64), net["col"])
        assert np.array_equal(g.network["cost"].astype(np.int64), net["cost"])
        assert g.flow_cost == orc.run(A, B, eps=0.1, flags=orc.ORC_PRUNE if prune else 0, fetch=False).flow


def test_stream_emission_small(orc, ctx):
    """Streamed emission through a small arena (many runs of chunks, each
    overwriting the last): every pair's records are written once, the
    streamed count equals the oracle's pair count and the record checksum
    equals the oracle's; a cap on the runs writes a prefix; an arena smaller
    than one chunk is an error."""
    import paper_2110_14734_amd as w1

    _say("[gpu] streamed emission, small arena")
    t0 = ctx.tuning
    try:
        for name, make, eps in cases.STAGE_CASES:
            A, B = make()
            r = orc.run(A, B, eps=eps, flags=orc.ORC_COUNT_ONLY, fetch=False)
            ctx.tuning = dict(t0, stream_arena_pairs=max(20_000, r.n_pairs // 7))
            g = ctx.approx(A, B, eps=eps, flags=w1.COUNT_ONLY)
            assert g.n_pairs == r.n_pairs == g.n_pairs_streamed, name
            assert g.pair_checksum == tuple(r.checksum), name
            assert ctx.kernel_times()["stream_emit_ms"] > 0
        A, B = cases.STAGE_CASES[2][1]()
        n = orc.run(A, B, eps=0.2, flags=orc.ORC_COUNT_ONLY, fetch=False).n_pairs
        ctx.tuning = dict(t0, stream_arena_pairs=n // 5, stream_max_rounds=1)
        g = ctx.approx(A, B, eps=0.2, flags=w1.COUNT_ONLY)
        assert g.n_pairs == n and 0 < g.n_pairs_streamed <= n // 5
        ctx.tuning = dict(t0, stream_arena_pairs=1)
        with pytest.raises(w1.W1Error) as e:
            ctx.approx(A, B, eps=0.2, flags=w1.COUNT_ONLY)
        assert e.value.code == w1.W1_EOVERFLOW
    finally:
        ctx.tuning = t0


def test_stream_emission_l2(orc, ctx):
    """Streamed emission under the Euclidean metric: the streamed count and
    the record checksum (records carry no cost there) equal the oracle's."""
    import paper_2110_14734_amd as w1

    _say("[gpu] streamed emission, Euclidean")
    t0 = ctx.tuning
    try:
        for name, make, eps in cases.STAGE_CASES[:3]:
            A, B = make()
            r = orc.run(A, B, eps=eps, flags=orc.ORC_COUNT_ONLY | orc.ORC_L2, fetch=False)
            ctx.tuning = dict(t0, stream_arena_pairs=max(20_000, r.n_pairs // 5))
            g = ctx.approx(A, B, eps=eps, flags=w1.COUNT_ONLY | w1.METRIC_L2)
            assert g.n_pairs == r.n_pairs == g.n_pairs_streamed, name
            assert g.pair_checksum == tuple(r.checksum), name
    finally:
        ctx.tuning = t0


def test_stream_emission_batched_sample(ctx):
    """Every 16th pair of the 4096-pair batched workload (256 pairs, eps 0.1)
    streamed in one batch call: per-pair counts and record checksums equal
    the oracle's (stored by tests/golden/make_stream_checksums.py)."""
    import paper_2110_14734_amd as w1

    _say("[gpu] streamed emission, batched workload sample")
    gold = _stream_gold()["batch"]
    sizes = pdsynth.batch_sizes(2 * 4096, 3)
    idx = gold["index"]
    As = [pdsynth.exp_pd(int(sizes[2 * i]), 10 + 2 * i, dtype=np.float32) for i in idx]
    Bs = [pdsynth.exp_pd(int(sizes[2 * i + 1]), 11 + 2 * i, dtype=np.float32) for i in idx]
    t0 = ctx.tuning
    try:
        ctx.tuning = dict(t0, stream_arena_pairs=1 << 28)
        res = ctx.approx_batch(As, Bs, eps=0.1, flags=w1.COUNT_ONLY)
    finally:
        ctx.tuning = t0
    for i, g, ref in zip(idx, res, gold["pairs"]):
        assert g.n_pairs == ref["n_pairs"] == g.n_pairs_streamed, i
        assert list(g.pair_checksum) == ref["checksum"], i


def test_stream_emission_graph_replay(orc, ctx):
    """The arena fills of the streamed emission replayed from one captured
    HIP graph equal the fills launched one by one, and the oracle's stored
    checksums, for every pair: 64 pairs of the batched workload through an
    arena of 2^22 records (dozens of fills, so the graph is replayed that
    many times), twice, with other work of the library (a full W1 call and a
    synchronisation) between the two graph calls."""
    import paper_2110_14734_amd as w1

    _say("[gpu] streamed emission, graph replay")
    gold = _stream_gold()["batch"]
    sizes = pdsynth.batch_sizes(2 * 4096, 3)
    idx = gold["index"][:64]
    As = [pdsynth.exp_pd(int(sizes[2 * i]), 10 + 2 * i, dtype=np.float32) for i in idx]
    Bs = [pdsynth.exp_pd(int(sizes[2 * i + 1]), 11 + 2 * i, dtype=np.float32) for i in idx]
    C1a, C1b = pdsynth.exp_pd(400, 0), pdsynth.exp_pd(400, 1)
    t0 = ctx.tuning
    runs = {}
    try:
        for mode in ("eager", "graph1", "between", "graph2"):
            if mode == "between":
                g = ctx.approx(C1a, C1b, eps=0.1)
                assert g.flow_cost == orc.run(C1a, C1b, eps=0.1, fetch=False).flow
                continue
            ctx.tuning = dict(t0, stream_arena_pairs=1 << 22, stream_graph=0 if mode == "eager" else 1)
            res = ctx.approx_batch(As, Bs, eps=0.1, flags=w1.COUNT_ONLY)
            runs[mode] = [(g.n_pairs, g.n_pairs_streamed, tuple(g.pair_checksum)) for g in res]
            assert ctx.kernel_times()["stream_emit_ms"] > 0
    finally:
        ctx.tuning = t0
    assert sum(n for n, _, _ in runs["eager"]) > 40 * (1 << 22)  # dozens of arena fills
    for mode in ("graph1", "graph2"):
        assert runs[mode] == runs["eager"], mode
    for i, (n, ns, chk), ref in zip(idx, runs["eager"], gold["pairs"]):
        assert n == ns == ref["n_pairs"] and list(chk) == ref["checksum"], i


def test_stream_emission_stress_subsample(ctx):
    """A 200k + 200k subsample of the stress workload (Pareto persistence,
    30% exact duplicates) at eps 0.01 (s = 503) with the large-item tuning
    of the stress run: the pair count and the checksum of every record,
    streamed through a 2^30-record arena, equal the oracle's."""
    import paper_2110_14734_amd as w1

    _say("[gpu] streamed emission, stress subsample eps 0.01")
    ref = _stream_gold()["stress"]
    A, B = pdsynth.pareto_pd(200_000, 0), pdsynth.pareto_pd(200_000, 1)
    t0 = ctx.tuning
    try:
        ctx.tuning = dict(t0, stack_depth=32, work_cap=65536, chunk_items=64, blocks_per_cu=2,
                          stream_arena_pairs=1 << 30)
        g = ctx.approx(A, B, eps=0.01, flags=w1.COUNT_ONLY)
    finally:
        ctx.tuning = t0
    assert g.s == ref["s"] == 503
    assert g.n_pairs == ref["n_pairs"] == g.n_pairs_streamed
    assert list(g.pair_checksum) == ref["checksum"]

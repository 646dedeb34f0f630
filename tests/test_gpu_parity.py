"""GPU parity: every stage of the HIP pipeline against the CPU oracle on the
same seeded inputs.  Integer and index outputs must match bit for bit; the
FP64 RWMD terms and L must match exactly too (same IEEE operations, exact
fixed-point sum), and W1 = (g/2)(F* + n) must be identical because F* is an
integer optimum on the identical network."""
import os
import sys

import numpy as np
import pytest

import pdsynth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2110_14734_amd as w1

    return w1.Context(0)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sorted_pairs(u, v, c):
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    c = np.asarray(c, np.int64)
    o = np.lexsort((v, u))
    return u[o], v[o], c[o]


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


def compare(orc, ctx, A, B, eps=0.1, s_override=0, flow=True, tree=True):
    import paper_2110_14734_amd as w1

    flags = w1.KEEP_NETWORK | w1.KEEP_STAGES | (0 if flow else w1.NO_FLOW)
    g = ctx.approx(A, B, eps=eps, s_override=s_override, flags=flags)
    r = orc.run(A, B, eps=eps, s_override=s_override, flags=0 if flow else orc.ORC_NO_FLOW)
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
    # a4: WSPD pairs (u, v, cost) as a set
    assert g.n_pairs == r.n_pairs
    gu, gv, gc = _sorted_pairs(net["pair_u"], net["pair_v"], net["pair_cost"])
    ou, ov, oc = _sorted_pairs(r.pairs["u"], r.pairs["v"], r.pairs["c"])
    assert np.array_equal(gu, ou) and np.array_equal(gv, ov) and np.array_equal(gc, oc)
    # a5: diagonal arcs and supplies
    src, dst, cost, sup = orc.network(A, B, eps=eps, s_override=s_override)
    nd = src.shape[0] - 2 * r.n_pairs
    d_o = _sorted_pairs(src[2 * r.n_pairs:], dst[2 * r.n_pairs:], cost[2 * r.n_pairs:])
    d_g = _sorted_pairs(net["diag_src"], net["diag_dst"], net["diag_cost"])
    assert net["diag_src"].shape[0] == nd
    for x, y in zip(d_g, d_o):
        assert np.array_equal(x, y)
    assert np.array_equal(net["supply"], sup)
    # flow and W1
    if flow:
        assert g.flow_cost == r.flow
        assert g.w1 == r.W1 and g.w1_paper == r.W1_paper
    return g, r


CASES = [
    ("exp400_eps0.1", lambda: (pdsynth.exp_pd(400, 0), pdsynth.exp_pd(400, 1)), 0.1),
    ("exp250_eps0.2", lambda: (pdsynth.exp_pd(250, 2), pdsynth.exp_pd(233, 3)), 0.2),
    ("mix_f32_3000_eps0.2", lambda: (pdsynth.mixture_pd(3000, 4), pdsynth.mixture_pd(2777, 5)), 0.2),
    ("pareto_dup_2000_eps0.5", lambda: (pdsynth.pareto_pd(2000, 6), pdsynth.pareto_pd(1500, 7)), 0.5),
    ("int_overlap_eps0.3", lambda: (pdsynth.integer_pd(300, 8, hi=12), pdsynth.integer_pd(280, 9, hi=12)), 0.3),
    ("exp_f32_odd_eps0.05", lambda: (pdsynth.exp_pd(129, 10, dtype=np.float32), pdsynth.exp_pd(65, 11, dtype=np.float32)), 0.05),
]


@pytest.mark.parametrize("name,make,eps", CASES, ids=[c[0] for c in CASES])
def test_stage_parity(orc, ctx, name, make, eps):
    _say(f"[gpu] stage parity {name}")
    A, B = make()
    compare(orc, ctx, A, B, eps=eps)


@pytest.mark.parametrize("s_override", [1, 2, 3, 6, 12])
def test_paper_mode_small_s(orc, ctx, s_override):
    _say(f"[gpu] s_override {s_override}")
    A, B = pdsynth.exp_pd(500, 12), pdsynth.exp_pd(480, 13)
    compare(orc, ctx, A, B, eps=0.1, s_override=s_override)


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


def test_bracket_against_exact(orc, ctx):
    _say("[gpu] bracket vs Hungarian")
    for k in range(10):
        A, B = pdsynth.exp_pd(400, 2 * k), pdsynth.exp_pd(400, 2 * k + 1)
        g = ctx.approx(A, B, eps=0.1)
        ex = orc.exact_w1(A, B)
        assert g.lower_bound <= ex <= g.w1 <= 1.1 * ex


def test_batch_equals_single_and_oracle(orc, ctx):
    _say("[gpu] batch vs single")
    import paper_2110_14734_amd as w1

    sizes = pdsynth.batch_sizes(24, 99, lo=20, hi=3000)
    As = [pdsynth.exp_pd(int(sizes[i]), 1000 + 2 * i, dtype=np.float32) for i in range(12)]
    Bs = [pdsynth.exp_pd(int(sizes[12 + i]), 1001 + 2 * i, dtype=np.float32) for i in range(12)]
    As[3] = np.zeros((0, 2), np.float32)
    Bs[5] = As[5].copy()
    flags = w1.KEEP_NETWORK
    batch = ctx.approx_batch(As, Bs, eps=0.2, flags=flags)
    for i in range(12):
        single = ctx.approx(As[i], Bs[i], eps=0.2, flags=flags)
        r = orc.run(As[i], Bs[i], eps=0.2)
        for x in (batch[i], single):
            assert x.w1 == r.W1 and x.flow_cost == (r.flow if r.n else 0) and x.n_pairs == r.n_pairs
            assert x.lower_bound == r.L
        for f in ("pair_u", "pair_v", "pair_cost", "diag_src", "diag_dst", "supply", "cell_i", "cell_j"):
            assert np.array_equal(batch[i].network.get(f, np.zeros(0)), single.network.get(f, np.zeros(0))), f


def test_determinism_and_count_only(ctx):
    _say("[gpu] determinism")
    import paper_2110_14734_amd as w1

    A, B = pdsynth.mixture_pd(20000, 20), pdsynth.mixture_pd(19000, 21)
    g1 = ctx.approx(A, B, eps=0.2, flags=w1.KEEP_NETWORK | w1.NO_FLOW)
    g2 = ctx.approx(A, B, eps=0.2, flags=w1.KEEP_NETWORK | w1.NO_FLOW)
    for f in ("pair_u", "pair_v", "pair_cost", "diag_src", "supply"):
        assert np.array_equal(g1.network[f], g2.network[f]), f
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
    gu, gv, gc = _sorted_pairs(g_dev.network["pair_u"], g_dev.network["pair_v"], g_dev.network["pair_cost"])
    ou, ov, oc = _sorted_pairs(r.pairs["u"], r.pairs["v"], r.pairs["c"])
    assert np.array_equal(gu, ou) and np.array_equal(gv, ov) and np.array_equal(gc, oc)
    assert g_host.lower_bound <= g_host.w1


def _mix(u, v, c):
    u = u.astype(np.uint64)
    v = v.astype(np.uint64)
    c = c.astype(np.int64).astype(np.uint64)
    with np.errstate(over="ignore"):
        x = ((u + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15) + (v + np.uint64(1))) * np.uint64(0xC2B2AE3D27D4EB4F) + c
        x = x * np.uint64(0x165667B19E3779F9)
        return int(x.sum(dtype=np.uint64)), int((x * x).sum(dtype=np.uint64))


def test_full_size_config2(orc, ctx):
    """200k + 200k FP32 points (mixture), eps 0.2: every cell, L, the pair
    count and an order-independent checksum of all 6.8e8 pairs."""
    import paper_2110_14734_amd as w1

    _say("[gpu] full-size mixture 200k+200k eps 0.2")
    A, B = pdsynth.mixture_pd(200_000, 0), pdsynth.mixture_pd(200_000, 1)
    r = orc.run(A, B, eps=0.2, flags=orc.ORC_COUNT_ONLY)
    g = ctx.approx(A, B, eps=0.2, flags=w1.KEEP_NETWORK | w1.KEEP_STAGES | w1.NO_FLOW)
    assert g.lower_bound == r.L and g.grid_exp == r.e
    assert np.array_equal(g.stages["loc_t"], r.locs["t"])
    net = g.network
    assert np.array_equal(net["cell_i"], r.cells["i"]) and np.array_equal(net["cell_j"], r.cells["j"])
    assert np.array_equal(net["cell_ca"], r.cells["cA"]) and np.array_equal(net["cell_cb"], r.cells["cB"])
    assert g.n_pairs == r.n_pairs
    assert _mix(net["pair_u"], net["pair_v"], net["pair_cost"]) == r.checksum


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
            pa = _sorted_pairs(a.network["pair_u"], a.network["pair_v"], a.network["pair_cost"])
            pb = _sorted_pairs(b.network["pair_u"], b.network["pair_v"], b.network["pair_cost"])
            assert all(np.array_equal(x, y) for x, y in zip(pa, pb))
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
    records give the same pairs in the same order; a pair whose grid extent
    exceeds 2^28 cells, where the packed records cannot be used, still
    matches the oracle stage by stage."""
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
            for key in ("pair_u", "pair_v", "pair_cost"):
                assert np.array_equal(a.network[key], b.network[key])
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

"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and its host parts (parameter choice, network simplex) agree
with the oracle and with LP optimality conditions.  No GPU needed."""
import os
import re

import numpy as np
import pytest

import paper_2110_14734_amd as w1
import pdsynth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "w1approx.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(w1_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = w1.lib()
    declared = _header_functions()
    assert len(declared) >= 10
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(w1.EXPORTS) == declared


def test_strerror_and_separation(orc):
    assert w1.strerror(0) == "ok"
    assert "invalid" in w1.strerror(-1)
    for eps in (0.2, 0.1, 0.05, 0.01, 0.37):
        assert w1.separation_for_eps(eps) == orc.choose_s(eps)
    with pytest.raises(w1.W1Error):
        w1.separation_for_eps(0.0)


def test_context_without_gpu_fails_cleanly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(w1.W1Error) as e:
        w1.Context()
    assert e.value.code == w1.W1_ENODEV


def _certificate(n, src, dst, cost, supply, flow, pot):
    bal = np.zeros(n, np.int64)
    np.add.at(bal, src.astype(np.int64), flow)
    np.add.at(bal, dst.astype(np.int64), -flow)
    assert np.array_equal(bal, supply)
    assert (flow >= 0).all()
    red = cost.astype(np.int64) + pot[src] - pot[dst]
    assert (red >= 0).all()
    assert (red[flow > 0] == 0).all()


def test_network_simplex_random_networks(orc):
    rng = np.random.default_rng(17)
    for trial in range(40):
        n = int(rng.integers(3, 60))
        m = int(rng.integers(n, 8 * n))
        src = rng.integers(0, n, m)
        dst = rng.integers(0, n, m)
        keep = src != dst
        src = np.concatenate([src[keep], np.arange(n)])
        dst = np.concatenate([dst[keep], (np.arange(n) + 1) % n])
        cost = rng.integers(0, 30, src.shape[0])
        if trial % 3 == 0:
            cost[:] = rng.integers(0, 2, src.shape[0])  # many ties: degenerate pivots
        supply = rng.integers(-6, 7, n)
        supply[-1] -= supply.sum()
        c, piv, st, flow, pot = w1.flow_solve(n, src, dst, cost, supply, certificate=True)
        assert st == w1.W1_OPTIMAL
        assert c == orc.mcf(n, src, dst, cost, supply)
        _certificate(n, src, dst, cost, supply, flow, pot)


def test_network_simplex_on_oracle_networks(orc):
    # the sparse transshipment networks the method builds (oracle side)
    for seed in range(4):
        A = pdsynth.exp_pd(120, 2 * seed)
        B = pdsynth.exp_pd(110, 2 * seed + 1)
        src, dst, cost, sup = orc.network(A, B, eps=0.2)
        r = orc.run(A, B, eps=0.2)
        c, piv, st, flow, pot = w1.flow_solve(sup.shape[0], src, dst, cost, sup, certificate=True)
        assert c == r.flow
        _certificate(sup.shape[0], src.astype(np.uint32), dst.astype(np.uint32), cost, sup, flow, pot)


def test_network_simplex_full_size_network(orc):
    # the 400 + 400 point network at eps 0.1 (about 400k arcs, blocks that
    # wrap past the last arc, tens of thousands of pivots)
    A, B = pdsynth.exp_pd(400, 0), pdsynth.exp_pd(400, 1)
    src, dst, cost, sup = orc.network(A, B, eps=0.1)
    assert src.shape[0] > 300_000
    r = orc.run(A, B, eps=0.1)
    c, piv, st, flow, pot = w1.flow_solve(sup.shape[0], src, dst, cost, sup, certificate=True)
    assert st == w1.W1_OPTIMAL and piv > 1000
    assert c == r.flow
    _certificate(sup.shape[0], src.astype(np.uint32), dst.astype(np.uint32), cost, sup, flow, pot)


def test_network_simplex_pivot_cap_and_errors():
    src = np.array([0, 1, 0], np.uint32)
    dst = np.array([1, 2, 2], np.uint32)
    cost = np.array([1, 1, 5], np.int32)
    sup = np.array([3, 0, -3], np.int64)
    c, piv, st = w1.flow_solve(3, src, dst, cost, sup)
    assert c == 6 and st == w1.W1_OPTIMAL
    c2, piv2, st2 = w1.flow_solve(3, src, dst, cost, sup, pivot_cap=1)
    # after one pivot the 3 units still sit on artificial arcs: no flow that
    # meets the supplies has been reached, so no cost is reported
    assert st2 == w1.W1_STALLED and piv2 == 1 and c2 == -1
    c4, piv4, st4 = w1.flow_solve(3, src, dst, cost, sup, pivot_cap=2)
    assert (c4, piv4, st4) == (6, 2, w1.W1_OPTIMAL)
    with pytest.raises(w1.W1Error):
        w1.flow_solve(3, src, dst, cost, np.array([3, 0, -2], np.int64))  # unbalanced
    with pytest.raises(w1.W1Error):
        w1.flow_solve(3, src[:2], dst[:2], cost[:2], np.array([0, 3, -3], np.int64)[::-1].copy())  # infeasible
    with pytest.raises(w1.W1Error):
        w1.flow_solve(3, src, dst, np.array([1, -1, 5], np.int32), sup)  # negative cost
    with pytest.raises(w1.W1Error):
        w1.flow_solve(3, src, np.array([1, 3, 2], np.uint32), cost, sup)  # node out of range
    # no arcs: only an all-zero supply is feasible
    c3, piv3, st3 = w1.flow_solve(2, src[:0], dst[:0], cost[:0], np.zeros(2, np.int64))
    assert c3 == 0 and piv3 == 0 and st3 == w1.W1_OPTIMAL


def test_network_simplex_stalled_flows():
    """A solve stopped by the pivot cap reports a cost only for a flow that
    meets every supply; that flow is then a certified upper bound."""
    rng = np.random.default_rng(5)
    feasible_stalls = 0
    for trial in range(12):
        n = 40
        src = rng.integers(0, n, 300)
        dst = rng.integers(0, n, 300)
        keep = src != dst
        src = np.concatenate([src[keep], np.arange(n)]).astype(np.uint32)
        dst = np.concatenate([dst[keep], (np.arange(n) + 1) % n]).astype(np.uint32)
        cost = rng.integers(0, 50, src.shape[0]).astype(np.int32)
        supply = rng.integers(-5, 6, n)
        supply[-1] -= supply.sum()
        opt, piv, st = w1.flow_solve(n, src, dst, cost, supply)
        assert st == w1.W1_OPTIMAL
        for cap in range(1, piv):
            c, p, s, flow, pot = w1.flow_solve(n, src, dst, cost, supply, pivot_cap=cap, certificate=True)
            assert s == w1.W1_STALLED and p == cap
            if c == -1:
                continue
            feasible_stalls += 1
            bal = np.zeros(n, np.int64)
            np.add.at(bal, src.astype(np.int64), flow)
            np.add.at(bal, dst.astype(np.int64), -flow)
            assert np.array_equal(bal, supply) and (flow >= 0).all()
            assert c == int((cost.astype(np.int64) * flow).sum()) and c >= opt
    assert feasible_stalls > 0


def test_learned_form_entry_points_reject_bad_arguments():
    """The surrogate, 1-NN and tuning entry points validate their arguments
    before any device work (null handles, bad sizes, out-of-range values)."""
    import ctypes

    L = w1.lib()
    vp = ctypes.c_void_p
    out = vp()
    assert L.w1_surrogate_create(None, ctypes.c_uint64(0), ctypes.byref(out)) == w1.W1_EINVAL
    assert L.w1_surrogate_destroy(None) == w1.W1_EINVAL
    buf = (ctypes.c_float * w1.SURR_NPARAM)()
    assert L.w1_surrogate_get_params(None, buf, w1.SURR_NPARAM) == w1.W1_EINVAL
    assert L.w1_surrogate_set_params(None, buf, w1.SURR_NPARAM) == w1.W1_EINVAL
    t = (ctypes.c_double * 3)()
    assert L.w1_surrogate_last_times(None, t, 3) == w1.W1_EINVAL
    assert L.w1_nn_build(None, None, None, 0, 0, None, ctypes.byref(out)) == w1.W1_EINVAL
    assert L.w1_nn_destroy(None) == w1.W1_EINVAL
    prm = w1._NNParams(0.1, w1.NN_RWMD, 0)
    nn = (ctypes.c_int64 * 1)()
    assert L.w1_nn_query(None, None, None, None, 1, ctypes.byref(prm), 0, None, nn, None, None,
                         None) == w1.W1_EINVAL
    assert L.w1_ctx_set_tuning(None, None) == w1.W1_EINVAL
    tun = w1._Tuning()
    assert L.w1_ctx_get_tuning(None, ctypes.byref(tun)) == w1.W1_EINVAL
    assert L.w1_surrogate_embed(None, None, None, 0, 0, None, None) == w1.W1_EINVAL
    assert L.w1_surrogate_grad(None, None, None, 0, None, None, None, 0, 0, None, None, None) == w1.W1_EINVAL
    assert L.w1_surrogate_train(None, None, None, 0, None, None, None, 0, None, 0, None, None) == w1.W1_EINVAL


def test_tune_workload_keys():
    """The autotuner's cache key depends on the workload's size class and mode only."""
    from paper_2110_14734_amd import tune

    A = [np.zeros((1000, 2))] * 4
    B = [np.zeros((3000, 2))] * 4
    k1 = tune.workload_key(A, B, 0.1, True)
    k2 = tune.workload_key(A, B, 0.1, False)
    assert k1 != k2 and k1.endswith("count") and k2.endswith("emit")
    assert k1.startswith("pts2^14/pair2^12/")
    assert tune.workload_key(A, B, 0.05, True) != k1


def test_nn_query_marshalling(monkeypatch):
    """The 1-NN binding passes mode, seed_k and keep through to the C-ABI
    structure (checked with a stand-in for the library; no GPU)."""
    import ctypes

    assert ctypes.sizeof(w1._NNParams) == 24 and ctypes.sizeof(w1._NNStats) == 72
    seen = []

    class Fake:
        def w1_nn_build(self, *a):
            return 0

        def w1_nn_query(self, ctx, idx, sur, arr, nq, prm, *rest):
            p = prm._obj
            seen.append((p.eps, p.mode, p.seed_k, p.keep, p.reserved, sur))
            return 0

        def w1_nn_destroy(self, *a):
            return 0

    monkeypatch.setattr(w1, "lib", lambda: Fake())

    class Ctx:
        _h = None

    db = [np.array([[0.0, 1.0]])]
    idx = w1.NNIndex(Ctx(), db)
    idx.query(db, eps=0.2, mode="pipeline", seed_k=3, keep=15)
    idx.query(db, eps=0.1, mode="sparse")
    idx.query(db, eps=0.1, mode="rwmd", seed_k=2)
    idx.close()
    assert seen == [(0.2, w1.NN_PIPELINE, 3, 15, 0, None), (0.1, w1.NN_SPARSE, 0, 0, 0, None),
                    (0.1, w1.NN_RWMD, 2, 0, 0, None)]


def test_tune_cache_lookup():
    """The tuning cache: the exact key first, else the same device, points
    per pair, eps and mode with the closest total size."""
    from paper_2110_14734_amd import tune

    data = {"dev/pts2^23/pair2^14/eps0.1/count": {"v": 1}, "dev/pts2^19/pair2^14/eps0.1/count": {"v": 2},
            "dev/pts2^26/pair2^14/eps0.1/emit": {"v": 3}, "other/pts2^26/pair2^14/eps0.1/count": {"v": 4}}
    assert tune.lookup(data, "dev", "pts2^23/pair2^14/eps0.1/count") == {"v": 1}
    assert tune.lookup(data, "dev", "pts2^26/pair2^14/eps0.1/count") == {"v": 1}
    assert tune.lookup(data, "dev", "pts2^20/pair2^14/eps0.1/count") == {"v": 2}
    assert tune.lookup(data, "dev", "pts2^26/pair2^15/eps0.1/count") is None
    assert tune.lookup(data, "dev", "pts2^26/pair2^14/eps0.2/count") is None

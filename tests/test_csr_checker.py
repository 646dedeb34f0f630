"""The row checker used by the full-size GPU parity test (tests/native/
csr_check.cpp) run on the oracle's own network: it must accept it, reproduce
the oracle's pair count and pair checksum in both orientations, and reject
planted mistakes (a swapped pair of heads, a wrong cost, a missing or extra
diagonal arc, a wrong B-diagonal row)."""
import ctypes

import numpy as np
import pytest

import pdsynth


def _run(L, net, r, chunk=None):
    n = net["n_cells"]
    rp = net["row_ptr"]
    col = net["col"].astype(np.uint32)
    cost = net["cost"].astype(np.int32)
    ci, cj = r.cells["i"].astype(np.int32), r.cells["j"].astype(np.int32)
    ca, cb = r.cells["cA"].astype(np.int32), r.cells["cB"].astype(np.int32)
    sums = np.zeros(4, np.uint64)
    counts = np.zeros(2, np.int64)
    first = ctypes.c_int64(-1)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    bad = 0
    step = chunk or (n + 2)
    for r0 in range(0, n + 2, step):
        r1 = min(n + 2, r0 + step)
        a0, a1 = int(rp[r0]), int(rp[r1])
        c, k = np.ascontiguousarray(col[a0:a1]), np.ascontiguousarray(cost[a0:a1])
        bad += L.csr_check_rows(n, r0, r1, p(rp), a0, a1 - a0, p(c), p(k), p(ci), p(cj), p(ca), p(cb),
                                p(sums), p(counts), ctypes.byref(first))
    return bad, sums, counts


def test_checker_accepts_oracle_network_and_catches_mistakes(orc, csr_checker):
    checker = csr_checker
    A, B = pdsynth.mixture_pd(700, 41), pdsynth.mixture_pd(650, 42)
    r = orc.run(A, B, eps=0.1, flags=orc.ORC_COUNT_ONLY)
    net = orc.csr(A, B, eps=0.1)
    for chunk in (None, 37):
        bad, sums, counts = _run(checker, net, r, chunk)
        assert bad == 0
        assert counts[0] == counts[1] == r.n_pairs
        assert (int(sums[0]), int(sums[1])) == r.checksum and (int(sums[2]), int(sums[3])) == r.checksum
    n, rp = net["n_cells"], net["row_ptr"]
    row = int(np.argmax(np.diff(rp)[:n]))
    a = int(rp[row])

    def planted(edit):
        m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in net.items()}
        edit(m)
        return _run(checker, m, r)[0]

    def swap(m):
        m["col"][a], m["col"][a + 1] = m["col"][a + 1], m["col"][a]

    def wrong_cost(m):
        m["cost"][a] += 2

    assert planted(swap) > 0
    assert planted(wrong_cost) > 0
    # a cell with A mass whose arc to the A-diagonal node is replaced
    cA = r.cells["cA"]
    c = int(np.flatnonzero(cA > 0)[0])

    def no_diag(m):
        m["col"][int(rp[c + 1]) - 1] = m["col"][int(rp[c + 1]) - 2] + 1 if rp[c + 1] - rp[c] > 1 else 0

    assert planted(no_diag) > 0

    def bdiag(m):
        m["cost"][int(rp[n + 1])] += 1

    assert planted(bdiag) > 0
    # a head moved to another cell, kept sorted and with the right cost for
    # that cell, passes the row check but not the checksum
    ci, cj = r.cells["i"], r.cells["j"]
    m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in net.items()}
    cols = m["col"][int(rp[row]):int(rp[row + 1])]
    k = int(np.flatnonzero((np.diff(cols) > 1) & (cols[1:] < n))[0])
    h = int(cols[k]) + 1
    m["col"][int(rp[row]) + k] = h
    m["cost"][int(rp[row]) + k] = 2 * max(abs(int(ci[row]) - int(ci[h])), abs(int(cj[row]) - int(cj[h])))
    bad, sums, _ = _run(checker, m, r)
    assert bad == 0 and (int(sums[0]), int(sums[1]), int(sums[2]), int(sums[3])) != r.checksum * 2

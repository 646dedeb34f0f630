"""CPU oracle for the approximate W1 pipeline (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links
or calls it, and it shares no code with the GPU library.

Contents
* ``run``            the plain pipeline (oracle.cpp) through ctypes.
* ``network``, ``csr`` its sparse transshipment network as an arc list, and
                     as (tail, head)-sorted compressed sparse rows.
* ``mcf``            exact min-cost flow (successive shortest paths).
* ``exact_w1``       exact W1 by Hungarian matching on the diagonal-augmented
                     bipartite graph Bi(A, B) (Sec. 4.3), L-infinity metric.
* ``brute_w1``       exhaustive partial matchings for tiny diagrams.
* ``wspd_coverage``  brute-force WSPD checks on small cell sets.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "_oracle.so")

ORC_STOP_AFTER_TREE = 1
ORC_COUNT_ONLY = 2
ORC_NO_FLOW = 4
ORC_KEEP_PAIR_NODES = 8
ORC_SKIP_RWMD = 16
ORC_PRUNE = 32
ORC_L2 = 64
ORC_PAPER_GRID = 128

STAGE_NAMES = ("O0-O1 condense", "O2 RWMD", "O3-O5 grid + Morton", "O6 tree", "O7 WSPD", "O8 network",
               "O9 flow")
_K = dict(STATUS=0, NA=1, NB=2, N=3, NLOC=4, S=5, E=6, M0=7, NCELLS=8, NNODES=9, ROOT=10,
          NPAIRS=11, FLOW=12, SA=13, SB=14, FA=15, FB=16, CHK1=17, CHK2=18, COSTK=19)
_D = dict(L=0, LA=1, LB=2, W1=3, W1P=4, G=5, EPSC=6)


def build(force: bool = False) -> str:
    """Compile oracle.cpp into a shared library next to it (g++, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        vp, i64, f64, ip = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        L.orc_new.restype = vp
        L.orc_free.argtypes = [vp]
        L.orc_run.argtypes = [vp, vp, i64, vp, i64, f64, f64, ip, ip, f64]
        L.orc_run.restype = ip
        L.orc_i64.argtypes = [vp, ip]
        L.orc_i64.restype = i64
        L.orc_f64.argtypes = [vp, ip]
        L.orc_f64.restype = f64
        for name in ("orc_locs", "orc_cells", "orc_nodes", "orc_pairs"):
            getattr(L, name).restype = None
        L.orc_locs.argtypes = [vp] * 6
        L.orc_cells.argtypes = [vp] * 6
        L.orc_nodes.argtypes = [vp, vp]
        L.orc_pairs.argtypes = [vp] * 6
        L.orc_network.argtypes = [vp] * 5
        L.orc_network.restype = i64
        L.orc_csr.argtypes = [vp] * 4
        L.orc_csr.restype = i64
        L.orc_mcf.argtypes = [i64, i64, vp, vp, vp, vp, vp, vp]
        L.orc_mcf.restype = i64
        L.orc_stage_seconds.argtypes = [vp, vp]
        L.orc_stage_seconds.restype = None
        L.orc_choose_s.argtypes = [f64, f64]
        L.orc_choose_s.restype = ip
        L.orc_grid_exponent.argtypes = [f64, f64, i64, ip]
        L.orc_grid_exponent.restype = ip
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _as_f64(X) -> np.ndarray:
    X = np.asarray(X)
    if X.size == 0:
        return np.zeros((0, 2), np.float64)
    return np.ascontiguousarray(X, dtype=np.float64).reshape(-1, 2)


@dataclass
class Result:
    status: int
    nA: int = 0
    nB: int = 0
    n: int = 0
    s: int = 0
    e: int = 0
    m0: int = 0
    L: float = 0.0
    LA: float = 0.0
    LB: float = 0.0
    SA: int = 0
    SB: int = 0
    FA: int = 0
    FB: int = 0
    g: float = 0.0
    eps_c: float = 0.0
    W1: float = 0.0
    W1_paper: float = 0.0
    flow: int = -1
    n_pairs: int = 0
    checksum: tuple = (0, 0)
    locs: dict = field(default_factory=dict)
    cells: dict = field(default_factory=dict)
    nodes: np.ndarray | None = None
    root: int = -1
    pairs: dict = field(default_factory=dict)
    stage_s: dict = field(default_factory=dict)
    K: int = 0


def run(A, B, eps: float = 0.1, kappa: float = 0.1, s_override: int = 0, flags: int = 0,
        given_L: float = 0.0, fetch: bool = True) -> Result:
    """Run the oracle pipeline.  A, B: (n, 2) arrays of (birth, death)."""
    L_ = lib()
    A64, B64 = _as_f64(A), _as_f64(B)
    h = L_.orc_new()
    try:
        st = L_.orc_run(h, _ptr(A64), A64.shape[0], _ptr(B64), B64.shape[0], float(eps), float(kappa),
                        int(s_override), int(flags), float(given_L))
        gi = lambda k: int(L_.orc_i64(h, _K[k]))
        gd = lambda k: float(L_.orc_f64(h, _D[k]))
        r = Result(status=st)
        if st != 0:
            return r
        r.nA, r.nB, r.n, r.s, r.e, r.m0 = gi("NA"), gi("NB"), gi("N"), gi("S"), gi("E"), gi("M0")
        r.L, r.LA, r.LB, r.g, r.eps_c = gd("L"), gd("LA"), gd("LB"), gd("G"), gd("EPSC")
        r.SA, r.SB, r.FA, r.FB = gi("SA"), gi("SB"), gi("FA"), gi("FB")
        r.W1, r.W1_paper, r.flow, r.n_pairs = gd("W1"), gd("W1P"), gi("FLOW"), gi("NPAIRS")
        r.checksum = (gi("CHK1") & (2**64 - 1), gi("CHK2") & (2**64 - 1))
        r.root = gi("ROOT")
        r.K = gi("COSTK")
        st = np.zeros(7)
        L_.orc_stage_seconds(h, _ptr(st))
        r.stage_s = dict(zip(STAGE_NAMES, st.tolist()))
        if not fetch:
            return r
        m = gi("NLOC")
        b, d, t, term = (np.zeros(m) for _ in range(4))
        w = np.zeros(m, np.int64)
        L_.orc_locs(h, _ptr(b), _ptr(d), _ptr(w), _ptr(t), _ptr(term))
        r.locs = dict(b=b, d=d, w=w, t=t, term=term)
        N = gi("NCELLS")
        ci, cj, ca, cb = (np.zeros(N, np.int64) for _ in range(4))
        key = np.zeros(N, np.uint64)
        L_.orc_cells(h, _ptr(ci), _ptr(cj), _ptr(ca), _ptr(cb), _ptr(key))
        r.cells = dict(i=ci, j=cj, cA=ca, cB=cb, key=key)
        nn = gi("NNODES")
        nodes = np.zeros((nn, 10), np.int64)
        L_.orc_nodes(h, _ptr(nodes))
        r.nodes = nodes
        P = r.n_pairs if not (flags & ORC_COUNT_ONLY) else 0
        if P:
            u, v, c, nu, nv = (np.zeros(P, np.int64) for _ in range(5))
            keep = bool(flags & ORC_KEEP_PAIR_NODES)
            L_.orc_pairs(h, _ptr(u), _ptr(v), _ptr(c), _ptr(nu) if keep else None, _ptr(nv) if keep else None)
            r.pairs = dict(u=u, v=v, c=c)
            if keep:
                r.pairs.update(nu=nu, nv=nv)
        else:
            z = np.zeros(0, np.int64)
            r.pairs = dict(u=z, v=z, c=z)
        return r
    finally:
        L_.orc_free(h)


def network(A, B, eps=0.1, kappa=0.1, s_override=0, prune=False, l2=False, paper_grid=False):
    """Sparse transshipment network of the oracle: (src, dst, cost, supply).
    prune: leave out the diagonal-dominated WSPD pairs (O7'); paper_grid: the
    grid of Alg. 2 / Alg. 3 for the given s_override."""
    L_ = lib()
    A64, B64 = _as_f64(A), _as_f64(B)
    h = L_.orc_new()
    try:
        st = L_.orc_run(h, _ptr(A64), A64.shape[0], _ptr(B64), B64.shape[0], float(eps), float(kappa),
                        int(s_override), ORC_NO_FLOW | (ORC_PRUNE if prune else 0) | (ORC_L2 if l2 else 0)
                        | (ORC_PAPER_GRID if paper_grid else 0), 0.0)
        if st != 0:
            raise RuntimeError(f"oracle status {st}")
        m = int(L_.orc_network(h, None, None, None, None))
        N = int(L_.orc_i64(h, _K["NCELLS"]))
        src, dst, cost = (np.zeros(m, np.int64) for _ in range(3))
        sup = np.zeros(N + 2, np.int64)
        L_.orc_network(h, _ptr(src), _ptr(dst), _ptr(cost), _ptr(sup))
        return src, dst, cost, sup
    finally:
        L_.orc_free(h)


def csr(A, B, eps=0.1, kappa=0.1, s_override=0, prune=False, l2=False, paper_grid=False):
    """The oracle's network in compressed sparse row form (O8): arcs sorted by
    (tail, head).  Returns dict(row_ptr, col, cost, supply, n_cells).
    prune: leave out the diagonal-dominated WSPD pairs (O7'); paper_grid: the
    grid of Alg. 2 / Alg. 3 for the given s_override."""
    L_ = lib()
    A64, B64 = _as_f64(A), _as_f64(B)
    h = L_.orc_new()
    try:
        st = L_.orc_run(h, _ptr(A64), A64.shape[0], _ptr(B64), B64.shape[0], float(eps), float(kappa),
                        int(s_override), ORC_NO_FLOW | (ORC_PRUNE if prune else 0) | (ORC_L2 if l2 else 0)
                        | (ORC_PAPER_GRID if paper_grid else 0), 0.0)
        if st != 0:
            raise RuntimeError(f"oracle status {st}")
        N = int(L_.orc_i64(h, _K["NCELLS"]))
        if int(L_.orc_i64(h, _K["N"])) == 0:
            z = np.zeros(0, np.int64)
            return dict(row_ptr=np.zeros(3, np.int64), col=z, cost=z, supply=np.zeros(2, np.int64), n_cells=0)
        m = int(L_.orc_csr(h, None, None, None))
        rp = np.zeros(N + 3, np.int64)
        col, cost = np.zeros(m, np.int64), np.zeros(m, np.int64)
        L_.orc_csr(h, _ptr(rp), _ptr(col), _ptr(cost))
        sup = np.zeros(N + 2, np.int64)
        src_, dst_, c_ = (np.zeros(m, np.int64) for _ in range(3))
        L_.orc_network(h, _ptr(src_), _ptr(dst_), _ptr(c_), _ptr(sup))
        return dict(row_ptr=rp, col=col, cost=cost, supply=sup, n_cells=N)
    finally:
        L_.orc_free(h)


def mcf(n_nodes, src, dst, cost, supply, want_certificate=False):
    """Exact uncapacitated min-cost flow; returns cost (and flow, potentials)."""
    L_ = lib()
    src = np.ascontiguousarray(src, np.int64)
    dst = np.ascontiguousarray(dst, np.int64)
    cost = np.ascontiguousarray(cost, np.int64)
    supply = np.ascontiguousarray(supply, np.int64)
    flow = np.zeros(src.shape[0], np.int64)
    pot = np.zeros(n_nodes, np.int64)
    c = int(L_.orc_mcf(n_nodes, src.shape[0], _ptr(src), _ptr(dst), _ptr(cost), _ptr(supply), _ptr(flow), _ptr(pot)))
    if want_certificate:
        return c, flow, pot
    return c


def choose_s(eps: float, kappa: float = 0.1) -> int:
    return int(lib().orc_choose_s(float(eps), float(kappa)))


def grid_exponent(eps_c: float, L: float, n: int, l2: bool = False) -> int:
    return int(lib().orc_grid_exponent(float(eps_c), float(L), int(n), int(bool(l2))))


# ------------------------------------------------------------- exact W1 --
def _clean(X):
    X = _as_f64(X)
    return X[X[:, 1] != X[:, 0]]


def _ground(P, Q, l2):
    """Ground distances between point sets (rows (birth, death))."""
    db = P[:, None, 0] - Q[None, :, 0]
    dd = P[:, None, 1] - Q[None, :, 1]
    return np.hypot(db, dd) if l2 else np.maximum(np.abs(db), np.abs(dd))


def _to_diag(P, l2):
    """Distance to the diagonal: (d - b)/sqrt(2) (Euclidean), (d - b)/2 (L-infinity)."""
    return (P[:, 1] - P[:, 0]) / np.sqrt(2.0) if l2 else 0.5 * (P[:, 1] - P[:, 0])


def exact_w1(A, B, l2=False) -> float:
    """Exact W1 by a min-weight perfect matching on Bi(A, B), L-infinity or
    (l2=True) Euclidean ground metric.

    Rows are the points of A followed by the diagonal projections of B's
    points; columns are B's points followed by A's projections (Sec. 4.3):
    A-B edges cost the ground distance, a point and its own projection cost
    the distance to the diagonal, projection-projection edges cost 0, every
    other edge is forbidden.
    """
    from scipy.optimize import linear_sum_assignment

    A, B = _clean(A), _clean(B)
    na, nb = A.shape[0], B.shape[0]
    if na + nb == 0:
        return 0.0
    dA = _to_diag(A, l2)
    dB = _to_diag(B, l2)
    big = 4.0 * (float(dA.sum() + dB.sum()) + 1.0) + 4.0 * float(np.abs(np.concatenate([A, B])).max(initial=0.0)) * (na + nb)
    C = np.full((na + nb, nb + na), big)
    if na and nb:
        C[:na, :nb] = _ground(A, B, l2)
    C[:na, nb:] = np.where(np.eye(na, dtype=bool), dA[:, None], big) if na else C[:na, nb:]
    C[na:, :nb] = np.where(np.eye(nb, dtype=bool), dB[None, :], big) if nb else C[na:, :nb]
    C[na:, nb:] = 0.0
    r, c = linear_sum_assignment(C)
    return float(C[r, c].sum())


def brute_w1(A, B, l2=False) -> float:
    """Exact W1 by enumerating every partial matching (tiny inputs only)."""
    A, B = _clean(A), _clean(B)
    na, nb = A.shape[0], B.shape[0]
    dA = list(_to_diag(A, l2))
    dB = list(_to_diag(B, l2))
    best = float("inf")
    for k in range(min(na, nb) + 1):
        for ia in itertools.combinations(range(na), k):
            for ib in itertools.permutations(range(nb), k):
                cost = 0.0
                for x, y in zip(ia, ib):
                    cost += (float(np.hypot(A[x, 0] - B[y, 0], A[x, 1] - B[y, 1])) if l2
                             else max(abs(A[x, 0] - B[y, 0]), abs(A[x, 1] - B[y, 1])))
                cost += sum(dA[x] for x in range(na) if x not in ia)
                cost += sum(dB[y] for y in range(nb) if y not in ib)
                best = min(best, cost)
    return best if (na + nb) else 0.0


# ------------------------------------------------------ brute-force checks --
def wspd_coverage(res: Result, l2: bool = False) -> None:
    """Assert every unordered pair of distinct cells is covered by exactly one
    output pair and every output pair is s-well-separated (boxes recomputed
    from the member cells; L-infinity: gap >= s * longest side; Euclidean:
    gap >= s * longest diagonal, on exact integer squares).  Needs
    ORC_KEEP_PAIR_NODES."""
    N = res.cells["i"].shape[0]
    ci, cj = res.cells["i"], res.cells["j"]
    nodes = res.nodes
    cover = np.zeros((N, N), np.int64)
    for U, V in zip(res.pairs["nu"], res.pairs["nv"]):
        lu, hu = nodes[U, 0], nodes[U, 1]
        lv, hv = nodes[V, 0], nodes[V, 1]
        cover[lu:hu + 1, lv:hv + 1] += 1
        iu, ju = ci[lu:hu + 1], cj[lu:hu + 1]
        iv, jv = ci[lv:hv + 1], cj[lv:hv + 1]
        if l2:
            gi = max(0, int(iu.min() - iv.max()), int(iv.min() - iu.max()))
            gj = max(0, int(ju.min() - jv.max()), int(jv.min() - ju.max()))
            d2 = max(int(iu.max() - iu.min()) ** 2 + int(ju.max() - ju.min()) ** 2,
                     int(iv.max() - iv.min()) ** 2 + int(jv.max() - jv.min()) ** 2)
            assert gi * gi + gj * gj >= res.s ** 2 * d2, (U, V, gi, gj, d2)
        else:
            diam = max(iu.max() - iu.min(), ju.max() - ju.min(), iv.max() - iv.min(), jv.max() - jv.min())
            gap = max(0, iu.min() - iv.max(), iv.min() - iu.max(), ju.min() - jv.max(), jv.min() - ju.max())
            assert gap >= res.s * diam, (U, V, gap, diam)
    sym = cover + cover.T
    off = ~np.eye(N, dtype=bool)
    assert np.all(sym[off] == 1), "pair of cells not covered exactly once"
    assert np.all(np.diag(sym) == 0)

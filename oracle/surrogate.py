"""Oracle for the learned form (test infrastructure only): the DeepSets
surrogate's forward pass and gradient, the dual lower bound, and exhaustive
1-NN search.  Only the test suite, ``__graft_entry__.smoke()`` and the CPU
baseline of ``bench.py`` may import it; the GPU library never does.

Network (the 1-NN problem is Problem NN of Sec. 6; the network itself is not
in the paper, it only orders candidates):
    x = (birth, death - birth) of each off-diagonal point
    h1 = ReLU(W1 x + b1)          2 -> 128
    h2 = ReLU(W2 h1 + b2)         128 -> 128
    pool = sum of h2 over the points
    e = W3 pool + b3              128 -> 64,  prediction ||e_A - e_B||_2
    loss = (1/P) sum_j ((||e_a - e_b|| - w_j) / w_j)^2

``emulate=True`` places the roundings the library's precision contract
names.  x is first rounded to FP32 and then written as hi + lo, with hi =
bf16(x) and lo = bf16(x - hi).  W1, b1, W2 and h1 are rounded to BF16.  The
gradient of dZ2 enters both weight products as bf16(dpool).  Everything else
is exact FP64.  The roundings pass gradients unchanged (straight-through).
``emulate=False`` is the plain FP64 network; finite differences pin its
gradient.
"""
from __future__ import annotations

import numpy as np

H, E = 128, 64
OFF_W1, OFF_B1 = 0, 256
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + E * H
NPARAM = OFF_B3 + E  # 25152
NSTATS = 33


def bf16(x) -> np.ndarray:
    """Round to the nearest BF16 value (8 significant bits), ties to even."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)                    # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)


def unpack(p) -> dict:
    """Parameter tensors.  A FP32 vector (the library's master parameters) is
    widened exactly; a FP64 vector is used as it is."""
    p = np.asarray(p)
    if p.dtype != np.float64:
        p = p.astype(np.float32).astype(np.float64)
    assert p.shape == (NPARAM,)
    return dict(W1=p[OFF_W1:OFF_B1].reshape(H, 2), b1=p[OFF_B1:OFF_W2], W2=p[OFF_W2:OFF_B2].reshape(H, H),
                b2=p[OFF_B2:OFF_W3], W3=p[OFF_W3:OFF_B3].reshape(E, H), b3=p[OFF_B3:NPARAM])


def features(A) -> np.ndarray:
    """(birth, death - birth) of the off-diagonal points, each rounded to
    FP32 (the difference is taken in FP64 first)."""
    A = np.asarray(A, np.float64).reshape(-1, 2)
    if A.size and (not np.isfinite(A).all() or (A[:, 1] < A[:, 0]).any()):
        raise ValueError("invalid diagram point")
    A = A[A[:, 1] > A[:, 0]]
    x = np.stack([A[:, 0], A[:, 1] - A[:, 0]], axis=1) if len(A) else np.zeros((0, 2))
    return x.astype(np.float32).astype(np.float64)


def _weights(P, emulate):
    if not emulate:
        return P["W1"], P["b1"], P["W2"]
    return bf16(P["W1"]), bf16(P["b1"]), bf16(P["W2"])


def _inputs(x, emulate):
    if not emulate:
        return x
    hi = bf16(x)
    return hi + bf16(x - hi)


def forward(p, diagrams, emulate=True):
    """Embeddings (D x 64) and the per-diagram intermediates."""
    P = unpack(p)
    W1, b1, W2 = _weights(P, emulate)
    emb, cache = [], []
    for A in diagrams:
        x = _inputs(features(A), emulate)
        z1 = x @ W1.T + b1
        h1 = np.maximum(z1, 0.0)
        if emulate:
            h1 = bf16(h1)
        z2 = h1 @ W2.T + P["b2"]
        h2 = np.maximum(z2, 0.0)
        pool = h2.sum(axis=0)
        emb.append(P["W3"] @ pool + P["b3"])
        cache.append((x, h1, z2, pool))
    return np.array(emb).reshape(-1, E), cache


def loss_grad(p, diagrams, pa, pb, w, emulate=True):
    """Loss and its gradient with respect to the parameter vector."""
    P = unpack(p)
    W1, b1, W2 = _weights(P, emulate)
    emb, cache = forward(p, diagrams, emulate)
    pa, pb, w = np.asarray(pa), np.asarray(pb), np.asarray(w, np.float64)
    nP = len(w)
    demb = np.zeros_like(emb)
    loss = 0.0
    for j in range(nP):
        diff = emb[pa[j]] - emb[pb[j]]
        pred = np.sqrt(diff @ diff)
        rel = (pred - w[j]) / w[j]
        loss += rel * rel / nP
        if pred > 0:
            g = 2.0 * rel / (w[j] * nP) / pred * diff
            demb[pa[j]] += g
            demb[pb[j]] -= g
    grad = np.zeros(NPARAM)
    gW1, gb1, gW2, gb2 = (np.zeros((H, 2)), np.zeros(H), np.zeros((H, H)), np.zeros(H))
    gW3 = np.zeros((E, H))
    gb3 = demb.sum(axis=0)
    for d, (x, h1, z2, pool) in enumerate(cache):
        gW3 += np.outer(demb[d], pool)
        dpool = P["W3"].T @ demb[d]
        mask2 = z2 > 0.0
        gb2 += (mask2 * dpool).sum(axis=0)
        dz2 = mask2 * (bf16(dpool) if emulate else dpool)
        gW2 += dz2.T @ h1
        dh1 = dz2 @ W2
        dz1 = dh1 * (h1 > 0.0)
        gW1 += dz1.T @ x
        gb1 += dz1.sum(axis=0)
    grad[OFF_W1:OFF_B1] = gW1.ravel()
    grad[OFF_B1:OFF_W2] = gb1
    grad[OFF_W2:OFF_B2] = gW2.ravel()
    grad[OFF_B2:OFF_W3] = gb2
    grad[OFF_W3:OFF_B3] = gW3.ravel()
    grad[OFF_B3:NPARAM] = gb3
    return loss, grad


# ---------------------------------------------------------------- 1-NN --
def dual_stats(A) -> np.ndarray:
    """Sums over the points of f_c(x) = max(0, (d - b)/2 - c) for c = 0 and
    c = 2^-20 .. 2^11 (33 test functions, each 1-Lipschitz in L-infinity and
    zero on the diagonal)."""
    A = np.asarray(A, np.float64).reshape(-1, 2)
    h = (A[:, 1] - A[:, 0]) * 0.5
    cs = np.concatenate([[0.0], np.ldexp(1.0, np.arange(-20, 12))])
    return np.array([np.maximum(0.0, h - c).sum() for c in cs])


def dual_bound(A, B) -> float:
    """max_c |sum_A f_c - sum_B f_c| <= W1(A, B) (Kantorovich duality)."""
    return float(np.abs(dual_stats(A) - dual_stats(B)).max())


def wcd_half(A, B, l2=False) -> float:
    """Half the word centroid distance of the diagonal-augmented diagrams
    (appendix, WCD): with A~ and B~ the diagonal projections of A's and B's
    points, the classical transport distance between A u B~ and B u A~ is at
    most 2 W1(A, B), and the distance of the two sums (total masses equal)
    is at most that transport distance, so half of it is a lower bound.
    Computed as written: the augmented sets, their coordinate sums, the norm
    of the difference (L-infinity, or Euclidean with l2)."""
    A = np.asarray(A, np.float64).reshape(-1, 2)
    B = np.asarray(B, np.float64).reshape(-1, 2)
    proj = lambda X: np.repeat(((X[:, 0] + X[:, 1]) * 0.5)[:, None], 2, axis=1)
    left = np.concatenate([A, proj(B)])
    right = np.concatenate([B, proj(A)])
    d = left.sum(axis=0) - right.sum(axis=0)
    return 0.5 * float(np.hypot(d[0], d[1]) if l2 else np.abs(d).max())


def nn_pipeline(db, queries, eps=0.1, keep=15, c2=3):
    """The keep-c2-1 pipeline of the 1-NN experiments (Sec. 7), with RWMD as
    its first stage: the keep candidates of smallest RWMD (ties to the lower
    index), of those the c2 of smallest method value at s = 1 on the paper's
    grid for s = 1 (ties to the earlier in RWMD order), and the best certified
    W1 at eps among them (ties to the lower index).  Returns (index, W1) per
    query.  Not exact: the nearest neighbour may be cut."""
    from . import ORC_PAPER_GRID, ORC_STOP_AFTER_TREE, run

    out = []
    for q in queries:
        L = []
        for D in db:
            r = run(q, D, eps=eps, flags=ORC_STOP_AFTER_TREE, fetch=False)
            if r.status != 0:
                raise RuntimeError(f"oracle status {r.status}")
            L.append(r.L)
        order = sorted(range(len(db)), key=lambda i: (L[i], i))[:keep]
        s1 = {}
        for i in order:
            r = run(q, db[i], eps=eps, s_override=1, flags=ORC_PAPER_GRID, fetch=False)
            if r.status != 0:
                raise RuntimeError(f"oracle status {r.status}")
            s1[i] = r.W1
        pos = {i: k for k, i in enumerate(order)}
        cand = sorted(order, key=lambda i: (s1[i], pos[i]))[:c2]
        best, bi = np.inf, -1
        for i in sorted(cand):
            r = run(q, db[i], eps=eps, fetch=False)
            if r.status != 0:
                raise RuntimeError(f"oracle status {r.status}")
            if r.W1 < best:
                best, bi = r.W1, i
        out.append((bi, best))
    return out


def nn_exhaustive(db, queries, eps=0.1):
    """Problem NN (Sec. 6) by exhaustive search over the oracle's certified
    W1 at eps; ties go to the lowest index.  Returns (index, W1) per query."""
    from . import run

    out = []
    for q in queries:
        best, bi = np.inf, -1
        for i, D in enumerate(db):
            r = run(q, D, eps=eps, fetch=False)
            if r.status != 0:
                raise RuntimeError(f"oracle status {r.status}")
            if r.W1 < best:
                best, bi = r.W1, i
        out.append((bi, best))
    return out


# --- element-wise gradient bound (used by the GPU parity test and the smoke check) ---

def dyadic_case(seed=11):
    """Parameters and points on coarse dyadic grids (W1, b1 in steps of 2^-3,
    W2 and W3 of 2^-2, all within [-1/2, 1/2]; b2 in steps of 2^-9, b3 of
    2^-11; births and persistences in steps of 2^-4 below 1/2; at most 8
    points per diagram), so that every product of the forward pass is exact
    in FP32, every h1 is a BF16 number, and every sum is exact in any order
    (checked below through the magnitude sums).  The only rounding left is
    in the per-pair loss coefficients and in the backward sums."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM)
    q = lambda n, step: rng.integers(-int(0.5 / step), int(0.5 / step) + 1, n) * step
    p[OFF_W1:OFF_B1], p[OFF_B1:OFF_W2] = q(256, 2.0**-3), q(128, 2.0**-3)
    p[OFF_W2:OFF_B2], p[OFF_B2:OFF_W3] = q(128 * 128, 2.0**-2), q(128, 2.0**-9)
    p[OFF_W3:OFF_B3], p[OFF_B3:] = q(64 * 128, 2.0**-2), q(64, 2.0**-11)
    ds = []
    for _ in range(8):
        n = int(rng.integers(1, 9))
        b, pe = rng.integers(0, 8, n) * 2.0**-4, rng.integers(1, 8, n) * 2.0**-4
        ds.append(np.stack([b, b + pe], 1).astype(np.float32))
    pa = np.array([0, 1, 2, 3, 4, 5, 6, 0, 2, 7, 7, 3])
    pb = np.array([1, 2, 3, 4, 5, 6, 7, 7, 5, 1, 2, 0])
    return p.astype(np.float32), ds, pa, pb, rng.uniform(0.5, 5.0, len(pa))


def exact_forward(p, ds):
    """Every forward sum is a multiple of its grid step and its magnitude sum
    is below 2^24 steps, so FP32 adds it exactly in any order."""
    P = unpack(p)
    for A in ds:
        x = features(A)
        h1 = np.maximum(x @ P["W1"].T + P["b1"], 0.0)
        if not (np.array_equal(h1, bf16(h1)) and (np.abs(x) @ np.abs(P["W1"]).T + np.abs(P["b1"])).max() < 2.0**17):
            return False
        if (h1 @ np.abs(P["W2"]).T + np.abs(P["b2"])).max() >= 2.0**15:
            return False
        pool = np.maximum(h1 @ P["W2"].T + P["b2"], 0.0).sum(axis=0)
        if pool.max() >= 2.0**15 or (np.abs(P["W3"]) @ pool + np.abs(P["b3"])).max() >= 2.0**13:
            return False
    return True


def gradient_tolerance(p, ds, pa, pb, w, gam=2.0**-16):
    """Element-wise bound on |g_gpu - g_oracle| when the forward pass is exact.

    The GPU's per-pair coefficients c_j = 2 (pred - w) / (w^2 P pred) differ
    from the FP64 ones by a few FP32 ulps and its backward sums round in
    FP32; both are covered by gam = 2^-16 (256 terms of 2^-24) times the
    magnitude of each gradient entry, i.e. the backward pass run on absolute
    values with the embedding gradient replaced by sum_j |c_j| |diff_j|.  dpool is rounded to
    BF16 before it enters dW2 and dH1; where dpool +- gam * its magnitude
    straddles a BF16 rounding boundary, the full BF16 step is added and
    carried through dW2, dH1, dW1 and db1."""
    P = unpack(p)
    W2b = bf16(P["W2"])
    emb, cache = forward(p, ds, emulate=True)
    nP = len(w)
    dsum, mag = np.zeros_like(emb), np.zeros_like(emb)
    for j in range(nP):
        diff = emb[pa[j]] - emb[pb[j]]
        pred = np.sqrt(diff @ diff)
        if pred > 0:
            g = 2.0 * (pred - w[j]) / (w[j] ** 2 * nP * pred) * diff
            dsum[pa[j]] += g
            dsum[pb[j]] = dsum[pb[j]] - g
            mag[pa[j]] += np.abs(g)
            mag[pb[j]] += np.abs(g)
    A3 = np.abs(P["W3"])
    t = dict(W1=np.zeros((128, 2)), b1=np.zeros(128), W2=np.zeros((128, 128)), b2=np.zeros(128),
             W3=np.zeros((64, 128)), b3=gam * mag.sum(axis=0))
    for d, (x, h1, z2, pool) in enumerate(cache):
        t["W3"] += gam * np.outer(mag[d], np.abs(pool))
        if not len(x):
            continue
        dpool, mpool = P["W3"].T @ dsum[d], A3.T @ mag[d]
        m2 = (z2 > 0.0).astype(np.float64)
        t["b2"] += gam * (m2 * mpool).sum(axis=0)
        rb = bf16(dpool)
        flip = np.maximum(np.abs(bf16(dpool + gam * mpool) - rb), np.abs(rb - bf16(dpool - gam * mpool)))
        e_dz2 = m2 * flip + gam * m2 * (np.abs(rb) + flip)
        t["W2"] += e_dz2.T @ np.abs(h1)
        e_dz1 = (e_dz2 @ np.abs(W2b)) * (h1 > 0.0)
        t["W1"] += e_dz1.T @ np.abs(x)
        t["b1"] += e_dz1.sum(axis=0)
    return np.concatenate([t["W1"].ravel(), t["b1"], t["W2"].ravel(), t["b2"], t["W3"].ravel(), t["b3"]])

"""Pins of the learned-form oracle (oracle/surrogate.py) against facts that
do not come from the oracle itself: finite differences, closed forms,
invariances of sum pooling, an independent bit-level BF16 rounding, and the
exact W1 (Hungarian) for the dual lower bound."""
import numpy as np
import pytest

import oracle
from oracle import surrogate as S
import pdsynth


def _bf16_bits(x32: np.ndarray) -> np.ndarray:
    """BF16 rounding of FP32 values by integer arithmetic on the bit pattern."""
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_known_values():
    one = 1.0
    assert S.bf16(one) == 1.0
    assert S.bf16(1 + 2.0**-8) == 1.0                     # tie -> even mantissa
    assert S.bf16(1 + 3 * 2.0**-8) == 1 + 2.0**-6         # tie -> even (upwards)
    assert S.bf16(1 + 2.0**-8 + 2.0**-20) == 1 + 2.0**-7  # above the tie
    assert S.bf16(-(1 + 2.0**-8 + 2.0**-20)) == -(1 + 2.0**-7)
    assert S.bf16(0.0) == 0.0
    assert S.bf16(3.0) == 3.0 and S.bf16(255.0) == 255.0 and S.bf16(257.0) == 256.0


def test_bf16_matches_bit_rounding():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(200_000) * np.exp(rng.uniform(-20, 20, 200_000))).astype(np.float32)
    assert np.array_equal(S.bf16(x.astype(np.float64)), _bf16_bits(x))
    y = S.bf16(x.astype(np.float64))
    assert np.array_equal(S.bf16(y), y)                    # idempotent


def _rand_params(seed, scale_w3=0.05):
    rng = np.random.default_rng(seed)
    p = np.zeros(S.NPARAM, np.float32)
    p[S.OFF_W1:S.OFF_B1] = rng.uniform(-1.5, 1.5, 256)
    p[S.OFF_B1:S.OFF_W2] = rng.uniform(-0.2, 0.2, 128)
    p[S.OFF_W2:S.OFF_B2] = rng.uniform(-0.2, 0.2, 128 * 128)
    p[S.OFF_B2:S.OFF_W3] = rng.uniform(-0.1, 0.1, 128)
    p[S.OFF_W3:S.OFF_B3] = rng.uniform(-scale_w3, scale_w3, 64 * 128)
    p[S.OFF_B3:] = rng.uniform(-0.1, 0.1, 64)
    return p


def _small_set(seed=1):
    return [pdsynth.exp_pd(n, seed + i) for i, n in enumerate((7, 12, 5, 9))]


def test_gradient_finite_differences():
    """Plain FP64 gradient against central differences of the loss."""
    p = _rand_params(3).astype(np.float64)
    ds = _small_set()
    pa, pb, w = [0, 1, 2, 0], [1, 2, 3, 3], [0.3, 0.5, 0.2, 0.4]
    _, g = S.loss_grad(p, ds, pa, pb, w, emulate=False)
    gmax = np.abs(g).max()
    assert gmax > 0
    rng = np.random.default_rng(7)
    idx = np.concatenate([rng.choice(np.arange(lo, hi), 6, replace=False) for lo, hi in
                          ((S.OFF_W1, S.OFF_B1), (S.OFF_B1, S.OFF_W2), (S.OFF_W2, S.OFF_B2),
                           (S.OFF_B2, S.OFF_W3), (S.OFF_W3, S.OFF_B3), (S.OFF_B3, S.NPARAM))])
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        e = np.zeros_like(p)
        e[i] = h
        fd = (S.loss_grad(p + e, ds, pa, pb, w, emulate=False)[0]
              - S.loss_grad(p - e, ds, pa, pb, w, emulate=False)[0]) / (2 * h)
        # central differences: truncation O(h^2), rounding O(u |loss| / h)
        assert abs(fd - g[i]) <= 1e-5 * abs(g[i]) + 1e-7 * gmax, (i, fd, g[i])


def _identity_params():
    """phi(x) = (b, p, 0, ...), pool = (sum b, sum p, 0...), e = pool[:64]."""
    p = np.zeros(S.NPARAM, np.float32)
    W1 = np.zeros((128, 2), np.float32)
    W1[0, 0] = 1.0
    W1[1, 1] = 1.0
    p[S.OFF_W1:S.OFF_B1] = W1.ravel()
    p[S.OFF_W2:S.OFF_B2] = np.eye(128, dtype=np.float32).ravel()
    W3 = np.zeros((64, 128), np.float32)
    W3[np.arange(64), np.arange(64)] = 1.0
    p[S.OFF_W3:S.OFF_B3] = W3.ravel()
    return p


def test_closed_form_identity_network():
    p = _identity_params()
    A = pdsynth.exp_pd(50, 3)
    e, _ = S.forward(p, [A], emulate=False)
    x = S.features(A)
    assert np.allclose(e[0, :2], x.sum(axis=0), rtol=1e-14)
    assert np.all(e[0, 2:] == 0.0)
    # emulated: points on a dyadic grid with <= 8 significant bits are exact
    B = np.array([[0.25, 0.75], [0.5, 0.625], [1.0, 3.0], [2.0, 2.0]])
    e2, _ = S.forward(p, [B], emulate=True)
    assert e2[0, 0] == 0.25 + 0.5 + 1.0 and e2[0, 1] == 0.5 + 0.125 + 2.0


def test_pooling_invariances():
    p = _rand_params(5)
    A = pdsynth.mixture_pd(300, 4)
    perm = np.random.default_rng(1).permutation(len(A))
    diag = np.array([[0.3, 0.3], [0.9, 0.9]], np.float32)
    AA = np.concatenate([A, A])
    e, cache = S.forward(p, [A, A[perm], np.concatenate([A, diag]), AA], emulate=True)
    assert np.allclose(e[1], e[0], rtol=1e-12, atol=1e-12)
    assert np.array_equal(e[2], e[0])
    P = S.unpack(p)
    assert np.allclose(cache[3][3], 2 * cache[0][3], rtol=1e-12)
    assert np.allclose(e[3] - P["b3"], 2 * (e[0] - P["b3"]), rtol=1e-10, atol=1e-12)


def test_emulation_matches_plain_on_representable_values():
    rng = np.random.default_rng(2)
    p = np.zeros(S.NPARAM, np.float32)
    p[S.OFF_W1:S.OFF_B1] = rng.integers(-4, 5, 256) / 4.0
    p[S.OFF_B1:S.OFF_W2] = rng.integers(-2, 3, 128) / 8.0
    p[S.OFF_W2:S.OFF_B2] = rng.integers(-4, 5, 128 * 128) / 16.0
    p[S.OFF_B2:S.OFF_W3] = rng.uniform(-1, 1, 128)
    p[S.OFF_W3:S.OFF_B3] = rng.uniform(-1, 1, 64 * 128)
    b = rng.integers(0, 8, 40) / 8.0
    A = np.stack([b, b + rng.integers(1, 8, 40) / 8.0], axis=1)
    e1, _ = S.forward(p, [A], emulate=True)
    e2, _ = S.forward(p, [A], emulate=False)
    assert np.array_equal(e1, e2)


def test_emulated_gradient_close_to_plain():
    """The emulated backward differs from the plain one only by BF16
    roundings (relative size 2^-8 per rounded value)."""
    p = _rand_params(9)
    ds = _small_set(11)
    pa, pb, w = [0, 1, 2], [1, 2, 3], [0.3, 0.5, 0.2]
    l1, g1 = S.loss_grad(p, ds, pa, pb, w, emulate=True)
    l2, g2 = S.loss_grad(p, ds, pa, pb, w, emulate=False)
    assert abs(l1 - l2) <= 0.05 * abs(l2)
    assert np.linalg.norm(g1 - g2) <= 0.05 * np.linalg.norm(g2)


@pytest.mark.parametrize("seed", range(12))
def test_dual_bound_below_exact(seed):
    A = pdsynth.exp_pd(15 + seed, 100 + seed)
    B = pdsynth.mixture_pd(10 + 2 * seed, 200 + seed, dtype=np.float64)
    lb = S.dual_bound(A, B)
    w = oracle.exact_w1(A, B)
    assert lb <= w * (1 + 1e-12) + 1e-15


def test_dual_bound_closed_forms():
    A = np.array([[0.2, 1.0]])
    assert S.dual_bound(A, np.zeros((0, 2))) == pytest.approx(0.4)   # = d_diag
    assert S.dual_bound(A, A) == 0.0


def test_nn_exhaustive_self_and_ties():
    db = [pdsynth.exp_pd(8, 40 + i) for i in range(5)]
    db.insert(3, db[1].copy())   # exact copy at a higher index
    out = S.nn_exhaustive(db, [db[1], db[4]], eps=0.2)
    assert out[0] == (1, 0.0)    # itself, lowest of the two copies
    assert out[1][0] == 4 and out[1][1] == 0.0


# ----------------------------------------------------------------- WCD --
@pytest.mark.parametrize("l2", [False, True])
def test_wcd_half_is_a_lower_bound(l2):
    # half the word centroid distance of the augmented diagrams stays below
    # the exact W1 (Hungarian), and the dual bound's c = 0 test function
    # (the distance to the diagonal) gives twice as much
    for seed in range(12):
        A = pdsynth.exp_pd(40, 500 + 2 * seed, mean_pers=0.1)
        B = pdsynth.exp_pd(30 + seed, 501 + 2 * seed, mean_pers=0.1)
        w = S.wcd_half(A, B, l2=l2)
        ex = oracle.exact_w1(A, B, l2=l2)
        assert w <= ex * (1 + 1e-12)
        if not l2:
            assert w <= S.dual_bound(A, B) * (1 + 1e-12)


def test_wcd_half_closed_forms():
    # a point minus its projection is (-p/2, p/2) for persistence p, so the
    # difference of the sums is (P_B - P_A)/2 * (1, -1) and half its norm is
    # |P_A - P_B| / 4 (L-infinity) or |P_A - P_B| / (2 sqrt 2) (Euclidean)
    A = np.array([[0.0, 1.0], [0.5, 0.75]])
    B = np.array([[0.25, 0.5]])
    PA, PB = 1.25, 0.25
    assert S.wcd_half(A, B) == pytest.approx(abs(PA - PB) / 4)
    assert S.wcd_half(A, B, l2=True) == pytest.approx(abs(PA - PB) / (2 * np.sqrt(2)))
    assert S.wcd_half(A, A) == 0.0
    # one point against nothing: W1 is its distance to the diagonal, p/2,
    # and the bound gives half of that
    assert S.wcd_half(A[:1], np.zeros((0, 2))) == pytest.approx(0.25)


def test_nn_pipeline_limits():
    # the pipeline keeping every candidate is the exhaustive search, and its
    # answer is never closer than the true nearest neighbour
    rng = np.random.default_rng(3)
    db = [pdsynth.exp_pd(int(rng.integers(10, 30)), 600 + i, mean_pers=0.1) for i in range(12)]
    qs = [pdsynth.exp_pd(20, 700 + i, mean_pers=0.1) for i in range(3)]
    want = S.nn_exhaustive(db, qs)
    assert S.nn_pipeline(db, qs, keep=len(db), c2=len(db)) == want
    for keep, c2 in ((4, 1), (6, 2)):
        got = S.nn_pipeline(db, qs, keep=keep, c2=c2)
        assert all(g[1] >= w[1] for g, w in zip(got, want))

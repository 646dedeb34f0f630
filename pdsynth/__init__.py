"""Seeded synthetic persistence diagrams.

This module only draws random point sets; it holds none of the method's
arithmetic, so both the CPU oracle and the GPU path can share it as their
common input source.  A diagram is an (n, 2) array of (birth, death) rows,
death >= birth.  Diagram A of pair k uses seed 2k and diagram B seed 2k+1.

Workload families (the paper's own datasets are not available, so these
stand in for them with the shapes the paper describes: most points close to
the diagonal, a heavy tail of persistent features, many exact repeats):

* ``exp_pd``      birth ~ U[0,1), persistence ~ Exponential(mean 0.05), FP64.
* ``mixture_pd``  80% persistence ~ LogNormal(-4, 1), 20% ~ U[0.1, 1],
                  birth ~ U[0,1), cast to FP32 (rows whose FP32 death is not
                  above the FP32 birth are redrawn).
* ``pareto_pd``   birth ~ U[0,1), persistence ~ min(Lomax(1.5), 10), plus a
                  fraction of exact copies of random rows, shuffled, FP32.
* ``batch_sizes`` log-uniform point counts for batched workloads.
* ``family_pd``   per-diagram latent parameters (near-diagonal scale, far
                  fraction, far cluster centre/spread) so that nearest
                  neighbours in a database are meaningful.
* ``integer_pd``  small integer coordinates, for exact-arithmetic pins.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "exp_pd",
    "mixture_pd",
    "pareto_pd",
    "batch_sizes",
    "family_pd",
    "family_params",
    "integer_pd",
    "pair_seeds",
]


def pair_seeds(k: int) -> tuple[int, int]:
    """Seeds of diagram A and diagram B of pair k."""
    return 2 * k, 2 * k + 1


def exp_pd(n: int, seed: int, mean_pers: float = 0.05, dtype=np.float64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    b = rng.random(n)
    p = rng.exponential(mean_pers, n)
    d = b + p
    out = np.stack([b, d], axis=1)
    if dtype == np.float32:
        out = _to_f32_redraw(out, rng, lambda m: _exp_rows(rng, m, mean_pers))
    return out


def _exp_rows(rng, m, mean_pers):
    b = rng.random(m)
    return np.stack([b, b + rng.exponential(mean_pers, m)], axis=1)


def _mixture_rows(rng, m, near_frac=0.8, mu=-4.0, sigma=1.0, far_lo=0.1, far_hi=1.0):
    b = rng.random(m)
    near = rng.random(m) < near_frac
    p = np.where(near, rng.lognormal(mu, sigma, m), rng.uniform(far_lo, far_hi, m))
    return np.stack([b, b + p], axis=1)


def mixture_pd(n: int, seed: int, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    rows = _mixture_rows(rng, n)
    if dtype == np.float32:
        return _to_f32_redraw(rows, rng, lambda m: _mixture_rows(rng, m))
    return rows


def _to_f32_redraw(rows, rng, draw):
    out = rows.astype(np.float32)
    bad = out[:, 1] <= out[:, 0]
    while bad.any():
        fresh = draw(int(bad.sum())).astype(np.float32)
        out[bad] = fresh
        bad = out[:, 1] <= out[:, 0]
    return out


def pareto_pd(n: int, seed: int, dup_frac: float = 0.3, alpha: float = 1.5,
              cap: float = 10.0, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    n_dup = int(round(n * dup_frac))
    n_base = n - n_dup

    def draw(m):
        b = rng.random(m)
        return np.stack([b, b + np.minimum(rng.pareto(alpha, m), cap)], axis=1)

    base = draw(n_base)
    if dtype == np.float32:
        base = _to_f32_redraw(base, rng, draw)
    base = base.astype(dtype)
    if n_dup > 0 and n_base > 0:
        dup = base[rng.integers(0, n_base, n_dup)]
        allrows = np.concatenate([base, dup], axis=0)
    else:
        allrows = base
    return allrows[rng.permutation(allrows.shape[0])]


def batch_sizes(k: int, seed: int, lo: int = 100, hi: int = 50_000) -> np.ndarray:
    """k point counts drawn log-uniformly in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), k))).astype(np.int64)


def family_params(seed: int) -> dict:
    rng = np.random.default_rng(seed)
    return {
        "scale": float(np.exp(rng.uniform(np.log(0.01), np.log(0.1)))),
        "far_frac": float(rng.uniform(0.05, 0.4)),
        "far_centre": rng.random(2).tolist(),
        "far_spread": float(np.exp(rng.uniform(np.log(0.02), np.log(0.2)))),
    }


def family_pd(n: int, seed: int, params: dict | None = None, dtype=np.float32) -> np.ndarray:
    """Diagram from a latent family; ``params`` defaults to family_params(seed)."""
    if params is None:
        params = family_params(seed)
    rng = np.random.default_rng(seed + 7_919)

    def draw(m):
        far = rng.random(m) < params["far_frac"]
        b_near = rng.random(m)
        p_near = rng.lognormal(np.log(params["scale"]), 1.0, m)
        cb, cp = params["far_centre"]
        b_far = cb + params["far_spread"] * rng.standard_normal(m)
        p_far = np.abs(0.2 + cp + params["far_spread"] * rng.standard_normal(m))
        b = np.where(far, b_far, b_near)
        p = np.where(far, p_far, p_near)
        return np.stack([b, b + p], axis=1)

    rows = draw(n)
    if dtype == np.float32:
        return _to_f32_redraw(rows, rng, draw)
    return rows


def integer_pd(n: int, seed: int, hi: int = 20) -> np.ndarray:
    """Points with small integer coordinates, death > birth (FP64)."""
    rng = np.random.default_rng(seed)
    b = rng.integers(0, hi, n)
    d = b + rng.integers(1, hi, n)
    return np.stack([b, d], axis=1).astype(np.float64)

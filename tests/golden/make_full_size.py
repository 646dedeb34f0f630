"""Writes c2_full.json: the CPU oracle's results on the 200k + 200k-point
mixture pair (diagram A seed 0, diagram B seed 1, FP32; 80% persistence
LogNormal(-4, 1), 20% U[0.1, 1]) at eps 0.2, 0.1 and 0.05, for the
full-size GPU parity test, without and with diagonal-dominance pruning.  It
calls only oracle/ (count-only runs: the WSPD
pair set enters through the oracle's order-independent pair checksum), so
the stored values never come from the GPU library.  Per-location and
per-cell arrays are stored as SHA-256 digests of their little-endian bytes
(FP64 for coordinates and RWMD costs, int64 for counts and grid
coordinates).

    python tests/golden/make_full_size.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import pdsynth  # noqa: E402

N = 200_000
EPS = (0.2, 0.1, 0.05)


def digest(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).astype(dtype.newbyteorder("<")).tobytes()).hexdigest()


def main():
    A, B = pdsynth.mixture_pd(N, 0), pdsynth.mixture_pd(N, 1)
    out = {"workload": f"mixture_pd({N}, 0) vs mixture_pd({N}, 1), FP32", "eps": {}}
    for eps in EPS:
        t0 = time.time()
        r = oracle.run(A, B, eps=eps, flags=oracle.ORC_COUNT_ONLY)
        assert r.status == 0
        f64, i64 = np.dtype(np.float64), np.dtype(np.int64)
        out["eps"][str(eps)] = {
            "nA": r.nA, "nB": r.nB, "n": r.n, "s": r.s, "e": r.e, "m0": r.m0,
            "L": r.L.hex(), "LA": r.LA.hex(), "LB": r.LB.hex(), "SA": r.SA, "SB": r.SB, "FA": r.FA, "FB": r.FB,
            "n_locations": int(r.locs["b"].shape[0]), "n_cells": int(r.cells["i"].shape[0]),
            "n_pairs": r.n_pairs, "checksum": [r.checksum[0], r.checksum[1]],
            "sha256": {
                "loc_b": digest(r.locs["b"], f64), "loc_d": digest(r.locs["d"], f64),
                "loc_w": digest(r.locs["w"], i64), "loc_t": digest(r.locs["t"], f64),
                "cell_i": digest(r.cells["i"], i64), "cell_j": digest(r.cells["j"], i64),
                "cell_ca": digest(r.cells["cA"], i64), "cell_cb": digest(r.cells["cB"], i64),
            },
            "oracle_seconds": round(time.time() - t0, 1),
        }
        # the same pair with diagonal-dominance pruning (O7'): pairs kept
        t0 = time.time()
        rp = oracle.run(A, B, eps=eps, flags=oracle.ORC_COUNT_ONLY | oracle.ORC_PRUNE, fetch=False)
        assert rp.status == 0
        out["eps"][str(eps)]["pruned"] = {"n_pairs": rp.n_pairs, "checksum": [rp.checksum[0], rp.checksum[1]],
                                          "oracle_seconds": round(time.time() - t0, 1)}
        print(eps, out["eps"][str(eps)]["n_pairs"], out["eps"][str(eps)]["oracle_seconds"], flush=True)
    with open(os.path.join(HERE, "c2_full.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()

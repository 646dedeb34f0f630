"""Writes stream_checksums.json: the CPU oracle's WSPD pair counts and
order-independent pair checksums (count-only runs) for the streamed-emission
GPU tests:
  * a sample of 256 pairs of the batched workload (4096 pairs, point counts
    from batch_sizes(8192, 3), A_i = exp_pd(n, 10 + 2i), B_i =
    exp_pd(n, 11 + 2i), FP32; every 16th pair) at eps 0.1;
  * a 200k + 200k subsample of the stress workload (pareto_pd(200000, 0)
    vs pareto_pd(200000, 1), FP32: persistence min(Lomax(1.5), 10), 30%
    exact duplicates) at eps 0.01 (s = 503).
Calls only oracle/ and pdsynth, so no stored value comes from the GPU
library.

    python tests/golden/make_stream_checksums.py
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import pdsynth  # noqa: E402

BATCH_PAIRS, STEP = 4096, 16
STRESS_N, STRESS_EPS = 200_000, 0.01


def batch_pair(i):
    s = pdsynth.batch_sizes(2 * BATCH_PAIRS, 3)
    return (pdsynth.exp_pd(int(s[2 * i]), 10 + 2 * i, dtype=np.float32),
            pdsynth.exp_pd(int(s[2 * i + 1]), 11 + 2 * i, dtype=np.float32))


def _count(args):
    kind, i = args
    if kind == "batch":
        A, B = batch_pair(i)
        eps = 0.1
    else:
        A, B = pdsynth.pareto_pd(STRESS_N, 0), pdsynth.pareto_pd(STRESS_N, 1)
        eps = STRESS_EPS
    r = oracle.run(A, B, eps=eps, flags=oracle.ORC_COUNT_ONLY, fetch=False)
    assert r.status == 0
    return {"n_pairs": r.n_pairs, "checksum": [r.checksum[0], r.checksum[1]], "s": r.s}


def main():
    t0 = time.time()
    idx = list(range(0, BATCH_PAIRS, STEP))
    jobs = [("stress", 0)] + [("batch", i) for i in idx]
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(_count, jobs, chunksize=1)
    out = {"batch": {"workload": f"every {STEP}th pair of the 4096-pair batched workload, eps 0.1",
                     "index": idx, "pairs": res[1:]},
           "stress": dict(res[0], workload=f"pareto_pd({STRESS_N}, 0) vs pareto_pd({STRESS_N}, 1), FP32, "
                                           f"eps {STRESS_EPS}"),
           "seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "stream_checksums.json"), "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print(res[0], out["seconds"])


if __name__ == "__main__":
    main()

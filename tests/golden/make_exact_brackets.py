"""Writes exact_w1.json: exact W1 (Hungarian matching on the diagonal-augmented
bipartite graph, oracle.exact_w1) of
  * the 400 + 400-point pairs k = 0..99 (diagram A exp_pd(400, 2k), B
    exp_pd(400, 2k + 1), FP64), for the (1 + eps) bracket at eps 0.1;
  * every pair of the batched workload (4096 pairs, point counts from
    batch_sizes(8192, 3), A_i = exp_pd(n, 10 + 2i), B_i = exp_pd(n, 11 + 2i),
    FP32) with n_A + n_B <= 3000.
It calls only oracle/ and pdsynth, so the stored values never come from the
GPU library.  Values are stored as float.hex strings.

    python tests/golden/make_exact_brackets.py
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

C1_PAIRS = 100
C3_PAIRS = 4096
C3_MAX_POINTS = 3000


def c1_pair(k):
    return pdsynth.exp_pd(400, 2 * k), pdsynth.exp_pd(400, 2 * k + 1)


def c3_sizes():
    s = pdsynth.batch_sizes(2 * C3_PAIRS, 3)
    return s[0::2], s[1::2]


def c3_pair(i, na, nb):
    return (pdsynth.exp_pd(int(na), 10 + 2 * i, dtype=np.float32),
            pdsynth.exp_pd(int(nb), 11 + 2 * i, dtype=np.float32))


def _c1(k):
    return oracle.exact_w1(*c1_pair(k))


def _c3(args):
    i, na, nb = args
    return oracle.exact_w1(*c3_pair(i, na, nb))


def main():
    t0 = time.time()
    a, b = c3_sizes()
    idx = [int(i) for i in np.flatnonzero(a + b <= C3_MAX_POINTS)]
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        c1 = pool.map(_c1, range(C1_PAIRS))
        c3 = pool.map(_c3, [(i, int(a[i]), int(b[i])) for i in idx], chunksize=4)
    out = {
        "c1": {"workload": "exp_pd(400, 2k) vs exp_pd(400, 2k + 1), FP64, k = 0..99", "w1": [float(x).hex() for x in c1]},
        "c3_small": {"workload": f"batched workload pairs with n_A + n_B <= {C3_MAX_POINTS}", "index": idx,
                     "w1": [float(x).hex() for x in c3]},
        "seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, "exact_w1.json"), "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print(len(c1), len(c3), out["seconds"])


if __name__ == "__main__":
    main()

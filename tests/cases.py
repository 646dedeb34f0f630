"""Seeded inputs shared by the GPU parity tests and the script that stores
the oracle's optimal flows for them (tests/golden/make_oracle_flows.py).
Generators only: no arithmetic of the method."""
import numpy as np

import pdsynth

# (name, inputs, eps) of the stage-parity cases
STAGE_CASES = [
    ("exp400_eps0.1", lambda: (pdsynth.exp_pd(400, 0), pdsynth.exp_pd(400, 1)), 0.1),
    ("exp250_eps0.2", lambda: (pdsynth.exp_pd(250, 2), pdsynth.exp_pd(233, 3)), 0.2),
    ("mix_f32_3000_eps0.2", lambda: (pdsynth.mixture_pd(3000, 4), pdsynth.mixture_pd(2777, 5)), 0.2),
    ("pareto_dup_2000_eps0.5", lambda: (pdsynth.pareto_pd(2000, 6), pdsynth.pareto_pd(1500, 7)), 0.5),
    ("int_overlap_eps0.3", lambda: (pdsynth.integer_pd(300, 8, hi=12), pdsynth.integer_pd(280, 9, hi=12)), 0.3),
    ("exp_f32_odd_eps0.05",
     lambda: (pdsynth.exp_pd(129, 10, dtype=np.float32), pdsynth.exp_pd(65, 11, dtype=np.float32)), 0.05),
]

# sparsity-parameter cases: one pair, eps 0.1, s = 1, 2, 3, 6, 12
SMALL_S = (1, 2, 3, 6, 12)


def small_s_pair():
    return pdsynth.exp_pd(500, 12), pdsynth.exp_pd(480, 13)


def batch_pairs():
    """Twelve uneven FP32 pairs (20 to 3000 points), one empty diagram and
    one pair of identical diagrams, eps 0.2."""
    sizes = pdsynth.batch_sizes(24, 99, lo=20, hi=3000)
    As = [pdsynth.exp_pd(int(sizes[i]), 1000 + 2 * i, dtype=np.float32) for i in range(12)]
    Bs = [pdsynth.exp_pd(int(sizes[12 + i]), 1001 + 2 * i, dtype=np.float32) for i in range(12)]
    As[3] = np.zeros((0, 2), np.float32)
    Bs[5] = As[5].copy()
    return As, Bs

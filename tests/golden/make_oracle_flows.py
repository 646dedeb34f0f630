"""Writes oracle_flows.json: the CPU oracle's optimal flow cost F*, W1 and
W1_paper for the GPU parity cases that run an exact flow (tests/cases.py;
the stage cases also with the Euclidean metric, keys ending in _l2),
so that the GPU machine does not spend minutes in the oracle's successive-
shortest-path solver.  Calls only oracle/ and pdsynth (through
tests/cases.py); values stored as integers and float.hex strings.

    python tests/golden/make_oracle_flows.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import cases  # noqa: E402
import oracle  # noqa: E402


def entry(A, B, eps, s_override=0, flags=0):
    r = oracle.run(A, B, eps=eps, s_override=s_override, flags=flags, fetch=False)
    assert r.status == 0
    return {"flow": r.flow if r.n else 0, "W1": r.W1.hex(), "W1_paper": r.W1_paper.hex(), "n_pairs": r.n_pairs}


def main():
    t0 = time.time()
    out = {}
    for name, make, eps in cases.STAGE_CASES:
        out[name] = entry(*make(), eps)
        out[name + "_l2"] = entry(*make(), eps, flags=oracle.ORC_L2)
        print(name, out[name]["flow"], out[name + "_l2"]["flow"], flush=True)
    A, B = cases.small_s_pair()
    for s in cases.SMALL_S:
        out[f"small_s{s}"] = entry(A, B, 0.1, s)
    As, Bs = cases.batch_pairs()
    for i, (A, B) in enumerate(zip(As, Bs)):
        out[f"batch{i}"] = entry(A, B, 0.2)
    out["seconds"] = round(time.time() - t0, 1)
    with open(os.path.join(HERE, "oracle_flows.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("done", out["seconds"])


if __name__ == "__main__":
    main()

"""Autotuner of the WSPD traversal tunables (w1_tuning).

The traversal's work-list granularity (stack_depth, work_cap), its chunking
(chunk_items) and its occupancy (blocks_per_cu) change its speed, never its
output.  This tuner measures candidates with the library's own HIP-event
timers of the WSPD kernels on a given workload, searches coordinate-wise from
the current setting, and keeps the fastest.  The choice is cached in a JSON
file keyed by device architecture, compute-unit count, workload size class and
mode.

    python -m paper_2110_14734_amd.tune [--cache FILE] [--workload c2|c3|c3full]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

CHOICES = {
    "stack_depth": [12, 16, 20, 24],
    "work_cap": [256, 512, 1024, 2048, 4096],
    "chunk_items": [128, 256, 512, 1024, 2048],
    "blocks_per_cu": [2, 3, 4, 5, 6, 8],
}
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")


def device_key() -> str:
    import torch

    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "gfx").split(":")[0]
    return f"{arch}/{p.multi_processor_count}cu"


def workload_key(As, Bs, eps: float, count_only: bool) -> str:
    pts = sum(len(a) + len(b) for a, b in zip(As, Bs))
    per_pair = pts / max(len(As), 1)
    return f"pts2^{round(math.log2(max(pts, 1)))}/pair2^{round(math.log2(max(per_pair, 1)))}/eps{eps}/" + \
        ("count" if count_only else "emit")


def measure(ctx, As, Bs, eps, flags, reps) -> float:
    """Median over reps of the WSPD device time (work list + count + emit), ms."""
    import paper_2110_14734_amd as w1

    ts = []
    for _ in range(reps):
        if len(As) == 1:
            ctx.approx(As[0], Bs[0], eps=eps, flags=flags)
            kt = ctx.kernel_times()
            ts.append(kt["worklist_ms"] + kt["count_ms"] + kt["emit_ms"])
        else:  # batches may run in several launch groups: time the whole call
            import torch

            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.approx_batch(As, Bs, eps=eps, flags=flags)
            torch.cuda.synchronize()
            ts.append(1e3 * (time.perf_counter() - t0))
    del w1
    return sorted(ts)[len(ts) // 2]


def tune(ctx, As, Bs, eps=0.1, flags=0, reps=3, passes=2, log=print) -> dict:
    """Coordinate search over CHOICES from the context's current tuning.
    Leaves the best setting applied to ctx and returns it with its time."""
    best = ctx.tuning
    best_t = measure(ctx, As, Bs, eps, flags, reps)
    log(f"[tune] start {best} {best_t:.2f} ms")
    for _ in range(passes):
        improved = False
        for name, values in CHOICES.items():
            for v in values:
                if v == best[name]:
                    continue
                cand = dict(best, **{name: v})
                ctx.tuning = cand
                t = measure(ctx, As, Bs, eps, flags, reps)
                log(f"[tune] {name}={v}: {t:.2f} ms")
                if t < 0.97 * best_t:
                    best, best_t, improved = cand, t, True
            ctx.tuning = best
        if not improved:
            break
    ctx.tuning = best
    return dict(best, ms=best_t)


def save(cache: str, key: str, result: dict) -> None:
    data = {}
    if os.path.exists(cache):
        with open(cache) as f:
            data = json.load(f)
    data[key] = result
    tmp = cache + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, cache)


def lookup(data: dict, dev: str, key: str) -> dict | None:
    """The cached entry for this device and workload class; failing that,
    the entry of the same device, points per pair, eps and mode whose total
    size is closest (the tunables follow the pair sizes more than their
    number)."""
    if dev + "/" + key in data:
        return data[dev + "/" + key]
    tot, rest = key.split("/", 1)
    best, dist = None, None
    for k, v in data.items():
        if not k.startswith(dev + "/"):
            continue
        kt, kr = k[len(dev) + 1:].split("/", 1)
        if kr != rest:
            continue
        d = abs(int(kt[len("pts2^"):]) - int(tot[len("pts2^"):]))
        if dist is None or d < dist:
            best, dist = v, d
    return best


def apply_cached(ctx, As, Bs, eps=0.1, count_only=False, cache: str = DEFAULT_CACHE) -> dict | None:
    """Apply the cached tuning of this device and workload class, if any."""
    if not os.path.exists(cache):
        return None
    with open(cache) as f:
        data = json.load(f)
    hit = lookup(data, device_key(), workload_key(As, Bs, eps, count_only))
    if hit:
        ctx.tuning = {k: v for k, v in hit.items() if k in ctx.tuning}
    return hit


def _workload(name: str):
    import numpy as np

    import pdsynth

    if name == "c2":
        return [pdsynth.mixture_pd(200_000, 0)], [pdsynth.mixture_pd(200_000, 1)], 0
    sizes = pdsynth.batch_sizes(2 * (4096 if name == "c3full" else 512), 3)
    As = [pdsynth.exp_pd(int(n), 10 + 2 * i, dtype=np.float32) for i, n in enumerate(sizes[0::2])]
    Bs = [pdsynth.exp_pd(int(n), 11 + 2 * i, dtype=np.float32) for i, n in enumerate(sizes[1::2])]
    return As, Bs, 2  # COUNT_ONLY


def main():
    import torch

    import paper_2110_14734_amd as w1

    ap = argparse.ArgumentParser()
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c3full"])
    ap.add_argument("--eps", type=float, default=0.1)
    a = ap.parse_args()
    As, Bs, flags = _workload(a.workload)
    As = [torch.from_numpy(x).cuda() for x in As]
    Bs = [torch.from_numpy(x).cuda() for x in Bs]
    ctx = w1.Context(0)
    ctx.approx_batch(As, Bs, eps=a.eps, flags=flags | w1.NO_FLOW)  # warm-up
    res = tune(ctx, As, Bs, a.eps, flags | w1.NO_FLOW, log=lambda m: print(m, flush=True))
    key = device_key() + "/" + workload_key(As, Bs, a.eps, bool(flags & w1.COUNT_ONLY))
    save(a.cache, key, res)
    print(json.dumps({key: res}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

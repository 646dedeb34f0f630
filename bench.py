"""Benchmark of the approximate-W1 sparsification hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--eps 0.1] [--n 200000]

Workload (a "step"): one pass of the whole GPU hot path -- 0-condensation,
RWMD, grid condensation, radix tree, WSPD pairs and the sparse transshipment
network -- over one pair of synthetic persistence diagrams of 200k points each
(80% near the diagonal with persistence LogNormal(-4, 1), 20% with persistence
U[0.1, 1], birth U[0, 1), FP32) at eps = 0.1.  Inputs are resident in HBM
before the timed region.  The host min-cost flow is not part of the step (at
this size the network has ~3.6e9 arcs); its cost is reported separately on
the 400-point workload, end to end.

Prints one JSON line.  `value` = sparsified points per second (whole job).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PD pairs/sec (approx W1 at eps) + sparsify pts/s & HBM GB/s frac; 1-NN q/s"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes of the WSPD and network kernels, per WSPD pair (both
# arcs of a pair) and per cell, for pair records of w words (w = 2: u32 u,
# u32 v; w = 3: also i32 cost):
#   emit          writes the 4w-byte pair record and counts both arcs per
#                 tail bucket in LDS;
#   bucket_scatter reads the record, writes two 4-byte bucket entries;
#   row_hist      reads the two entries;
#   row_scatter   reads the two entries, writes two 4-byte row heads;
#   row_sort      reads the two heads, writes two (u32 head, i32 cost) arcs
#                 of the final rows and an int64 row pointer per cell.
# The final network alone is 16 B per pair and 8 B per cell.
def kernel_bytes(w):
    return {"emit_ms": (4 * w, 0), "bucket_scatter_ms": (4 * w + 8, 0),
            "row_hist_ms": (8, 0), "row_scatter_ms": (16, 0), "row_sort_ms": (24, 8)}


KERNEL_BYTES = kernel_bytes(2)
NETWORK_BYTES = (16, 8)
KERNEL_NAMES = {"emit_ms": "k_wspd<emit> (WSPD pair records)",
                "bucket_scatter_ms": "k_bucket_scatter", "row_hist_ms": "k_row_hist",
                "row_scatter_ms": "k_row_scatter", "row_sort_ms": "k_row_sort (sorted rows, costs)"}

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE and WRITE_SIZE
# counter runs on the benchmark workload (each scaled by a copy-kernel
# calibration), valid only for the kernel source they were measured on:
# {kernel key: (source file, sha256 prefix of that file, bytes per launch)}.
# (profiles/a4_a5_kernels_c2_200k_eps0.1_hbm_counters.md)
MEASURED_TRAFFIC = {
    "emit_ms": ("paper_2110_14734_amd/csrc/wspd.hip", "29711b414e76cfa6", 23_838_175_396),
    "bucket_scatter_ms": ("paper_2110_14734_amd/csrc/csr.hip", "fa11260a58425148", 30_224_031_670),
    "row_hist_ms": ("paper_2110_14734_amd/csrc/csr.hip", "fa11260a58425148", 14_810_458_574),
    "row_scatter_ms": ("paper_2110_14734_amd/csrc/csr.hip", "fa11260a58425148", 31_811_291_743),
    "row_sort_ms": ("paper_2110_14734_amd/csrc/csr.hip", "fa11260a58425148", 47_948_840_548),
}


def measured_traffic(key, n_points, eps):
    import hashlib

    if key not in MEASURED_TRAFFIC or n_points != 400_000 or eps != 0.1:
        return None
    path, prefix, nbytes = MEASURED_TRAFFIC[key]
    h = hashlib.sha256(open(os.path.join(ROOT, path), "rb").read()).hexdigest()
    return nbytes if h.startswith(prefix) else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--eps", type=float, default=0.1)
    ap.add_argument("--n", type=int, default=200_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c1", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one device-to-device copy of this many MiB (HBM counter calibration)")
    ap.add_argument("--no-nn", action="store_true", help="skip the learned form (surrogate + 1-NN)")
    ap.add_argument("--no-nn-search", action="store_true",
                    help="learned form: only the embedding workload (no labels, training or 1-NN search)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched form")
    ap.add_argument("--no-stress", action="store_true",
                    help="skip the 2M+2M Pareto stress pair (30%% duplicates): WSPD count at --stress-eps and "
                         "the emission of one arena fill of pair records")
    ap.add_argument("--stress-eps", type=float, default=0.01)
    ap.add_argument("--batch-pairs", type=int, default=4096)
    ap.add_argument("--loop-sample", type=int, default=256,
                    help="pairs of the batch also run one call each (the per-pair loop)")
    ap.add_argument("--nn-db", type=int, default=2000, help="1-NN database size")
    ap.add_argument("--nn-queries", type=int, default=64)
    ap.add_argument("--nn-c4", type=int, default=0,
                    help="also run 1-NN search at the configured database (10k diagrams of 1k-20k points) with "
                         "this many queries (off by default: a query in RWMD order can take many minutes)")
    ap.add_argument("--nn-c4-labels", type=int, default=400, help="method labels for that search's surrogate")
    ap.add_argument("--nn-c4-extra", type=int, default=0,
                    help="further queries of that search run in the surrogate-seeded mode only")
    ap.add_argument("--embed-db", type=int, default=10_000,
                    help="diagrams in the embedding (MFMA) workload, sizes log-uniform in [1k, 20k]")
    return ap.parse_args()


MFMA_BF16_PEAK_TFLOPS = 2500.0
EMBED_FLOP_PER_POINT = 2 * (2 * 128 + 128 * 128)  # multiply-adds of phi's two layers, x2


def family_db(m, n_fam, seed, lo, hi):
    import numpy as np
    import pdsynth

    rng = np.random.default_rng(seed)
    fams = [pdsynth.family_params(50_000 + seed * 1000 + f) for f in range(n_fam)]
    sizes = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), m))).astype(int)
    fid = rng.integers(0, n_fam, m)
    db = [pdsynth.family_pd(int(sizes[i]), seed * 1_000_000 + i, fams[fid[i]]) for i in range(m)]
    return db, fams, rng


def run_batch(ctx, args):
    """Batched form: 4096 pairs with point counts log-uniform in [100, 50k]
    per diagram (birth U[0,1), persistence Exponential(mean 0.05), FP32),
    eps = 0.1, sparsified in launch groups of the per-launch point budget,
    WSPD pairs counted (the pair lists of the whole batch, ~1e11 arcs, are
    not materialised).  The per-pair loop runs the same pairs one call each
    on a sample of the batch; the batch runs that sample too, so both rates
    are on identical work."""
    import numpy as np
    import torch

    import paper_2110_14734_amd as w1
    import pdsynth
    from paper_2110_14734_amd import tune

    K = args.batch_pairs
    sizes = pdsynth.batch_sizes(2 * K, 3)
    t0 = time.perf_counter()
    As = [pdsynth.exp_pd(int(n), 10 + 2 * i, dtype=np.float32) for i, n in enumerate(sizes[0::2])]
    Bs = [pdsynth.exp_pd(int(n), 11 + 2 * i, dtype=np.float32) for i, n in enumerate(sizes[1::2])]
    gen_s = time.perf_counter() - t0
    dA = [torch.from_numpy(x).cuda() for x in As]
    dB = [torch.from_numpy(x).cuda() for x in Bs]
    npts = int(sizes.sum())
    flags = w1.COUNT_ONLY
    tuned = tune.apply_cached(ctx, dA, dB, args.eps, count_only=True)
    ctx.approx_batch(dA, dB, eps=args.eps, flags=flags)  # warm-up: buffers sized for the whole batch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ctx.approx_batch(dA, dB, eps=args.eps, flags=flags)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    wspd = sum(r.n_pairs for r in res)
    rng = np.random.default_rng(1)
    sample = np.sort(rng.choice(K, min(args.loop_sample, K), replace=False))
    sA, sB = [dA[i] for i in sample], [dB[i] for i in sample]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs_batch = ctx.approx_batch(sA, sB, eps=args.eps, flags=flags)
    torch.cuda.synchronize()
    t_sb = time.perf_counter() - t0
    t0 = time.perf_counter()
    rs_loop = [ctx.approx(a, b, eps=args.eps, flags=flags) for a, b in zip(sA, sB)]
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    same = all(x.n_pairs == y.n_pairs and x.n_cells == y.n_cells for x, y in zip(rs_batch, rs_loop))
    same = same and all(res[i].n_pairs == rs_loop[j].n_pairs for j, i in enumerate(sample))
    # every pair record of the batch written once, streamed through a
    # recycled arena, with per-pair record checksums
    t_cur = ctx.tuning
    ctx.tuning = dict(t_cur, stream_arena_pairs=1 << 30, stream_max_rounds=0)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rst = ctx.approx_batch(dA, dB, eps=args.eps, flags=flags)
        torch.cuda.synchronize()
        t_stream = time.perf_counter() - t0
    finally:
        ctx.tuning = t_cur
    streamed = sum(r.n_pairs_streamed for r in rst)
    stream = {"what": "the same batch with every WSPD pair record emitted through a 2^30-record arena that each "
                      "run of chunks overwrites, with per-pair record checksums",
              "seconds": t_stream, "pd_pairs_per_s": K / t_stream, "pairs_written": streamed,
              "all_written": bool(streamed == wspd and all(r.n_pairs_streamed == r.n_pairs for r in rst)),
              "record_GBs": 12 * streamed / t_stream / 1e9}
    # end to end (network and exact flow, W1 certified) on every pair of the
    # batch with n_A + n_B <= 3000, in one batch call: the host flows run in
    # parallel threads
    small = [i for i in range(K) if sizes[2 * i] + sizes[2 * i + 1] <= 3000]
    e2e = {}
    if small:
        sa, sb = [dA[i] for i in small], [dB[i] for i in small]
        ctx.approx_batch(sa[:64], sb[:64], eps=args.eps)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        re2e = ctx.approx_batch(sa, sb, eps=args.eps)
        t_e2e = time.perf_counter() - t0
        e2e = {"what": "W1 end to end (GPU network, host flow from the diagonal start) for every pair with "
                       "n_A + n_B <= 3000, one batch call",
               "pairs": len(small), "seconds": t_e2e, "pd_pairs_per_s": len(small) / t_e2e,
               "all_solved": bool(all(r.status == 0 and r.flow_solved == 1 for r in re2e)),
               "flow_ms_last_group": float(re2e[-1].t_ms["flow"])}
    return {
        "workload": f"{K} pairs, points per diagram log-uniform in [100, 50k] (birth U[0,1), persistence "
                    f"Exponential(mean 0.05), FP32), eps={args.eps}, a0-a4 with WSPD pairs counted",
        "end_to_end_small": e2e,
        "points": npts, "wspd_pairs": wspd,
        "batch_s": t_batch, "pd_pairs_per_s": K / t_batch, "points_per_s": npts / t_batch,
        "wspd_pairs_per_s": wspd / t_batch,
        "sample_pairs": int(len(sample)),
        "sample_batch_pd_pairs_per_s": len(sample) / t_sb,
        "sample_loop_pd_pairs_per_s": len(sample) / t_loop,
        "batch_over_loop": t_loop / t_sb,
        "identical_counts": bool(same),
        "tuning": ctx.tuning, "tuning_from_cache": bool(tuned), "gen_s": gen_s,
        "streamed": stream,
    }


def run_stress(ctx, args):
    """Stress pair: 2M points per diagram, birth U[0,1), persistence
    min(Lomax(1.5), 10), 30% exact copies of random rows, FP32.  The WSPD is
    counted, not stored (~1e12 pairs at eps 0.01), with a large-item tuning
    (work-list items up to 65,536 cell pairs, 32-entry traversal stacks)."""
    import torch

    import paper_2110_14734_amd as w1
    import pdsynth

    A, B = pdsynth.pareto_pd(2_000_000, 0), pdsynth.pareto_pd(2_000_000, 1)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    t0_tuning = ctx.tuning
    arena = 1 << 33  # pair records per arena fill (103 GB)
    ctx.tuning = dict(t0_tuning, stack_depth=32, work_cap=65536, chunk_items=64, blocks_per_cu=2,
                      stream_arena_pairs=arena, stream_max_rounds=1)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.approx(tA, tB, eps=args.stress_eps, flags=w1.COUNT_ONLY)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kt = ctx.kernel_times()
    except w1.W1Error as e:
        return {"error": str(e), "eps": args.stress_eps}
    finally:
        ctx.tuning = t0_tuning
    em_ms = kt["stream_emit_ms"]
    em_bytes = 12 * r.n_pairs_streamed
    return {"workload": f"2M+2M Pareto(1.5, cap 10) diagrams with 30% exact duplicates, FP32, eps={args.stress_eps}, "
                        "a0-a4 with every WSPD pair counted, then the first arena fill of pair records emitted",
            "s": r.s, "grid_exp": r.grid_exp, "n_points_after_cancellation": r.n_points, "cells": r.n_cells,
            "wspd_pairs": r.n_pairs, "seconds": dt, "wspd_pairs_per_s": r.n_pairs / dt,
            "stage_ms": {k: round(r.t_ms[k], 3) for k in w1.T_NAMES[:5]},
            "worklist_ms": kt["worklist_ms"], "count_ms": kt["count_ms"],
            "emission": {"what": "k_wspd<emit> over the longest prefix of work-list chunks whose pair records "
                                 "fit one arena fill (12 B per record)",
                         "pairs": r.n_pairs_streamed, "arena_pairs": arena, "ms": round(em_ms, 3),
                         "achieved_GBs": round(em_bytes / (em_ms * 1e-3) / 1e9, 1) if em_ms > 0 else None,
                         "frac": round(em_bytes / (em_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if em_ms > 0 else None}}


def run_nn(ctx, args):
    """Learned form: DeepSets surrogate trained on the GPU on W1 labels that
    the method computes, then 1-NN search with and without it."""
    import numpy as np
    import torch

    import paper_2110_14734_amd as w1
    import pdsynth

    out = {}
    # (1) embedding throughput on a database of the 1-NN configuration's size
    t0 = time.perf_counter()
    big, _, _ = family_db(args.embed_db, 200, 9, 1000, 20_000)
    gen_s = time.perf_counter() - t0
    big_dev = [torch.from_numpy(d).cuda() for d in big]
    sur0 = w1.Surrogate(ctx, seed=1)
    sur0.embed(big_dev)  # warm-up (also sizes the buffers)
    ms = []
    for _ in range(3):
        sur0.embed(big_dev)
        ms.append(sur0.last_times()["embed_ms"])
    lt = sur0.last_times()
    flops = EMBED_FLOP_PER_POINT * lt["points"]
    tfl = flops / (min(ms) * 1e-3) / 1e12
    out["embed"] = {"diagrams": lt["diagrams"], "points": lt["points"], "kernel_ms": min(ms),
                    "points_per_s": lt["points"] / (min(ms) * 1e-3), "tflops": tfl,
                    "mfma_util": tfl / MFMA_BF16_PEAK_TFLOPS, "gen_s": gen_s}
    del big_dev, big
    sur0.close()
    torch.cuda.synchronize()
    if args.no_nn_search:
        return out

    # (1b) what one training label costs at the 1-NN configuration's sizes
    # (the method's certified W1 on pairs of 1k-20k-point diagrams), written
    # through the resumable label store
    import tempfile

    from paper_2110_14734_amd import labels as lbl

    cdb, _, _ = family_db(32, 20, 11, 1000, 20_000)
    cpairs = [(2 * k, 2 * k + 1) for k in range(16)]
    with tempfile.TemporaryDirectory() as td:
        store = lbl.LabelStore(os.path.join(td, "labels.bin"))
        t0 = time.perf_counter()
        _, _, cw = lbl.label_pairs(store, cpairs, lbl.method_solver(ctx, cdb, args.eps), batch=16)
        lab_s = time.perf_counter() - t0
        t0 = time.perf_counter()
        lbl.label_pairs(lbl.LabelStore(store.path), cpairs, lbl.method_solver(ctx, cdb, args.eps))  # all stored
        resume_s = time.perf_counter() - t0
    npts = float(np.mean([len(cdb[i]) + len(cdb[j]) for i, j in cpairs]))
    out["label_cost"] = {
        "what": "16 labels (the method's W1, diagonal-dominated pairs left out) on pairs of 1k-20k-point "
                "diagrams, one batch call with the host flows in parallel threads, through the label store",
        "seconds": lab_s, "s_per_label": lab_s / 16, "mean_points_per_pair": npts,
        "hours_for_200k_labels": lab_s / 16 * 200_000 / 3600, "rerun_from_store_s": resume_s,
        "all_positive": bool(np.all(np.asarray(cw) > 0))}
    del cdb

    # (2) 1-NN search on a database whose exact-flow verifications are affordable
    m, nq = args.nn_db, args.nn_queries
    db, fams, rng = family_db(m, 100, 3, 50, 500)
    rand = [(int(i), int(j)) for i, j in rng.integers(0, m, (4 * m, 2)) if i != j]
    cand = rng.integers(0, m, (m, 16))
    L = ctx.rwmd([db[i] for i in range(m) for _ in range(16)], [db[j] for j in cand.ravel()]).reshape(m, 16)
    near = [(i, int(cand[i][np.argsort(L[i])[k]])) for i in range(m) for k in range(2)]
    pairs = [p for p in rand + near if p[0] != p[1]]
    t0 = time.perf_counter()
    labels = []
    for k in range(0, len(pairs), 512):
        part = pairs[k:k + 512]
        labels += [r.w1 for r in ctx.approx_batch([db[i] for i, _ in part], [db[j] for _, j in part], eps=args.eps)]
    label_s = time.perf_counter() - t0
    labels = np.array(labels)
    keep = labels > 0
    pa = np.array([p[0] for p in pairs])[keep]
    pb = np.array([p[1] for p in pairs])[keep]
    sur = w1.Surrogate(ctx, seed=7)
    t0 = time.perf_counter()
    losses = sur.train(db, pa, pb, labels[keep], epochs=30, batch_pairs=256, lr=3e-3, seed=5)
    train_s = time.perf_counter() - t0
    qs = [pdsynth.family_pd(int(rng.integers(50, 500)), 9_000_000 + i, fams[int(rng.integers(0, 100))])
          for i in range(nq)]
    idx = w1.NNIndex(ctx, db, sur)
    res = {}
    # the method alone, the surrogate-seeded search, the s = 1 stage of the
    # paper's pipelines kept exact, and the paper's 15-3-1 pipeline (inexact)
    for mode, extra in (("rwmd", {}), ("surrogate", {}), ("sparse", {"keep": 15, "seed_k": 1}),
                        ("pipeline", {"keep": 15, "seed_k": 3})):
        idx.query(qs[:2], eps=args.eps, mode=mode, **extra)  # warm-up
        t0 = time.perf_counter()
        r = idx.query(qs, eps=args.eps, mode=mode, **extra)
        dt = time.perf_counter() - t0
        res[mode] = r
        out[f"nn_{mode}"] = {"queries_per_s": nq / dt, "verifications_per_query": r.stats["verifications"] / nq,
                             "rwmd_evals_per_query": r.stats["rwmd_evals"] / nq,
                             "sparse_evals_per_query": r.stats["sparse_evals"] / nq,
                             "t_rwmd_ms": r.stats["t_rwmd_ms"], "t_embed_ms": r.stats["t_embed_ms"],
                             "t_sparse_ms": r.stats["t_sparse_ms"], "t_verify_ms": r.stats["t_verify_ms"]}
    idx.close()
    out["nn_pipeline"]["what"] = ("keep the 15 nearest by RWMD, of those the 3 nearest by the method at s = 1 "
                                  "(the paper's grid for s = 1), return the best certified W1 of the 3: not exact")
    out["nn_pipeline"]["recall_at_1"] = float(np.mean(res["pipeline"].nn == res["rwmd"].nn))
    out["nn_identical_answers"] = bool(all(np.array_equal(res["rwmd"].nn, res[k].nn)
                                           and np.array_equal(res["rwmd"].w1, res[k].w1)
                                           for k in ("surrogate", "sparse")))
    out["nn_speedup"] = out["nn_surrogate"]["queries_per_s"] / out["nn_rwmd"]["queries_per_s"]
    out["nn_workload"] = (f"database {m} diagrams (latent-family generator, sizes log-uniform [50, 500]), "
                          f"{nq} queries, eps={args.eps}; surrogate trained on {int(keep.sum())} W1 labels "
                          f"from the method ({label_s:.1f} s to label, {train_s:.1f} s to train, "
                          f"loss {losses[0]:.3f} -> {losses[-1]:.3f})")
    sur.close()
    return out


def run_nn_c4(ctx, args):
    """1-NN search at the configured database size: 10k diagrams of 1k-20k
    points from the latent-family generator (the embedding workload's
    database), args.nn_c4 queries from the same generator, the method alone
    (RWMD order) against the surrogate-seeded search.  The surrogate is
    trained on args.nn_c4_labels method labels from that database (half on
    random pairs, half on each anchor's RWMD-nearest of 8 random candidates):
    the configured 200k labels would take ~9 hours of labelling."""
    import numpy as np

    import paper_2110_14734_amd as w1
    import pdsynth

    say = lambda msg: print(f"[bench] c4 1-NN: {msg}", file=sys.stderr, flush=True)
    db, fams, rng = family_db(10_000, 200, 9, 1000, 20_000)
    m, nl = len(db), args.nn_c4_labels
    rand = [(int(i), int(j)) for i, j in rng.integers(0, m, (nl // 2, 2)) if i != j]
    anchors = rng.integers(0, m, nl - nl // 2)
    cand = rng.integers(0, m, (anchors.shape[0], 8))
    Lr = ctx.rwmd([db[a] for a in anchors for _ in range(8)], [db[c] for c in cand.ravel()]).reshape(-1, 8)
    near = [(int(a), int(cand[k][np.argmin(Lr[k])])) for k, a in enumerate(anchors)]
    pairs = [p for p in rand + near if p[0] != p[1]]
    t0 = time.perf_counter()
    labels = []
    for k in range(0, len(pairs), 32):
        part = pairs[k:k + 32]
        labels += [r.w1 for r in ctx.approx_batch([db[i] for i, _ in part], [db[j] for _, j in part], eps=args.eps,
                                                 flags=w1.PRUNE)]
        say(f"{len(labels)} of {len(pairs)} labels")
    label_s = time.perf_counter() - t0
    labels = np.array(labels)
    keep = labels > 0
    sur = w1.Surrogate(ctx, seed=7)
    t0 = time.perf_counter()
    losses = sur.train(db, np.array([p[0] for p in pairs])[keep], np.array([p[1] for p in pairs])[keep],
                       labels[keep], epochs=40, batch_pairs=64, lr=3e-3, seed=5)
    train_s = time.perf_counter() - t0
    qs = [pdsynth.family_pd(int(np.rint(np.exp(rng.uniform(np.log(1000), np.log(20_000))))), 8_000_000 + i,
                            fams[int(rng.integers(0, 200))]) for i in range(args.nn_c4 + args.nn_c4_extra)]
    idx = w1.NNIndex(ctx, db, sur)
    out, ans = {}, {}
    for mode, qm in (("rwmd", qs[:args.nn_c4]), ("surrogate", qs[:args.nn_c4]), ("surrogate_extra", qs[args.nn_c4:])):
        if not qm:
            continue
        dt, st, nn, w = 0.0, {}, [], []
        for k, q in enumerate(qm):
            t0 = time.perf_counter()
            r = idx.query([q], eps=args.eps, mode=mode.split("_")[0])
            dt += time.perf_counter() - t0
            for key, v in r.stats.items():
                st[key] = st.get(key, 0) + v
            nn.append(int(r.nn[0]))
            w.append(float(r.w1[0]))
            say(f"{mode} query {k + 1} of {len(qm)}: {dt:.1f} s so far")
        ans[mode] = (nn, w)
        out[f"nn_{mode}"] = {"queries": len(qm), "queries_per_s": len(qm) / dt, "seconds_per_query": dt / len(qm),
                             "verifications_per_query": st["verifications"] / len(qm),
                             "rwmd_evals_per_query": st["rwmd_evals"] / len(qm),
                             "t_rwmd_ms": st["t_rwmd_ms"], "t_verify_ms": st["t_verify_ms"]}
    idx.close()
    sur.close()
    out["identical_answers"] = ans["rwmd"] == ans["surrogate"]
    out["speedup"] = out["nn_surrogate"]["queries_per_s"] / out["nn_rwmd"]["queries_per_s"]
    out["workload"] = (f"database 10000 diagrams (latent-family generator, sizes log-uniform [1k, 20k], "
                       f"{sum(len(d) for d in db)} points), {args.nn_c4} queries from the same generator in both "
                       f"modes and {args.nn_c4_extra} more in the surrogate-seeded mode, "
                       f"eps={args.eps}; surrogate trained on {int(keep.sum())} W1 labels from the method "
                       f"({label_s:.1f} s to label, {train_s:.1f} s to train, loss {losses[0]:.3f} -> "
                       f"{losses[-1]:.3f})")
    return out


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A, B, eps):
    """The CPU oracle as it stands, single thread, on the same workload:
    0-condensation, RWMD, grid, tree and the WSPD recursion with pairs
    counted rather than stored (the oracle would need ~44 GB for the pair
    list), each step timed on its own by the oracle's own timers.  The
    network O8 and the flow O9 are timed separately on the 400 + 400-point
    workload (end to end there)."""
    import oracle
    import pdsynth

    oracle.build()
    t0 = time.perf_counter()
    r = oracle.run(A, B, eps=eps, flags=oracle.ORC_COUNT_ONLY, fetch=False)
    dt = time.perf_counter() - t0
    C1a, C1b = pdsynth.exp_pd(400, 0), pdsynth.exp_pd(400, 1)
    t1 = time.perf_counter()
    c1 = oracle.run(C1a, C1b, eps=0.1, fetch=False)
    t_c1 = time.perf_counter() - t1
    n = A.shape[0] + B.shape[0]
    steps = {k: round(v, 4) for k, v in r.stage_s.items() if k not in ("O8 network", "O9 flow")}
    return {"value": n / dt, "unit": "pts/s", "cores": 1, "kind": "oracle",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "sample": f"the full {A.shape[0]}+{B.shape[0]}-point pair at eps={eps}, single thread, "
                      f"steps O0-O7 with WSPD pairs counted not stored ({r.n_pairs} pairs), {dt:.1f} s",
            "seconds": dt, "pairs": r.n_pairs, "stage_s": steps,
            "c1": {"what": "400+400-point pair at eps 0.1, end to end on one thread (exact W1 by "
                           "successive shortest paths)",
                   "pd_pairs_per_s": 1.0 / t_c1,
                   "stage_s": {k: round(v, 4) for k, v in c1.stage_s.items()}}}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the method runs on a single "
              f"MI355X; sharding across GPUs is designed but not built.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2110_14734_amd as w1
    import pdsynth

    A = pdsynth.mixture_pd(args.n, 0)
    B = pdsynth.mixture_pd(args.n, 1)
    tA = torch.from_numpy(A).cuda()
    tB = torch.from_numpy(B).cuda()
    ctx = w1.Context(0)
    flags = w1.NO_FLOW
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        ctx.approx(tA, tB, eps=args.eps, flags=flags)
    torch.cuda.synchronize()
    stage = {k: 0.0 for k in w1.T_NAMES[:6]}
    kern = {k: 0.0 for k in w1.Context.KERNEL_TIMES if k not in ("pairs", "stream_emit_ms", "record_words")}
    r = None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = ctx.approx(tA, tB, eps=args.eps, flags=flags)
        kt = ctx.kernel_times()
        for k in kern:
            kern[k] += kt[k] / args.steps
        for k in stage:
            stage[k] += r.t_ms[k] / args.steps
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    n = A.shape[0] + B.shape[0]
    P, N = r.n_pairs, r.n_cells
    kernels = {}
    rec_words = ctx.kernel_times()["record_words"]
    for k, (bp, bn) in kernel_bytes(rec_words).items():
        nbytes = bp * P + bn * N
        ach = nbytes / (kern[k] * 1e-3) / 1e9 if kern[k] > 0 else 0.0
        kernels[k] = {"kernel": KERNEL_NAMES[k], "avg_launch_ms": round(kern[k], 4), "algorithmic_bytes": nbytes,
                      "achieved_GBs": round(ach, 1), "frac": round(ach / HBM_PEAK_GBS, 4),
                      "traffic": measured_traffic(k, n, args.eps)}
    dom = max(KERNEL_BYTES, key=lambda k: kern[k])
    traffic = measured_traffic(dom, n, args.eps)
    d = kernels[dom]
    net_bytes = NETWORK_BYTES[0] * P + NETWORK_BYTES[1] * N
    a45_ms = stage["wspd"] + stage["arcs"]
    out = {
        "metric": METRIC,
        "value": n / (dt / args.steps),
        "unit": "pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+int32",
        "data": "synthetic",
        "config": {
            "workload": f"plain method at scale: two {args.n}-point FP32 persistence diagrams "
                        f"(80% persistence LogNormal(-4,1), 20% U[0.1,1], birth U[0,1)), eps={args.eps}, "
                        f"GPU sparsification a0-a5 incl. the (tail, head)-sorted CSR network (host flow excluded)",
            "n_points": n, "eps": args.eps, "s": r.s, "grid_exp": r.grid_exp, "cells": N,
            "wspd_pairs": P, "network_arcs": r.n_arcs,
        },
        "pd_pairs_per_s": args.steps / dt,
        "wspd_pairs_per_s": P / (dt / args.steps),
        "stage_ms": {k: round(v, 3) for k, v in stage.items()},
        "wspd_kernel_ms": {k: round(v, 3) for k, v in kern.items()},
        "roofline": {
            "kernel": d["kernel"],
            "bound": "hbm",
            "achieved": d["achieved_GBs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": d["frac"],
            "traffic": traffic,
            "traffic_ratio": (traffic / d["algorithmic_bytes"]) if traffic else None,
            "algorithmic_bytes_per_launch": d["algorithmic_bytes"],
            "avg_launch_ms": d["avg_launch_ms"],
        },
        "kernels": kernels,
        "pair_record_bytes": 4 * rec_words,
        "network_roofline": {
            "what": "a4+a5 stage time against the final network's bytes (16 B per WSPD pair, 8 B per cell)",
            "bytes": net_bytes, "ms": round(a45_ms, 3),
            "achieved_GBs": round(net_bytes / (a45_ms * 1e-3) / 1e9, 1),
            "frac": round(net_bytes / (a45_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        },
    }
    # the same step with the Euclidean ground metric (the paper's own)
    ctx.approx(tA, tB, eps=args.eps, flags=flags | w1.METRIC_L2)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        rl = ctx.approx(tA, tB, eps=args.eps, flags=flags | w1.METRIC_L2)
    torch.cuda.synchronize()
    tl = (time.perf_counter() - t1) / args.steps
    out["l2_step"] = {"what": "the same step with the Euclidean ground metric (64-bit network costs)",
                      "ms_per_step": 1e3 * tl, "points_per_s": n / tl, "wspd_pairs": rl.n_pairs,
                      "network_arcs": rl.n_arcs, "grid_exp": rl.grid_exp, "cost_shift": rl.cost_shift}
    # the same step with the diagonal-dominated pairs left out (W1_PRUNE)
    ctx.approx(tA, tB, eps=args.eps, flags=flags | w1.PRUNE)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        rp = ctx.approx(tA, tB, eps=args.eps, flags=flags | w1.PRUNE)
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t1) / args.steps
    out["pruned_step"] = {"what": "the same step with diagonal-dominated WSPD pairs left out (F* unchanged)",
                          "ms_per_step": 1e3 * tp, "points_per_s": n / tp, "wspd_pairs": rp.n_pairs,
                          "network_arcs": rp.n_arcs}
    if args.calib_copy_mb:
        src = torch.empty(args.calib_copy_mb << 20, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = src.numel()
        del src, dst
    if not args.no_c1:
        # end to end incl. host network simplex, 400 + 400 points, eps 0.1
        C1a, C1b = pdsynth.exp_pd(400, 0), pdsynth.exp_pd(400, 1)
        reps = 20

        def per_call(flags):
            for _ in range(3):
                ctx.approx(C1a, C1b, eps=0.1, flags=flags)
            t1 = time.perf_counter()
            for _ in range(reps):
                r = ctx.approx(C1a, C1b, eps=0.1, flags=flags)
            return r, (time.perf_counter() - t1) / reps

        g, e2e = per_call(0)
        gp, e2p = per_call(w1.PRUNE)
        gl, e2l = per_call(w1.METRIC_L2)
        out["c1_l2_end_to_end"] = {"pd_pairs_per_s": 1.0 / e2l, "ms": 1e3 * e2l, "w1": gl.w1,
                                   "flow_ms": gl.t_ms["flow"], "wspd_pairs": gl.n_pairs}
        out["c1_end_to_end"] = {"pd_pairs_per_s": 1.0 / e2e, "ms": 1e3 * e2e, "w1": g.w1,
                                "flow_ms": g.t_ms["flow"], "wspd_pairs": g.n_pairs,
                                "pruned": {"what": "diagonal-dominated WSPD pairs left out (same F* and W1)",
                                           "pd_pairs_per_s": 1.0 / e2p, "ms": 1e3 * e2p, "w1": gp.w1,
                                           "flow_ms": gp.t_ms["flow"], "wspd_pairs": gp.n_pairs,
                                           "same_w1": bool(gp.w1 == g.w1)}}
    if not args.no_batch:
        out["batched"] = run_batch(ctx, args)
    if not args.no_stress:
        out["stress"] = run_stress(ctx, args)
    if not args.no_nn:
        out["learned"] = run_nn(ctx, args)
    if args.nn_c4 > 0:
        out["learned_c4"] = run_nn_c4(ctx, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, B, args.eps)
    ctx.close()
    print(json.dumps(out), flush=True)
    del np


if __name__ == "__main__":
    main()

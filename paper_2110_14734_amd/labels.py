"""Resumable store of W1 labels for training the surrogate.

Labels are the method's certified W1 on pairs (i, j) of database diagrams.
At the configured 1-NN scale each one is an exact flow on a network of 10^7
arcs or more, so a labelling run takes hours and must survive being stopped:
records (i, j, w1) are appended to a binary file and flushed to disk batch by
batch, and a run that starts again computes only the pairs the file lacks.

File layout: the 8-byte magic ``W1LABEL1``, then 24-byte records
(int64 i, int64 j, float64 w1), little-endian.  A record cut short by a crash
is dropped when the file is opened.
"""
from __future__ import annotations

import os

import numpy as np

MAGIC = b"W1LABEL1"
RECORD = np.dtype([("i", "<i8"), ("j", "<i8"), ("w1", "<f8")])


class LabelStore:
    """Append-only (i, j, w1) records in one file."""

    def __init__(self, path: str):
        self.path = path
        if not os.path.exists(path) or os.path.getsize(path) == 0:
            with open(path, "wb") as f:
                f.write(MAGIC)
                f.flush()
                os.fsync(f.fileno())
        with open(path, "rb") as f:
            if f.read(len(MAGIC)) != MAGIC:
                raise ValueError(f"{path} is not a label store")
        size = os.path.getsize(path)
        whole = len(MAGIC) + (size - len(MAGIC)) // RECORD.itemsize * RECORD.itemsize
        if whole != size:  # a record cut short: drop it
            with open(path, "r+b") as f:
                f.truncate(whole)

    def load(self) -> np.ndarray:
        """Every record, in the order written."""
        with open(self.path, "rb") as f:
            f.seek(len(MAGIC))
            return np.frombuffer(f.read(), dtype=RECORD).copy()

    def __len__(self) -> int:
        return (os.path.getsize(self.path) - len(MAGIC)) // RECORD.itemsize

    def append(self, i, j, w1) -> None:
        """Append records and make them durable before returning."""
        rec = np.empty(len(i), dtype=RECORD)
        rec["i"], rec["j"], rec["w1"] = i, j, w1
        with open(self.path, "ab") as f:
            f.write(rec.tobytes())
            f.flush()
            os.fsync(f.fileno())


def label_pairs(store: LabelStore, pairs, solve, batch: int = 512):
    """Labels of `pairs` ((i, j) tuples): those already in the store are
    reused, the rest are computed `batch` at a time by solve(list of (i, j))
    -> w1 values and appended as they come.  Returns (i, j, w1) arrays in the
    order of `pairs`."""
    have = {(int(r["i"]), int(r["j"])): float(r["w1"]) for r in store.load()}
    todo = [p for p in dict.fromkeys((int(a), int(b)) for a, b in pairs) if p not in have]
    for k in range(0, len(todo), batch):
        part = todo[k:k + batch]
        w = np.asarray(solve(part), dtype=np.float64)
        if w.shape != (len(part),):
            raise ValueError("solve must return one value per pair")
        store.append([a for a, _ in part], [b for _, b in part], w)
        have.update(zip(part, w.tolist()))
    i = np.array([int(a) for a, _ in pairs], np.int64)
    j = np.array([int(b) for _, b in pairs], np.int64)
    return i, j, np.array([have[(int(a), int(b))] for a, b in pairs])


def method_solver(ctx, db, eps: float = 0.1, flags: int = 0):
    """solve() for label_pairs: the method's certified W1 on the GPU, with the
    diagonal-dominated pairs left out of each network (the same W1)."""
    from . import PRUNE

    def solve(part):
        res = ctx.approx_batch([db[i] for i, _ in part], [db[j] for _, j in part], eps=eps, flags=PRUNE | flags)
        return [r.w1 for r in res]

    return solve

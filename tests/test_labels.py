"""The resumable label store (CPU): records survive reopening, a record cut
short by a crash is dropped, and a second run computes only missing pairs."""
import numpy as np
import pytest

from paper_2110_14734_amd import labels


def test_store_roundtrip_and_resume(tmp_path):
    path = str(tmp_path / "w.lbl")
    st = labels.LabelStore(path)
    calls = []

    def solve(part):
        calls.append(list(part))
        return [i * 100.0 + j for i, j in part]

    pairs = [(1, 2), (3, 4), (1, 2), (5, 6), (7, 8)]
    i, j, w = labels.label_pairs(st, pairs[:3], solve, batch=2)
    assert list(w) == [102.0, 304.0, 102.0] and calls == [[(1, 2), (3, 4)]]
    # a crash in the middle of the next append leaves a partial record
    with open(path, "ab") as f:
        f.write(b"\x01" * 10)
    st2 = labels.LabelStore(path)
    assert len(st2) == 2
    calls.clear()
    i, j, w = labels.label_pairs(st2, pairs, solve, batch=2)
    assert calls == [[(5, 6), (7, 8)]]
    assert list(i) == [a for a, _ in pairs] and list(j) == [b for _, b in pairs]
    assert list(w) == [a * 100.0 + b for a, b in pairs]
    rec = labels.LabelStore(path).load()
    assert [(int(r["i"]), int(r["j"])) for r in rec] == [(1, 2), (3, 4), (5, 6), (7, 8)]


def test_store_rejects_other_files(tmp_path):
    p = tmp_path / "x"
    p.write_bytes(b"not a store")
    with pytest.raises(ValueError):
        labels.LabelStore(str(p))


def test_solver_must_return_one_value_per_pair(tmp_path):
    st = labels.LabelStore(str(tmp_path / "w.lbl"))
    with pytest.raises(ValueError):
        labels.label_pairs(st, [(0, 1), (1, 2)], lambda part: [1.0])
    assert len(st) == 0

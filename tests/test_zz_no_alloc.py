"""The allocation-free RWMD entry point (w1_rwmd_noalloc) against w1_rwmd:
identical lower bounds (bit for bit: the same kernels on the same inputs) on
two calls in a row, the second smaller than the first, on a fresh context
that makes no device allocation; the size limits are rejected before any
work."""
import sys

import numpy as np
import pytest

import pdsynth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_rwmd_noalloc_matches_rwmd():
    import torch

    import paper_2110_14734_amd as w1

    _say("[gpu] rwmd noalloc: fresh context")
    torch.cuda.init()
    # load every kernel module and the runtime's pools through another
    # context first, so the fresh context below is the only new user
    warm = w1.Context(0)
    warm.rwmd([pdsynth.exp_pd(50, 1)], [pdsynth.exp_pd(40, 2)], noalloc=True)
    warm.rwmd([pdsynth.exp_pd(50, 1)], [pdsynth.exp_pd(40, 2)])
    warm.close()
    ctx = w1.Context(0)
    try:
        # first call: a batch of mixture pairs (FP32), 2^19 points in all
        sizes = [120_000, 131_072, 90_000, 100_000, 40_000, 20_000, 12_000, 11_216]
        assert sum(sizes) == 1 << 19
        As = [pdsynth.mixture_pd(sizes[2 * i], 7000 + 2 * i) for i in range(4)]
        Bs = [pdsynth.mixture_pd(sizes[2 * i + 1], 7001 + 2 * i) for i in range(4)]
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        L1 = ctx.rwmd(As, Bs, noalloc=True)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        # the normal path would allocate well over 100 MB for these points
        assert free0 - free1 < (8 << 20), (free0, free1)
        # second call: smaller, FP64, with an empty diagram and a one-sided pair
        C = [pdsynth.exp_pd(400, 11), np.zeros((0, 2)), pdsynth.exp_pd(3, 13)]
        D = [pdsynth.exp_pd(380, 12), pdsynth.exp_pd(50, 14), np.zeros((0, 2))]
        L2 = ctx.rwmd(C, D, noalloc=True)
        _say("[gpu] rwmd noalloc: reference calls")
        R1 = ctx.rwmd(As, Bs)
        R2 = ctx.rwmd(C, D)
        assert np.array_equal(L1, R1) and np.array_equal(L2, R2)
        assert (L1 > 0).all() and L2[0] > 0 and L2[1] > 0 and L2[2] > 0
        # a normal call in between leaves the allocation-free path unchanged
        assert np.array_equal(ctx.rwmd(C, D, noalloc=True), R2)
        # device inputs on the current stream
        tC = [torch.from_numpy(x).cuda() for x in C[:1]]
        tD = [torch.from_numpy(x).cuda() for x in D[:1]]
        assert np.array_equal(ctx.rwmd(tC, tD, noalloc=True), R2[:1])
        # limits: more than 2^19 points, more than 1024 pairs
        with pytest.raises(w1.W1Error) as e:
            ctx.rwmd(As + [pdsynth.exp_pd(1, 1)], Bs + [np.zeros((0, 2))], noalloc=True)
        assert e.value.code == w1.W1_ERANGE
        tiny = [pdsynth.exp_pd(1, 2)] * 1025
        with pytest.raises(w1.W1Error) as e:
            ctx.rwmd(tiny, tiny, noalloc=True)
        assert e.value.code == w1.W1_ERANGE
        # invalid point: NaN for that pair, like w1_rwmd
        bad = np.array([[1.0, 0.5]])
        Lb = ctx.rwmd([bad, C[0]], [C[0], D[0]], noalloc=True)
        Rb = ctx.rwmd([bad, C[0]], [C[0], D[0]])
        assert np.isnan(Lb[0]) and np.isnan(Rb[0]) and Lb[1] == Rb[1] == R2[0]
    finally:
        ctx.close()

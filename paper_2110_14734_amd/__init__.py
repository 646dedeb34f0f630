"""Python binding of libw1approx (approximate W1 between persistence diagrams
on AMD MI355X).  Argument marshalling only: every step of the method runs in
the HIP library; there is no Python or CPU fallback, and calls fail loudly
when the library is missing.

    import paper_2110_14734_amd as w1
    ctx = w1.Context()
    r = ctx.approx(A, B, eps=0.1)      # A, B: (n, 2) numpy arrays or torch tensors
    r.w1, r.lower_bound, r.n_pairs
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libw1approx.so")

W1_OK, W1_EINVAL, W1_ERANGE, W1_ENOMEM, W1_EHIP, W1_EOVERFLOW, W1_ENODEV = 0, -1, -2, -3, -4, -5, -6
W1_OPTIMAL, W1_STALLED = 0, 1
W1_F32, W1_F64 = 0, 1
INPUT_DEVICE, COUNT_ONLY, NO_FLOW, KEEP_NETWORK, KEEP_STAGES, PRUNE, METRIC_L2 = 1, 2, 4, 8, 16, 32, 64
PAPER_GRID = 128
T_NAMES = ("condense0", "rwmd", "grid", "tree", "wspd", "arcs", "d2h", "flow")


class W1Error(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        super().__init__(f"{what}: {strerror(code)} ({code})" if what else f"{strerror(code)} ({code})")
        self.code = code


class _PD(ctypes.Structure):
    _fields_ = [("xy", ctypes.c_void_p), ("n", ctypes.c_int64), ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("cond_frac", ctypes.c_double), ("s_override", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("pivot_cap", ctypes.c_int64)]


_P = ctypes.c_void_p


class _Result(ctypes.Structure):
    _fields_ = [
        ("w1", ctypes.c_double), ("w1_paper", ctypes.c_double), ("lower_bound", ctypes.c_double),
        ("grid", ctypes.c_double), ("grid_exp", ctypes.c_int32), ("s", ctypes.c_int32),
        ("status", ctypes.c_int32), ("flow_solved", ctypes.c_int32), ("n_points", ctypes.c_int64),
        ("n_a", ctypes.c_int64), ("n_b", ctypes.c_int64), ("n_locations", ctypes.c_int64),
        ("n_cells", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("n_arcs", ctypes.c_int64),
        ("flow_cost", ctypes.c_int64), ("pivots", ctypes.c_int64),
        ("n_pairs_streamed", ctypes.c_int64), ("pair_checksum", ctypes.c_uint64 * 2),
        ("cell_i", _P), ("cell_j", _P), ("cell_ca", _P), ("cell_cb", _P), ("supply", _P),
        ("row_ptr", _P), ("col", _P), ("cost", _P), ("cost64", _P), ("n_diag", ctypes.c_int64),
        ("metric_l2", ctypes.c_int32), ("cost_shift", ctypes.c_int32),
        ("loc_b", _P), ("loc_d", _P), ("loc_w", _P), ("loc_t", _P),
        ("rwmd_sum_a", ctypes.c_int64), ("rwmd_sum_b", ctypes.c_int64),
        ("rwmd_shift_a", ctypes.c_int32), ("rwmd_shift_b", ctypes.c_int32),
        ("node_lo", _P), ("node_hi", _P), ("node_left", _P), ("node_right", _P), ("node_box", _P),
        ("t_ms", ctypes.c_double * 8),
    ]


class _DevNet(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("n_arcs", ctypes.c_int64),
                ("cell_ij", _P), ("cell_ca", _P), ("cell_cb", _P), ("supply", _P), ("row_ptr", _P),
                ("col", _P), ("cost", _P), ("cost64", _P)]


class _TrainParams(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch_pairs", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("adam_eps", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class _Tuning(ctypes.Structure):
    _fields_ = [("stack_depth", ctypes.c_int32), ("work_cap", ctypes.c_int32), ("chunk_items", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("max_points_per_launch", ctypes.c_int64),
                ("compact_records", ctypes.c_int32), ("stream_max_rounds", ctypes.c_int32),
                ("stream_arena_pairs", ctypes.c_int64), ("blocked_emit", ctypes.c_int32),
                ("sort_window_words", ctypes.c_int32), ("emit_block_limit", ctypes.c_int64),
                ("fused_expand_cells", ctypes.c_int32), ("fused_expand_items", ctypes.c_int32),
                ("stream_graph", ctypes.c_int32)]


class _NNParams(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("mode", ctypes.c_int32), ("seed_k", ctypes.c_int32),
                ("keep", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _NNStats(ctypes.Structure):
    _fields_ = [("verifications", ctypes.c_int64), ("rwmd_evals", ctypes.c_int64), ("rounds", ctypes.c_int64),
                ("t_rwmd_ms", ctypes.c_double), ("t_embed_ms", ctypes.c_double), ("t_verify_ms", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("sparse_evals", ctypes.c_int64), ("t_sparse_ms", ctypes.c_double)]


SURR_NPARAM = 25152
SURR_EMB = 64
NN_RWMD, NN_SURROGATE, NN_EXHAUSTIVE, NN_SPARSE, NN_PIPELINE = 0, 1, 2, 3, 4
NN_MODES = {"rwmd": NN_RWMD, "surrogate": NN_SURROGATE, "exhaustive": NN_EXHAUSTIVE, "sparse": NN_SPARSE,
            "pipeline": NN_PIPELINE}

# Every symbol include/w1approx.h declares.
EXPORTS = ("w1_ctx_create", "w1_ctx_destroy", "w1_ctx_hip_error", "w1_ctx_last_kernel_times", "w1_approx",
           "w1_approx_batch", "w1_rwmd", "w1_rwmd_noalloc", "w1_device_network_get", "w1_flow_solve", "w1_separation_for_eps",
           "w1_ctx_get_tuning", "w1_ctx_set_tuning",
           "w1_result_free", "w1_strerror", "w1_surrogate_create", "w1_surrogate_destroy",
           "w1_surrogate_get_params", "w1_surrogate_set_params", "w1_surrogate_embed", "w1_surrogate_grad",
           "w1_surrogate_train", "w1_surrogate_last_times", "w1_nn_build", "w1_nn_destroy", "w1_nn_query")

_lib = None


def lib():
    """Load libw1approx.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: build it with "
                               "`python -m paper_2110_14734_amd.build` (there is no CPU fallback)")
        try:
            # Load torch's HIP runtime first so the library binds to the same
            # runtime instance that owns torch's device memory and streams.
            import torch  # noqa: F401
        except ImportError:  # pragma: no cover
            pass
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
        L.w1_ctx_create.argtypes = [i32, ctypes.POINTER(vp)]
        L.w1_ctx_destroy.argtypes = [vp]
        L.w1_ctx_hip_error.argtypes = [vp]
        L.w1_approx.argtypes = [vp, ctypes.POINTER(_PD), ctypes.POINTER(_PD), ctypes.POINTER(_Params), vp,
                                ctypes.POINTER(_Result)]
        L.w1_approx_batch.argtypes = [vp, ctypes.POINTER(_PD), ctypes.POINTER(_PD), i64, ctypes.POINTER(_Params), vp,
                                      ctypes.POINTER(_Result)]
        L.w1_rwmd.argtypes = [vp, ctypes.POINTER(_PD), ctypes.POINTER(_PD), i64, ctypes.c_uint32, vp,
                              ctypes.POINTER(ctypes.c_double)]
        L.w1_rwmd_noalloc.argtypes = [vp, ctypes.POINTER(_PD), ctypes.POINTER(_PD), i64, ctypes.c_uint32, vp,
                                      ctypes.POINTER(ctypes.c_double)]
        L.w1_device_network_get.argtypes = [vp, i64, ctypes.POINTER(_DevNet)]
        L.w1_flow_solve.argtypes = [i64, i64, vp, vp, vp, vp, i64, ctypes.POINTER(i64), vp, vp, ctypes.POINTER(i64),
                                    ctypes.POINTER(ctypes.c_int32)]
        L.w1_ctx_last_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32]
        L.w1_ctx_get_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
        L.w1_ctx_set_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
        L.w1_separation_for_eps.argtypes = [ctypes.c_double, ctypes.c_double]
        L.w1_result_free.argtypes = [ctypes.POINTER(_Result)]
        L.w1_result_free.restype = None
        L.w1_strerror.argtypes = [i32]
        L.w1_strerror.restype = ctypes.c_char_p
        f32p, f64p, i64p = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)
        L.w1_surrogate_create.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(vp)]
        L.w1_surrogate_destroy.argtypes = [vp]
        L.w1_surrogate_get_params.argtypes = [vp, f32p, i64]
        L.w1_surrogate_set_params.argtypes = [vp, f32p, i64]
        L.w1_surrogate_embed.argtypes = [vp, vp, ctypes.POINTER(_PD), i64, ctypes.c_uint32, vp, f32p]
        L.w1_surrogate_grad.argtypes = [vp, vp, ctypes.POINTER(_PD), i64, i64p, i64p, f64p, i64, ctypes.c_uint32, vp,
                                        f64p, f32p]
        L.w1_surrogate_train.argtypes = [vp, vp, ctypes.POINTER(_PD), i64, i64p, i64p, f64p, i64,
                                         ctypes.POINTER(_TrainParams), ctypes.c_uint32, vp, f64p]
        L.w1_surrogate_last_times.argtypes = [vp, f64p, i32]
        L.w1_nn_build.argtypes = [vp, vp, ctypes.POINTER(_PD), i64, ctypes.c_uint32, vp, ctypes.POINTER(vp)]
        L.w1_nn_destroy.argtypes = [vp]
        L.w1_nn_query.argtypes = [vp, vp, vp, ctypes.POINTER(_PD), i64, ctypes.POINTER(_NNParams), ctypes.c_uint32,
                                  vp, i64p, f64p, i64p, ctypes.POINTER(_NNStats)]
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().w1_strerror(int(code)).decode()


def separation_for_eps(eps: float, kappa: float = 0.1) -> int:
    s = lib().w1_separation_for_eps(float(eps), float(kappa))
    if s < 0:
        raise W1Error(s, "separation_for_eps")
    return s


def flow_solve(n_nodes, src, dst, cost, supply, pivot_cap=0, certificate=False):
    """Host network simplex of the library on any network (non-negative
    integer costs).  Returns (cost, pivots, status[, flow, potentials])."""
    src = np.ascontiguousarray(src, np.uint32)
    dst = np.ascontiguousarray(dst, np.uint32)
    cost = np.ascontiguousarray(cost, np.int32)
    supply = np.ascontiguousarray(supply, np.int64)
    m = src.shape[0]
    out_c, piv, st = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    flow = np.zeros(m, np.int64) if certificate else None
    pot = np.zeros(n_nodes, np.int64) if certificate else None
    p = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    rc = lib().w1_flow_solve(int(n_nodes), m, p(src), p(dst), p(cost), p(supply), int(pivot_cap),
                             ctypes.byref(out_c), p(flow), p(pot), ctypes.byref(piv), ctypes.byref(st))
    if rc != 0:
        raise W1Error(rc, "flow_solve")
    if certificate:
        return out_c.value, piv.value, st.value, flow, pot
    return out_c.value, piv.value, st.value


@dataclass
class Result:
    status: int
    w1: float
    w1_paper: float
    lower_bound: float
    grid: float
    grid_exp: int
    s: int
    flow_solved: bool
    n_points: int
    n_a: int
    n_b: int
    n_locations: int
    n_cells: int
    n_pairs: int
    n_arcs: int
    flow_cost: int
    pivots: int
    t_ms: dict
    n_pairs_streamed: int = 0
    metric_l2: bool = False
    cost_shift: int = 0
    pair_checksum: tuple = (0, 0)
    network: dict = field(default_factory=dict)
    stages: dict = field(default_factory=dict)


def _arr(ptr, n, dtype):
    if not ptr or n <= 0:
        return np.zeros(0, dtype)
    ct = np.ctypeslib.as_ctypes_type(np.dtype(dtype))
    return np.ctypeslib.as_array(ctypes.cast(ptr, ctypes.POINTER(ct)), shape=(int(n),)).copy()


def _convert(r: _Result) -> Result:
    out = Result(
        status=r.status, w1=r.w1, w1_paper=r.w1_paper, lower_bound=r.lower_bound, grid=r.grid,
        grid_exp=r.grid_exp, s=r.s, flow_solved=bool(r.flow_solved), n_points=r.n_points, n_a=r.n_a,
        n_b=r.n_b, n_locations=r.n_locations, n_cells=r.n_cells, n_pairs=r.n_pairs, n_arcs=r.n_arcs,
        flow_cost=r.flow_cost, pivots=r.pivots, t_ms={k: r.t_ms[i] for i, k in enumerate(T_NAMES)},
        n_pairs_streamed=r.n_pairs_streamed, metric_l2=bool(r.metric_l2), cost_shift=r.cost_shift, pair_checksum=(int(r.pair_checksum[0]), int(r.pair_checksum[1])))
    if r.row_ptr:
        nc = r.n_cells
        out.network = dict(
            cell_i=_arr(r.cell_i, nc, np.int32), cell_j=_arr(r.cell_j, nc, np.int32),
            cell_ca=_arr(r.cell_ca, nc, np.int32), cell_cb=_arr(r.cell_cb, nc, np.int32),
            supply=_arr(r.supply, nc + 2, np.int64), row_ptr=_arr(r.row_ptr, nc + 3, np.int64),
            col=_arr(r.col, r.n_arcs, np.uint32),
            cost=_arr(r.cost64, r.n_arcs, np.int64) if r.cost64 else _arr(r.cost, r.n_arcs, np.int32))
    if r.loc_b:
        nl = r.n_locations
        out.stages = dict(loc_b=_arr(r.loc_b, nl, np.float64), loc_d=_arr(r.loc_d, nl, np.float64),
                          loc_w=_arr(r.loc_w, nl, np.int32), loc_t=_arr(r.loc_t, nl, np.float64),
                          rwmd_sum_a=r.rwmd_sum_a, rwmd_sum_b=r.rwmd_sum_b, rwmd_shift_a=r.rwmd_shift_a,
                          rwmd_shift_b=r.rwmd_shift_b)
        if r.node_lo:
            ni = max(r.n_cells - 1, 0)
            out.stages.update(node_lo=_arr(r.node_lo, ni, np.int32), node_hi=_arr(r.node_hi, ni, np.int32),
                              node_left=_arr(r.node_left, ni, np.int32), node_right=_arr(r.node_right, ni, np.int32),
                              node_box=_arr(r.node_box, 4 * ni, np.int32).reshape(-1, 4))
    return out


def _is_torch(X) -> bool:
    return type(X).__module__.split(".")[0] == "torch"


def _pd_of(X, keep):
    """(w1_pd, is_device) of a numpy array or torch tensor."""
    if _is_torch(X):
        import torch

        if X.dtype not in (torch.float32, torch.float64):
            X = X.to(torch.float64)
        X = X.reshape(-1, 2).contiguous()
        keep.append(X)
        dt = W1_F32 if X.dtype == torch.float32 else W1_F64
        if X.is_cuda:
            return _PD(X.data_ptr() if X.numel() else None, X.shape[0], dt, 0), True
        X = X.numpy()
    X = np.asarray(X)
    if X.dtype not in (np.float32, np.float64):
        X = X.astype(np.float64)
    X = np.ascontiguousarray(X).reshape(-1, 2)
    keep.append(X)
    dt = W1_F32 if X.dtype == np.float32 else W1_F64
    return _PD(X.ctypes.data if X.size else None, X.shape[0], dt, 0), False


def _stream_of(dev):
    if not dev:
        return None
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _init_torch_device(device: int) -> None:
    """Initialise torch's device context (same HIP runtime instance as the
    library) before the library touches the device, so torch's own lazy
    initialisation never runs after the library has used the runtime."""
    try:
        import torch
    except ImportError:  # pragma: no cover
        return
    if torch.cuda.is_available() and device < torch.cuda.device_count():
        with torch.cuda.device(device):
            torch.cuda.current_stream().synchronize()


class Context:
    """A library context on one GPU (not thread-safe; one per thread)."""

    def __init__(self, device: int = 0):
        _init_torch_device(device)
        h = ctypes.c_void_p()
        rc = lib().w1_ctx_create(int(device), ctypes.byref(h))
        if rc != 0:
            raise W1Error(rc, "w1_ctx_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().w1_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _params(self, eps, kappa, s_override, flags, pivot_cap):
        return _Params(float(eps), float(kappa), int(s_override), int(flags), int(pivot_cap))

    def approx(self, A, B, eps=0.1, kappa=0.1, s_override=0, flags=0, pivot_cap=0) -> Result:
        """Approximate W1 of one pair (Alg. 3).  Raises W1Error on failure."""
        return self.approx_batch([A], [B], eps, kappa, s_override, flags, pivot_cap)[0]

    def approx_batch(self, As, Bs, eps=0.1, kappa=0.1, s_override=0, flags=0, pivot_cap=0, check=True):
        k = len(As)
        if k != len(Bs) or k == 0:
            raise ValueError("need equally many A and B diagrams")
        keep = []
        pa, pb = (_PD * k)(), (_PD * k)()
        devs = set()
        for i in range(k):
            pa[i], d1 = _pd_of(As[i], keep)
            pb[i], d2 = _pd_of(Bs[i], keep)
            devs.update((d1, d2))
        if len(devs) != 1:
            raise ValueError("mix of host and device diagrams")
        dev = devs.pop()
        if dev:
            flags |= INPUT_DEVICE
        res = (_Result * k)()
        prm = self._params(eps, kappa, s_override, flags, pivot_cap)
        rc = lib().w1_approx_batch(self._h, pa, pb, k, ctypes.byref(prm), _stream_of(dev), res)
        try:
            if rc != 0:
                raise W1Error(rc, f"w1_approx_batch (hip error {lib().w1_ctx_hip_error(self._h)})")
            out = [_convert(res[i]) for i in range(k)]
        finally:
            for i in range(k):
                lib().w1_result_free(ctypes.byref(res[i]))
        if check:
            for r in out:
                if r.status < 0:
                    raise W1Error(r.status, "pair")
        return out

    def rwmd(self, As, Bs, noalloc=False, flags=0) -> np.ndarray:
        """RWMD lower bounds of k pairs (Alg. 1); NaN marks an invalid pair.
        noalloc: through w1_rwmd_noalloc (no device allocation; at most 2^19
        points in all pairs and 1024 pairs).  flags: METRIC_L2 for the
        Euclidean metric."""
        k = len(As)
        keep = []
        pa, pb = (_PD * k)(), (_PD * k)()
        devs = set()
        for i in range(k):
            pa[i], d1 = _pd_of(As[i], keep)
            pb[i], d2 = _pd_of(Bs[i], keep)
            devs.update((d1, d2))
        dev = devs.pop()
        out = np.zeros(k)
        fn = lib().w1_rwmd_noalloc if noalloc else lib().w1_rwmd
        rc = fn(self._h, pa, pb, k, (INPUT_DEVICE if dev else 0) | int(flags), _stream_of(dev),
                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if rc != 0:
            raise W1Error(rc, "w1_rwmd_noalloc" if noalloc else "w1_rwmd")
        return out

    @property
    def tuning(self) -> dict:
        """WSPD traversal and batching tunables (see w1_tuning)."""
        t = _Tuning()
        rc = lib().w1_ctx_get_tuning(self._h, ctypes.byref(t))
        if rc != 0:
            raise W1Error(rc, "w1_ctx_get_tuning")
        return {f: getattr(t, f) for f, _ in _Tuning._fields_}

    @tuning.setter
    def tuning(self, v: dict):
        cur = self.tuning
        cur.update(v)
        t = _Tuning(*(int(cur[f]) for f, _ in _Tuning._fields_))
        rc = lib().w1_ctx_set_tuning(self._h, ctypes.byref(t))
        if rc != 0:
            raise W1Error(rc, "w1_ctx_set_tuning")

    KERNEL_TIMES = ("worklist_ms", "count_ms", "emit_ms", "pairs", "stream_emit_ms", "bucket_scatter_ms",
                    "row_hist_ms", "row_scatter_ms", "row_sort_ms", "emit_blocks", "fused_expand", "record_words")

    def kernel_times(self) -> dict:
        """HIP-event times (ms) of the last call's WSPD and network kernels."""
        n = len(self.KERNEL_TIMES)
        out = (ctypes.c_double * n)()
        rc = lib().w1_ctx_last_kernel_times(self._h, out, n)
        if rc != 0:
            raise W1Error(rc, "w1_ctx_last_kernel_times")
        d = {k: out[i] for i, k in enumerate(self.KERNEL_TIMES)}
        d["pairs"] = int(d["pairs"])
        d["emit_blocks"] = int(d["emit_blocks"])
        d["record_words"] = int(d["record_words"])
        return d

    def device_network(self, k: int = 0) -> dict:
        """Sizes and raw device pointers of pair k's network from the last call."""
        d = _DevNet()
        rc = lib().w1_device_network_get(self._h, int(k), ctypes.byref(d))
        if rc != 0:
            raise W1Error(rc, "w1_device_network_get")
        return {f: getattr(d, f) for f, _ in _DevNet._fields_}


def _pd_list(ds, keep):
    """w1_pd array of a list of diagrams (all host or all device)."""
    k = len(ds)
    arr = (_PD * k)()
    devs = set()
    for i, D in enumerate(ds):
        arr[i], dv = _pd_of(D, keep)
        devs.add(dv)
    if len(devs) > 1:
        raise ValueError("mix of host and device diagrams")
    return arr, (devs.pop() if devs else False)


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype)
    return a, a.ctypes.data_as(ctypes.POINTER(np.ctypeslib.as_ctypes_type(np.dtype(dtype))))


class Surrogate:
    """DeepSets surrogate of W1 on one GPU (its kernels run in the library)."""

    def __init__(self, ctx: Context, seed: int = 0):
        h = ctypes.c_void_p()
        rc = lib().w1_surrogate_create(ctx._h, ctypes.c_uint64(seed), ctypes.byref(h))
        if rc != 0:
            raise W1Error(rc, "w1_surrogate_create")
        self._h, self.ctx = h, ctx

    def close(self):
        if getattr(self, "_h", None):
            lib().w1_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def params(self) -> np.ndarray:
        out = np.zeros(SURR_NPARAM, np.float32)
        _, p = _c(out, np.float32)
        rc = lib().w1_surrogate_get_params(self._h, p, SURR_NPARAM)
        if rc != 0:
            raise W1Error(rc, "w1_surrogate_get_params")
        return out

    @params.setter
    def params(self, v):
        a, p = _c(v, np.float32)
        rc = lib().w1_surrogate_set_params(self._h, p, a.size)
        if rc != 0:
            raise W1Error(rc, "w1_surrogate_set_params")

    def embed(self, ds) -> np.ndarray:
        keep = []
        arr, dev = _pd_list(ds, keep)
        out = np.zeros((len(ds), SURR_EMB), np.float32)
        rc = lib().w1_surrogate_embed(self.ctx._h, self._h, arr, len(ds), INPUT_DEVICE if dev else 0,
                                      _stream_of(dev), out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        if rc != 0:
            raise W1Error(rc, "w1_surrogate_embed")
        return out

    def last_times(self) -> dict:
        out = (ctypes.c_double * 3)()
        lib().w1_surrogate_last_times(self._h, out, 3)
        return {"embed_ms": out[0], "points": int(out[1]), "diagrams": int(out[2])}

    def grad(self, ds, pa, pb, w):
        """(loss, gradient) over labelled pairs, without an update."""
        keep = []
        arr, dev = _pd_list(ds, keep)
        a, ap = _c(pa, np.int64)
        b, bp = _c(pb, np.int64)
        ww, wp = _c(w, np.float64)
        loss = ctypes.c_double()
        g = np.zeros(SURR_NPARAM, np.float32)
        rc = lib().w1_surrogate_grad(self.ctx._h, self._h, arr, len(ds), ap, bp, wp, a.size,
                                     INPUT_DEVICE if dev else 0, _stream_of(dev), ctypes.byref(loss),
                                     g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        if rc != 0:
            raise W1Error(rc, "w1_surrogate_grad")
        return loss.value, g

    def train(self, ds, pa, pb, w, epochs=10, batch_pairs=256, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8,
              seed=0) -> np.ndarray:
        """Adam training on the device; returns the mean loss of each epoch."""
        keep = []
        arr, dev = _pd_list(ds, keep)
        a, ap = _c(pa, np.int64)
        b, bp = _c(pb, np.int64)
        ww, wp = _c(w, np.float64)
        tp = _TrainParams(int(epochs), int(batch_pairs), lr, beta1, beta2, adam_eps, ctypes.c_uint64(seed))
        losses = np.zeros(max(int(epochs), 1))
        rc = lib().w1_surrogate_train(self.ctx._h, self._h, arr, len(ds), ap, bp, wp, a.size, ctypes.byref(tp),
                                      INPUT_DEVICE if dev else 0, _stream_of(dev),
                                      losses.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        if rc != 0:
            raise W1Error(rc, "w1_surrogate_train")
        return losses[:int(epochs)]


@dataclass
class NNResult:
    nn: np.ndarray
    w1: np.ndarray
    verifications: np.ndarray
    stats: dict


class NNIndex:
    """1-NN index over database diagrams (device copy, dual-bound sums and,
    with a surrogate, embeddings)."""

    def __init__(self, ctx: Context, db, surrogate: Surrogate | None = None):
        keep = []
        arr, dev = _pd_list(db, keep)
        h = ctypes.c_void_p()
        rc = lib().w1_nn_build(ctx._h, surrogate._h if surrogate else None, arr, len(db),
                               INPUT_DEVICE if dev else 0, _stream_of(dev), ctypes.byref(h))
        if rc != 0:
            raise W1Error(rc, "w1_nn_build")
        self._h, self.ctx, self.surrogate, self.m = h, ctx, surrogate, len(db)

    def close(self):
        if getattr(self, "_h", None):
            lib().w1_nn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self, qs, eps=0.1, mode="surrogate", seed_k=0, keep=0) -> NNResult:
        """keep / seed_k: the candidates kept after RWMD and after the s = 1
        stage (modes "sparse" and "pipeline"); seed_k also sets the
        surrogate's seeds.  0 selects the library's defaults."""
        hold = []
        arr, dev = _pd_list(qs, hold)
        nq = len(qs)
        nn = np.zeros(nq, np.int64)
        w = np.zeros(nq, np.float64)
        ver = np.zeros(nq, np.int64)
        st = _NNStats()
        prm = _NNParams(float(eps), NN_MODES[mode], int(seed_k), int(keep), 0)
        sur = self.surrogate._h if (self.surrogate is not None and mode == "surrogate") else None
        rc = lib().w1_nn_query(self.ctx._h, self._h, sur, arr, nq, ctypes.byref(prm), INPUT_DEVICE if dev else 0,
                               _stream_of(dev), nn.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ver.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(st))
        if rc != 0:
            raise W1Error(rc, f"w1_nn_query (hip error {lib().w1_ctx_hip_error(self.ctx._h)})")
        return NNResult(nn, w, ver, {f: getattr(st, f) for f, _ in _NNStats._fields_})


def build():
    """Compile the HIP library (hipcc, gfx950)."""
    from .build import build as _b

    return _b(force=True)

"""Python binding of libsg2v (colour-coding tree counting on MI355X).

Argument marshalling only: every step of the count runs in the HIP kernels of
``libsg2v.so``.  PyTorch provides device memory and the current stream.  If
the library is missing the import of the native handle fails loudly; there is
no CPU fallback.

The functions mirror the C ABI of ``include/sg2v.h``:
``Plan`` (sg2v_plan_*), ``Graph`` (sg2v_graph_*), ``Colorings``
(sg2v_color), ``count`` (sg2v_count), ``count_batch``, ``count_grad`` and
``debug_table``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsg2v.so")

FP64 = 0
FP32S = 1
U64 = 2
MODES = {"fp64": FP64, "fp32s": FP32S, "u64": U64}

GRAPH_DEVICE_PTRS = 1
GRAPH_VALIDATE = 2
GRAPH_RELABEL = 4

_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOTTREE", -3: "ERANGE", -4: "ENOMEM", -5: "EGRAPH",
           -6: "EDEVICE"}

_lib = None


class Sg2vError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {msg}")


class PlanInfo(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int32), ("k", ctypes.c_int32), ("n_nodes", ctypes.c_int32),
                ("n_splits", ctypes.c_int32), ("n_passive", ctypes.c_int32),
                ("root_node", ctypes.c_int32), ("alpha", ctypes.c_int64),
                ("colorful_prob", ctypes.c_double), ("spmm_columns", ctypes.c_int64),
                ("pairs_per_vertex", ctypes.c_int64), ("widest_table", ctypes.c_int64),
                ("n_templates", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("bytes_per_vertex_fp32", ctypes.c_int64), ("bytes_per_vertex_fp64", ctypes.c_int64)]


class EstimateResult(ctypes.Structure):
    _fields_ = [("n_colorings", ctypes.c_int64), ("n_bound", ctypes.c_int64),
                ("group_size", ctypes.c_int64), ("groups", ctypes.c_int32),
                ("stopped_early", ctypes.c_int32), ("capped", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("mean", ctypes.c_double),
                ("median_of_means", ctypes.c_double), ("variance", ctypes.c_double),
                ("std_error", ctypes.c_double), ("ci_low", ctypes.c_double),
                ("ci_high", ctypes.c_double), ("rel_half_width", ctypes.c_double)]


class NodeInfo(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int32), ("active", ctypes.c_int32), ("passive", ctypes.c_int32),
                ("vertex", ctypes.c_int32), ("n_kept", ctypes.c_int32),
                ("is_passive", ctypes.c_int32), ("columns", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("spmm_width", ctypes.c_int32), ("ema_rows", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("budget_bytes", ctypes.c_int64), ("xsplit_group", ctypes.c_int32),
                ("launch_chunks", ctypes.c_int32), ("xsplit_min", ctypes.c_int32)]


EXPORTS = ["sg2v_last_error", "sg2v_version", "sg2v_plan_create", "sg2v_plan_destroy",
           "sg2v_template_reroot",
           "sg2v_plan_info", "sg2v_plan_node", "sg2v_plan_pairs", "sg2v_graph_create", "sg2v_graph_destroy",
           "sg2v_color", "sg2v_colorings_destroy", "sg2v_colorings_download", "sg2v_count",
           "sg2v_count_batch", "sg2v_count_grad", "sg2v_debug_table", "sg2v_set_tuning",
           "sg2v_get_tuning", "sg2v_profile_start", "sg2v_profile_stop", "sg2v_autotune",
           "sg2v_count_noalloc", "sg2v_plan_create_multi", "sg2v_trees", "sg2v_count_multi",
           "sg2v_estimate"]

KERNEL_KINDS = ["color", "hist", "spmm", "spmm_combine", "ema_general", "ema_single", "root"]


class ProfEntry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("launches", ctypes.c_int32), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("work", ctypes.c_double)]


def lib():
    """Load libsg2v.so (raises if it has not been built).

    torch is imported first: its HIP runtime carries the same soname as the
    one libsg2v.so was linked against, so the dynamic loader binds libsg2v.so
    to torch's runtime and torch's streams and device pointers are valid in
    the library.  Loading libsg2v.so first would pull a second HIP runtime
    into the process."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with "
                              "`python -m paper_2009_11665_amd.build`")
        import torch  # noqa: F401  (binds the HIP runtime, see above)
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                 ctypes.c_uint64)
        L.sg2v_last_error.restype = ctypes.c_char_p
        L.sg2v_version.restype = ctypes.c_char_p
        L.sg2v_plan_create.argtypes = [P, i32, i32, ctypes.POINTER(P)]
        L.sg2v_plan_destroy.argtypes = [P]
        L.sg2v_template_reroot.argtypes = [P, i32, i32, ctypes.c_double, P, P]
        L.sg2v_plan_destroy.restype = None
        L.sg2v_plan_info.argtypes = [P, ctypes.POINTER(PlanInfo)]
        L.sg2v_plan_node.argtypes = [P, i32, ctypes.POINTER(NodeInfo)]
        L.sg2v_plan_pairs.argtypes = [P, i32, P]
        L.sg2v_graph_create.argtypes = [i64, i64, P, P, P, u32, P, ctypes.POINTER(P)]
        L.sg2v_graph_destroy.argtypes = [P]
        L.sg2v_graph_destroy.restype = None
        L.sg2v_color.argtypes = [P, i32, u64, i32, i32, P, ctypes.POINTER(P)]
        L.sg2v_colorings_destroy.argtypes = [P]
        L.sg2v_colorings_destroy.restype = None
        L.sg2v_colorings_download.argtypes = [P, P, P]
        L.sg2v_count.argtypes = [P, P, P, i32, P, P, P, P, P, P]
        L.sg2v_count_noalloc.argtypes = [P, P, P, i32, P, P, P, P, P, P]
        L.sg2v_plan_create_multi.argtypes = [P, P, i32, i32, ctypes.POINTER(P)]
        L.sg2v_trees.argtypes = [i32, i64, P, ctypes.POINTER(ctypes.c_int64)]
        L.sg2v_count_multi.argtypes = [P, P, P, i32, P, P, P, P, P, P, P]
        L.sg2v_estimate.argtypes = [P, P, u64, ctypes.c_double, ctypes.c_double, i32, i64, u32, P,
                                    ctypes.POINTER(EstimateResult), P]
        L.sg2v_count_batch.argtypes = [P, i32, P, u64, i32, i32, P, P, P]
        L.sg2v_count_grad.argtypes = [P, P, P, i32, P, P, P]
        L.sg2v_debug_table.argtypes = [P, P, P, i32, i32, i32, i32, P, P]
        L.sg2v_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
        L.sg2v_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
        L.sg2v_autotune.argtypes = [P, P, i32, i32, P, ctypes.POINTER(Tuning)]
        L.sg2v_profile_start.argtypes = []
        L.sg2v_profile_stop.argtypes = [ctypes.POINTER(ProfEntry)]
        for name in EXPORTS:
            f = getattr(L, name)
            if f.restype is ctypes.c_int:  # default restype: status codes
                f.restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(st: int, where: str):
    if st != 0:
        raise Sg2vError(st, where, lib().sg2v_last_error().decode())


def _stream(stream=None):
    """hipStream_t of `stream`, else of torch's current stream, else NULL."""
    import torch
    if stream is None:
        if not torch.cuda.is_available():
            return None
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(a.data_ptr())  # torch tensor


def version() -> str:
    return lib().sg2v_version().decode()


def reroot(parent: Sequence[int], k: Optional[int] = None, spmm_weight: float = 0.5):
    """Isomorphic template with a cheaper decomposition (sg2v_template_reroot).
    Returns (parent_out, perm) as lists; counts and estimates are unchanged."""
    par = np.ascontiguousarray(parent, np.int32)
    t = len(par)
    out = np.zeros(t, np.int32)
    perm = np.zeros(t, np.int32)
    _check(lib().sg2v_template_reroot(_ptr(par), t, t if k is None else int(k), float(spmm_weight),
                                      _ptr(out), _ptr(perm)), "sg2v_template_reroot")
    return [int(x) for x in out], [int(x) for x in perm]


def trees(t: int):
    """The non-isomorphic trees with t vertices as parent arrays (sg2v_trees)."""
    n = ctypes.c_int64(0)
    _check(lib().sg2v_trees(int(t), 0, None, ctypes.byref(n)), "sg2v_trees")
    out = np.zeros((n.value, int(t)), np.int32)
    _check(lib().sg2v_trees(int(t), n.value, _ptr(out), ctypes.byref(n)), "sg2v_trees")
    return [[int(x) for x in row] for row in out]


class Plan:
    """sg2v_plan: template partition, split tables, alpha and P."""

    def __init__(self, parent: Sequence[int], k: Optional[int] = None):
        par = np.ascontiguousarray(parent, np.int32)
        self.parent = [int(x) for x in par]
        self.t = len(par)
        self.k = self.t if k is None else int(k)
        self.n_templates = 1
        h = ctypes.c_void_p()
        _check(lib().sg2v_plan_create(_ptr(par), self.t, self.k, ctypes.byref(h)),
               "sg2v_plan_create")
        self.h = h

    @classmethod
    def multi(cls, parents: Sequence[Sequence[int]], k: Optional[int] = None):
        """One plan of several templates sharing isomorphic sub-templates
        (sg2v_plan_create_multi); count it with count_multi()."""
        sizes = np.ascontiguousarray([len(p) for p in parents], np.int32)
        flat = np.ascontiguousarray([int(x) for p in parents for x in p], np.int32)
        self = cls.__new__(cls)
        self.parent = [int(x) for x in parents[0]]
        self.parents = [[int(x) for x in p] for p in parents]
        self.t = len(parents[0])
        self.k = max(len(p) for p in parents) if k is None else int(k)
        self.n_templates = len(parents)
        h = ctypes.c_void_p()
        _check(lib().sg2v_plan_create_multi(_ptr(flat), _ptr(sizes), len(parents), self.k,
                                            ctypes.byref(h)), "sg2v_plan_create_multi")
        self.h = h
        return self

    def info(self) -> PlanInfo:
        i = PlanInfo()
        _check(lib().sg2v_plan_info(self.h, ctypes.byref(i)), "sg2v_plan_info")
        return i

    def node(self, idx: int) -> NodeInfo:
        i = NodeInfo()
        _check(lib().sg2v_plan_node(self.h, idx, ctypes.byref(i)), "sg2v_plan_node")
        return i

    def nodes(self):
        return [self.node(i) for i in range(self.info().n_nodes)]

    def pairs(self, idx: int) -> np.ndarray:
        """Split table of node idx: int32 [C(k,|T_s|), C(|T_s|,|T_a|), 2]."""
        from math import comb
        nd = self.node(idx)
        na = self.node(nd.active).size
        out = np.zeros((nd.columns, comb(nd.size, na), 2), np.int32)
        _check(lib().sg2v_plan_pairs(self.h, idx, _ptr(out)), "sg2v_plan_pairs")
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sg2v_plan_destroy(self.h)
            self.h = None


class Graph:
    """sg2v_graph: symmetric CSR registered on the current device.

    Pass numpy arrays (copied to the device) or torch device tensors
    (borrowed: the Graph keeps references to them)."""

    def __init__(self, n: int, row_ptr, col_idx, w=None, validate: bool = False, stream=None,
                 relabel: bool = False):
        self.n = int(n)
        flags = (GRAPH_VALIDATE if validate else 0) | (GRAPH_RELABEL if relabel else 0)
        self._keep = None
        if isinstance(row_ptr, np.ndarray):
            rp = np.ascontiguousarray(row_ptr, np.int64)
            ci = np.ascontiguousarray(col_idx, np.int32)
            wv = None if w is None else np.ascontiguousarray(w, np.float32)
            nnz = int(rp[-1])
        else:
            import torch
            rp = row_ptr.contiguous().to(torch.int64)
            ci = col_idx.contiguous().to(torch.int32)
            wv = None if w is None else w.contiguous().to(torch.float32)
            nnz = int(ci.numel())
            flags |= GRAPH_DEVICE_PTRS
            self._keep = (rp, ci, wv)
        self.nnz = nnz
        self.weighted = w is not None
        h = ctypes.c_void_p()
        _check(lib().sg2v_graph_create(self.n, nnz, _ptr(rp), _ptr(ci), _ptr(wv), flags,
                                       _stream(stream), ctypes.byref(h)), "sg2v_graph_create")
        self.h = h

    @classmethod
    def from_csr(cls, g, validate: bool = False, weighted: Optional[bool] = None, stream=None,
                 relabel: bool = False):
        """From any object with n, row_ptr, col_idx, w (numpy).  relabel: store
        the vertices renumbered by decreasing degree (SG2V_GRAPH_RELABEL)."""
        use_w = g.w if (weighted is None or weighted) else None
        return cls(g.n, g.row_ptr, g.col_idx, use_w, validate=validate, stream=stream,
                   relabel=relabel)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sg2v_graph_destroy(self.h)
            self.h = None


class Colorings:
    """sg2v_colorings: n_colorings random colourings on the device."""

    def __init__(self, graph: Graph, k: int, seed: int, n_colorings: int, first: int = 0,
                 stream=None):
        self.graph = graph
        self.k, self.seed, self.count, self.first = int(k), int(seed), int(n_colorings), int(first)
        h = ctypes.c_void_p()
        _check(lib().sg2v_color(graph.h, self.k, self.seed, self.first, self.count,
                                _stream(stream), ctypes.byref(h)), "sg2v_color")
        self.h = h

    def download(self, stream=None) -> np.ndarray:
        out = np.empty((self.count, self.graph.n), np.uint8)
        _check(lib().sg2v_colorings_download(self.h, _ptr(out), _stream(stream)),
               "sg2v_colorings_download")
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.sg2v_colorings_destroy(self.h)
            self.h = None


def count(plan: Plan, graph: Graph, col: Colorings, mode="fp32s", stream=None):
    """Colourful counts and estimates per colouring (sg2v_count).

    Returns dict(colorful=float64[n], colorful_u64=uint64[n], estimate=float64[n],
    mean_estimate=float, overflow=bool)."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    n = col.count
    cf = np.zeros(n, np.float64)
    cu = np.zeros(n, np.uint64)
    est = np.zeros(n, np.float64)
    mean = ctypes.c_double(0)
    ovf = ctypes.c_int32(0)
    _check(lib().sg2v_count(plan.h, graph.h, col.h, m, _stream(stream), _ptr(cf), _ptr(cu),
                            _ptr(est), ctypes.byref(mean), ctypes.byref(ovf)), "sg2v_count")
    return dict(colorful=cf, colorful_u64=cu, estimate=est, mean_estimate=mean.value,
                overflow=bool(ovf.value))


def count_multi(plan: Plan, graph: Graph, col: Colorings, mode="fp32s", stream=None):
    """Every template of a plan (sg2v_count_multi).  Returns dict(colorful,
    colorful_u64, estimate: [n_templates, n_colorings]; mean_estimate,
    frequency: [n_templates]; overflow)."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    r, n = plan.n_templates, col.count
    cf = np.zeros((r, n), np.float64)
    cu = np.zeros((r, n), np.uint64)
    est = np.zeros((r, n), np.float64)
    mean = np.zeros(r, np.float64)
    freq = np.zeros(r, np.float64)
    ovf = ctypes.c_int32(0)
    _check(lib().sg2v_count_multi(plan.h, graph.h, col.h, m, _stream(stream), _ptr(cf), _ptr(cu),
                                  _ptr(est), _ptr(mean), _ptr(freq), ctypes.byref(ovf)),
           "sg2v_count_multi")
    return dict(colorful=cf, colorful_u64=cu, estimate=est, mean_estimate=mean, frequency=freq,
                overflow=bool(ovf.value))


ESTIMATE_ADAPTIVE = 1


def estimate(plan: Plan, graph: Graph, seed: int, eps: float, delta: float, mode="fp64",
             max_colorings: int = 0, adaptive: bool = False, stream=None):
    """(eps, delta) estimate of the number of copies (sg2v_estimate).
    Returns (EstimateResult, trace of running means per group)."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    out = EstimateResult()
    groups = max(1, int(np.ceil(8.0 * np.log(1.0 / delta))))
    trace = np.zeros(groups, np.float64)
    _check(lib().sg2v_estimate(plan.h, graph.h, int(seed), float(eps), float(delta), m,
                               int(max_colorings), ESTIMATE_ADAPTIVE if adaptive else 0,
                               _stream(stream), ctypes.byref(out), _ptr(trace)), "sg2v_estimate")
    return out, trace[:out.groups]


def count_noalloc(plan: Plan, graph: Graph, col: Colorings, mode="fp32s", stream=None):
    """As count(), through sg2v_count_noalloc: no device allocation; every
    buffer comes from the library's fixed scratch area
    (NOALLOC_SCRATCH_BYTES per device).  The plan must have been counted once
    with count() on this device."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    n = col.count
    cf = np.zeros(n, np.float64)
    cu = np.zeros(n, np.uint64)
    est = np.zeros(n, np.float64)
    mean = ctypes.c_double(0)
    ovf = ctypes.c_int32(0)
    _check(lib().sg2v_count_noalloc(plan.h, graph.h, col.h, m, _stream(stream), _ptr(cf), _ptr(cu),
                                    _ptr(est), ctypes.byref(mean), ctypes.byref(ovf)),
           "sg2v_count_noalloc")
    return dict(colorful=cf, colorful_u64=cu, estimate=est, mean_estimate=mean.value,
                overflow=bool(ovf.value))


NOALLOC_SCRATCH_BYTES = 64 << 20


def count_batch(plans: Sequence[Plan], graph: Graph, seed: int, n_colorings: int, mode="fp32s",
                stream=None):
    """Several templates x n_colorings colourings (sg2v_count_batch).
    Returns (colorful, estimate) arrays of shape [n_plans, n_colorings]."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    arr = (ctypes.c_void_p * len(plans))(*[p.h.value for p in plans])
    cf = np.zeros((len(plans), n_colorings), np.float64)
    est = np.zeros((len(plans), n_colorings), np.float64)
    _check(lib().sg2v_count_batch(arr, len(plans), graph.h, seed, n_colorings, m, _stream(stream),
                                  _ptr(cf), _ptr(est)), "sg2v_count_batch")
    return cf, est


def debug_table(plan: Plan, graph: Graph, col: Colorings, node: int, kind: int = 0,
                which: int = 0, mode="fp64", stream=None) -> np.ndarray:
    """Table of `node` (kind 0: M_s, kind 1: B = A M_s) for colouring `which`,
    as float64 (uint64 in U64 mode), shape [n, C(k, |T_s|)]."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    ni = plan.node(node)
    cols = plan.k if (ni.size == 1) else ni.columns
    out = np.zeros((graph.n, cols), np.uint64 if m == U64 else np.float64)
    _check(lib().sg2v_debug_table(plan.h, graph.h, col.h, m, which, node, kind, _ptr(out),
                                  _stream(stream)), "sg2v_debug_table")
    return out


def count_grad(plan: Plan, graph: Graph, col: Colorings, grad_colorful, mode="fp64",
               stream=None):
    """d(sum_j grad_colorful[j] * colorful[j]) / d(A_G(i,j)) per directed CSR
    entry, as a torch tensor on the current device (sg2v_count_grad)."""
    import torch
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    gc = np.ascontiguousarray(grad_colorful, np.float64)
    out = torch.empty(graph.nnz, dtype=torch.float64, device="cuda")  # FP64 in both modes
    _check(lib().sg2v_count_grad(plan.h, graph.h, col.h, m, _ptr(gc), _ptr(out), _stream(stream)),
           "sg2v_count_grad")
    return out


TUNE_NO_COLOR_SKIP = 1
TUNE_NO_COLOR_EMA = 2
TUNE_SPMM_UNROLL4 = 4
TUNE_SPMM_UNROLL8 = 128
TUNE_NO_XSPLIT = 8
TUNE_FORCE_XSPLIT = 16
TUNE_XSPLIT = 32
TUNE_ROOT_ROWS = 64
TUNE_ROOT_THREAD = 256
TUNE_BATCH_SERIAL = 512
TUNE_SPMM_PANEL = 1024
TUNE_GRAD_RECOMPUTE = 2048
TUNE_BATCH_PERSISTENT = 4096


def set_tuning(spmm_width: int = 0, ema_rows: int = 0, batch: int = 0, budget_bytes: int = 0,
               flags: int = 0, xsplit_group: int = 0, launch_chunks: int = 0, xsplit_min: int = 0):
    t = Tuning(spmm_width, ema_rows, batch, flags, budget_bytes, xsplit_group, launch_chunks,
               xsplit_min)
    _check(lib().sg2v_set_tuning(ctypes.byref(t)), "sg2v_set_tuning")


def restore_tuning(t: Tuning):
    """Install a Tuning returned by get_tuning() (or autotune())."""
    _check(lib().sg2v_set_tuning(ctypes.byref(t)), "sg2v_set_tuning")


class tuned:
    """Context manager: ``with tuned(flags=..., spmm_width=...):`` installs
    the settings and restores the previous ones on exit."""

    def __init__(self, **kw):
        self.kw = kw

    def __enter__(self):
        self.old = get_tuning()
        set_tuning(**self.kw)
        return self

    def __exit__(self, *exc):
        restore_tuning(self.old)
        return False


def get_tuning() -> Tuning:
    t = Tuning()
    _check(lib().sg2v_get_tuning(ctypes.byref(t)), "sg2v_get_tuning")
    return t


def profile_start():
    """Start bracketing every kernel launch with HIP events."""
    _check(lib().sg2v_profile_start(), "sg2v_profile_start")


def profile_stop():
    """Stop timing; returns {kind: dict(launches, ms, bytes, work)}."""
    arr = (ProfEntry * len(KERNEL_KINDS))()
    _check(lib().sg2v_profile_stop(arr), "sg2v_profile_stop")
    return {KERNEL_KINDS[e.kind]: dict(launches=e.launches, ms=e.ms, bytes=e.bytes, work=e.work)
            for e in arr}


class SubgraphCount:
    """Differentiable colourful count: ``SubgraphCount.apply(w, plan, row_ptr,
    col_idx, seed, n_colorings, mode="fp64")`` returns the colourful count of
    each colouring (float64 [n_colorings]) of the graph whose CSR entries carry
    the weights ``w`` (device tensor [nnz]); its backward gives d/dw per
    directed entry via sg2v_count_grad.  mode "fp64" or "fp32s" applies to the
    forward and the adjoint."""

    _fn = None

    @classmethod
    def apply(cls, w, plan, row_ptr, col_idx, seed, n_colorings, mode="fp64"):
        if cls._fn is None:
            import torch

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(ctx, w, plan, row_ptr, col_idx, seed, n_colorings, mode):
                    n = row_ptr.numel() - 1
                    g = Graph(n, row_ptr, col_idx, w.detach())
                    c = Colorings(g, plan.k, seed, n_colorings)
                    r = count(plan, g, c, mode)
                    ctx.keep = (g, c, plan, mode)
                    return torch.as_tensor(r["colorful"], dtype=torch.float64, device=w.device)

                @staticmethod
                def backward(ctx, grad_out):
                    g, c, plan, mode = ctx.keep
                    gw = count_grad(plan, g, c, grad_out.detach().double().cpu().numpy(), mode)
                    return gw.to(w_dtype(ctx)), None, None, None, None, None, None

            def w_dtype(ctx):
                return ctx.keep[0]._keep[2].dtype

            cls._fn = _F
        return cls._fn.apply(w, plan, row_ptr, col_idx, seed, n_colorings, mode)


def autotune(plan: Plan, graph: Graph, mode="fp32s", n_colorings: int = 1, stream=None) -> Tuning:
    """Time candidate settings for this template and graph and install the
    fastest (sg2v_autotune)."""
    m = MODES[mode] if isinstance(mode, str) else int(mode)
    t = Tuning()
    _check(lib().sg2v_autotune(plan.h, graph.h, m, n_colorings, _stream(stream), ctypes.byref(t)),
           "sg2v_autotune")
    return t

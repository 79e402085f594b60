"""ORACLE -- test infrastructure only.

ctypes wrapper around ``oracle.c``, the plain CPU reference for
colour-coding tree counting.  Only ``tests/``, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path
(``paper_2009_11665_amd``) never does, and the two share no code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

FP64 = 0
U64 = 1
CUT_LAST = 0
CUT_FIRST = 1


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", src,
                               "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, u64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32
        lib.orc_splitmix64_next.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        lib.orc_splitmix64_next.restype = u64
        lib.orc_mix64.argtypes = [u64]
        lib.orc_mix64.restype = u64
        lib.orc_colors.argtypes = [i64, i32, u64, i32, P]
        lib.orc_count.argtypes = [i64, P, P, P, P, i32, i32, P, i32, i32, i32, P, P, P]
        lib.orc_node_table.argtypes = [i64, P, P, P, P, i32, i32, P, i32, i32, i32, i32, P, P, P]
        lib.orc_neighbour_sum.argtypes = [i64, P, P, P, i64, i32, P, P, P, P, P]
        lib.orc_colorful_probability.argtypes = [i32, i32]
        lib.orc_colorful_probability.restype = ctypes.c_double
        lib.orc_brute.argtypes = [i64, P, P, P, P, i32, P, i64, P, P, P]
        lib.orc_automorphisms.argtypes = [P, i32]
        lib.orc_automorphisms.restype = i64
        lib.orc_grad.argtypes = [i64, P, P, P, P, i32, i32, P, i32, P, P]
        lib.orc_num_threads.restype = ctypes.c_int
        for f in (lib.orc_colors, lib.orc_count, lib.orc_node_table, lib.orc_neighbour_sum,
                  lib.orc_brute, lib.orc_grad):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _graph_args(g):
    rp = np.ascontiguousarray(g.row_ptr, np.int64)
    ci = np.ascontiguousarray(g.col_idx, np.int32)
    return rp, ci


def _weights(g, weights):
    w = weights if weights is not None else g.w
    return None if w is None else np.ascontiguousarray(w, np.float64)


def _parent(parent: Sequence[int]):
    return np.ascontiguousarray(parent, np.int32)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def splitmix64_sequence(seed: int, count: int):
    st = ctypes.c_uint64(seed)
    return [int(_load().orc_splitmix64_next(ctypes.byref(st))) for _ in range(count)]


def colors(n: int, k: int, seed: int, j: int) -> np.ndarray:
    out = np.empty(n, np.uint8)
    rc = _load().orc_colors(n, k, seed, j, _p(out))
    if rc:
        raise OracleError(f"orc_colors: {rc}")
    return out


def colorful_probability(t: int, k: int) -> float:
    return float(_load().orc_colorful_probability(t, k))


def automorphisms(parent: Sequence[int]) -> int:
    a = _parent(parent)
    r = int(_load().orc_automorphisms(_p(a), len(a)))
    if r < 0:
        raise OracleError("orc_automorphisms: invalid template")
    return r


def count(g, parent, k: int, col: np.ndarray, mode: int = FP64, alg2: bool = False,
          cut: int = CUT_LAST, weights: Optional[np.ndarray] = None):
    """Colourful count of one colouring.  Returns (float, uint64, overflow)."""
    rp, ci = _graph_args(g)
    w = _weights(g, weights) if mode == FP64 else None
    par = _parent(parent)
    col = np.ascontiguousarray(col, np.uint8)
    f = ctypes.c_double(0)
    u = ctypes.c_uint64(0)
    ov = ctypes.c_int32(0)
    rc = _load().orc_count(g.n, _p(rp), _p(ci), _p(w), _p(par), len(par), k, _p(col), mode,
                           int(alg2), cut, ctypes.byref(f), ctypes.byref(u), ctypes.byref(ov))
    if rc:
        raise OracleError(f"orc_count: {rc}")
    return f.value, u.value, bool(ov.value)


def estimate(colorful: float, parent, k: int) -> float:
    """finalCount of Alg. 1: colourful / (P alpha)."""
    return colorful / (colorful_probability(len(parent), k) * automorphisms(parent))


def node_table(g, parent, k: int, col: np.ndarray, v: int, nkept: int, mode: int = FP64,
               cut: int = CUT_LAST, weights=None) -> np.ndarray:
    """Count table (n x C(k, size)) of sub-template (v, nkept children)."""
    from math import comb
    rp, ci = _graph_args(g)
    w = _weights(g, weights) if mode == FP64 else None
    par = _parent(parent)
    col = np.ascontiguousarray(col, np.uint8)
    # size of the sub-template, to size the output
    t = len(par)
    ch = [[] for _ in range(t)]
    for x in range(t):
        if par[x] >= 0:
            ch[par[x]].append(x)

    def sub(x):
        return 1 + sum(sub(c) for c in ch[x])

    kept = ch[v][:nkept] if cut == CUT_LAST else ch[v][len(ch[v]) - nkept:]
    size = 1 + sum(sub(c) for c in kept)
    nc = comb(k, size)
    out = np.zeros((g.n, nc), np.uint64 if mode == U64 else np.float64)
    ncols = ctypes.c_int64(0)
    rc = _load().orc_node_table(g.n, _p(rp), _p(ci), _p(w), _p(par), t, k, _p(col), mode, cut, v,
                                nkept, None if mode == U64 else _p(out),
                                _p(out) if mode == U64 else None, ctypes.byref(ncols))
    if rc:
        raise OracleError(f"orc_node_table: {rc}")
    assert ncols.value == nc
    return out


def neighbour_sum(g, M: np.ndarray, mode: int = FP64, weights=None) -> np.ndarray:
    """B = A_G M."""
    rp, ci = _graph_args(g)
    w = _weights(g, weights) if mode == FP64 else None
    M = np.ascontiguousarray(M, np.uint64 if mode == U64 else np.float64)
    B = np.empty_like(M)
    ov = ctypes.c_int32(0)
    rc = _load().orc_neighbour_sum(g.n, _p(rp), _p(ci), _p(w), M.shape[1], mode,
                                   None if mode == U64 else _p(M), _p(M) if mode == U64 else None,
                                   None if mode == U64 else _p(B), _p(B) if mode == U64 else None,
                                   ctypes.byref(ov))
    if rc:
        raise OracleError(f"orc_neighbour_sum: {rc}")
    return B


def brute(g, parent, col: Optional[np.ndarray] = None, weights=None, grad: bool = False,
          limit: int = 0):
    """Brute-force enumeration.  col=None: injective maps; else colourful maps.
    Returns (weighted total, map count, per-entry grad or None)."""
    rp, ci = _graph_args(g)
    w = _weights(g, weights)
    par = _parent(parent)
    colv = None if col is None else np.ascontiguousarray(col, np.uint8)
    tot = ctypes.c_double(0)
    cnt = ctypes.c_uint64(0)
    gr = np.zeros(g.nnz, np.float64) if grad else None
    rc = _load().orc_brute(g.n, _p(rp), _p(ci), _p(w), _p(par), len(par), _p(colv), limit,
                           ctypes.byref(tot), ctypes.byref(cnt), _p(gr))
    if rc < 0:
        raise OracleError(f"orc_brute: {rc}")
    if rc == 1:
        raise OracleError("orc_brute: enumeration limit reached")
    return tot.value, cnt.value, gr


def grad(g, parent, k: int, col: np.ndarray, weights=None, cut: int = CUT_LAST):
    """Reverse-mode d(colourful count)/d(w_e) per directed entry.  Returns (f, grad)."""
    rp, ci = _graph_args(g)
    w = _weights(g, weights)
    par = _parent(parent)
    col = np.ascontiguousarray(col, np.uint8)
    f = ctypes.c_double(0)
    gr = np.zeros(g.nnz, np.float64)
    rc = _load().orc_grad(g.n, _p(rp), _p(ci), _p(w), _p(par), len(par), k, _p(col), cut,
                          ctypes.byref(f), _p(gr))
    if rc:
        raise OracleError(f"orc_grad: {rc}")
    return f.value, gr


def fold_undirected(g, per_entry: np.ndarray) -> np.ndarray:
    """Sum the two directed entries of each undirected edge: out[e] for entry
    e = (i -> j) is per_entry[i->j] + per_entry[j->i]."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    cols = g.col_idx.astype(np.int64)
    key = rows * g.n + cols
    rkey = cols * g.n + rows
    order = np.argsort(key)
    pos = order[np.searchsorted(key[order], rkey)]
    return per_entry + per_entry[pos]

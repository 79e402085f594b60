"""Seeded synthetic graphs shared by the oracle tests, the GPU tests and the
benchmark.  Input synthesis only: nothing here computes any part of the
colour-coding count.

The paper's datasets (its Table 2: PPI networks, Graph500, Miami, Orkut, NYC,
RMAT-1M) are not available; the seeded generators below stand in for them
with the same vertex counts, edge counts and degree skew.

Graphs are returned as symmetric CSR: int64 ``row_ptr[n+1]``, int32
``col_idx[nnz]`` (sorted within each row, no self-loops, no duplicates) and an
optional float32 ``w[nnz]`` holding one value per undirected edge on both of
its directed entries.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the generator library (gcc, OpenMP)."""
    src = os.path.join(_HERE, "gen.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", src,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, u64, i32, f64 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
        lib.gg_er.argtypes = [i64, i64, u64, P, P]
        lib.gg_rmat.argtypes = [i32, i64, f64, f64, f64, u64, i32, P, P]
        lib.gg_chung_lu.argtypes = [i64, i64, f64, u64, P, P, P]
        lib.gg_csr.argtypes = [i64, i64, P, P, P, P, P, P]
        lib.gg_edge_weights.argtypes = [i64, P, P, u64, f64, f64, P]
        lib.gg_permutation.argtypes = [i64, u64, P]
        for f in (lib.gg_er, lib.gg_rmat, lib.gg_chung_lu, lib.gg_csr, lib.gg_edge_weights,
                  lib.gg_permutation):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"graphgen.{what} failed with code {rc}")


def er_edges(n: int, m: int, seed: int):
    """m distinct uniform undirected non-loop edges on n vertices (u < v)."""
    eu = np.empty(m, np.int32)
    ev = np.empty(m, np.int32)
    _check(_load().gg_er(n, m, seed, _ptr(eu), _ptr(ev)), "er")
    return eu, ev


def rmat_edges(scale: int, m: int, a: float, b: float, c: float, seed: int, relabel: bool = True):
    """m distinct undirected non-loop RMAT edges on 2**scale vertices."""
    eu = np.empty(m, np.int32)
    ev = np.empty(m, np.int32)
    _check(_load().gg_rmat(scale, m, a, b, c, seed, int(relabel), _ptr(eu), _ptr(ev)), "rmat")
    return eu, ev


def chung_lu_edges(n: int, m: int, gamma: float, seed: int):
    """m distinct undirected non-loop Chung-Lu edges with power-law weights."""
    eu = np.empty(m, np.int32)
    ev = np.empty(m, np.int32)
    _check(_load().gg_chung_lu(n, m, gamma, seed, _ptr(eu), _ptr(ev), None), "chung_lu")
    return eu, ev


def edge_weights(eu: np.ndarray, ev: np.ndarray, seed: int, lo: float, hi: float) -> np.ndarray:
    w = np.empty(len(eu), np.float32)
    _check(_load().gg_edge_weights(len(eu), _ptr(np.ascontiguousarray(eu)),
                                   _ptr(np.ascontiguousarray(ev)), seed, lo, hi, _ptr(w)), "weights")
    return w


def permutation(n: int, seed: int) -> np.ndarray:
    p = np.empty(n, np.uint32)
    _check(_load().gg_permutation(n, seed, _ptr(p)), "permutation")
    return p


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray          # int64 [n+1]
    col_idx: np.ndarray          # int32 [nnz]
    w: Optional[np.ndarray]      # float32 [nnz] or None
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def csr(n: int, eu: np.ndarray, ev: np.ndarray, ew: Optional[np.ndarray] = None,
        weighted: bool = False, name: str = "") -> Graph:
    """Symmetric CSR with sorted rows from a list of distinct undirected edges."""
    eu = np.ascontiguousarray(eu, np.int32)
    ev = np.ascontiguousarray(ev, np.int32)
    m = len(eu)
    row_ptr = np.empty(n + 1, np.int64)
    col_idx = np.empty(2 * m, np.int32)
    w = np.empty(2 * m, np.float32) if (weighted or ew is not None) else None
    if ew is not None:
        ew = np.ascontiguousarray(ew, np.float32)
    _check(_load().gg_csr(n, m, _ptr(eu), _ptr(ev), _ptr(ew), _ptr(row_ptr), _ptr(col_idx),
                          _ptr(w)), "csr")
    return Graph(n, row_ptr, col_idx, w, name)


def from_edge_list(n: int, edges, weights=None, name: str = "") -> Graph:
    """CSR from a small Python edge list (tests).  Edges must be distinct, u != v."""
    if len(edges) == 0:
        return Graph(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32),
                     None if weights is None else np.zeros(0, np.float32), name)
    e = np.asarray(edges, np.int64)
    lo = np.minimum(e[:, 0], e[:, 1]).astype(np.int32)
    hi = np.maximum(e[:, 0], e[:, 1]).astype(np.int32)
    ew = None if weights is None else np.asarray(weights, np.float32)
    return csr(n, lo, hi, ew, name=name)


# --------------------------------------------------------------------------
# The five seeded workloads.  Template parent arrays and colour counts live
# with the workloads that use them, here, so that tests and the benchmark
# build exactly the same inputs.

BINTREE7 = [-1, 0, 0, 1, 1, 2, 2]
BINTREE15 = [-1] + [(i - 1) // 2 for i in range(1, 15)]
PATH5 = [-1, 0, 1, 2, 3]
PATH8 = [-1, 0, 1, 2, 3, 4, 5, 6]
CATERPILLAR10 = [-1, 0, 1, 2, 3, 4, 1, 2, 3, 4]

RMAT_ABC = (0.57, 0.19, 0.19)


def tiny_er(seed: int = 1) -> Graph:
    """Erdos-Renyi, n=1000, 4000 undirected edges (nnz 8000)."""
    eu, ev = er_edges(1000, 4000, seed)
    return csr(1000, eu, ev, name="er-n1000-m4000")


def rmat(scale: int, m_undirected: int, seed: int, relabel: bool = True) -> Graph:
    eu, ev = rmat_edges(scale, m_undirected, *RMAT_ABC, seed=seed, relabel=relabel)
    return csr(1 << scale, eu, ev, name=f"rmat-s{scale}-m{m_undirected}")


def rmat16(seed: int = 2) -> Graph:
    """RMAT scale 16, 2**20 undirected edges (nnz 2,097,152)."""
    return rmat(16, 1 << 20, seed)


def rmat20(seed: int = 5) -> Graph:
    """RMAT scale 20, 100,000,000 undirected edges (nnz 200,000,000)."""
    return rmat(20, 100_000_000, seed)


def chung_lu(n: int, avg_deg: float, gamma: float, seed: int, weighted: bool = False,
             weight_range=(0.5, 1.5)) -> Graph:
    m = int(round(n * avg_deg / 2))
    eu, ev = chung_lu_edges(n, m, gamma, seed)
    ew = edge_weights(eu, ev, seed, *weight_range) if weighted else None
    return csr(n, eu, ev, ew, name=f"chunglu-n{n}-d{avg_deg:g}-g{gamma:g}" + ("-w" if weighted else ""))


def chung_lu_262k_weighted(seed: int = 3) -> Graph:
    """Chung-Lu, n=262,144, mean degree 16, gamma 2.1, weights U[0.5,1.5)."""
    return chung_lu(262_144, 16.0, 2.1, seed, weighted=True)


def chung_lu_500k(seed: int = 4) -> Graph:
    """Chung-Lu, n=500,000, mean degree 20, gamma 2.1."""
    return chung_lu(500_000, 20.0, 2.1, seed)

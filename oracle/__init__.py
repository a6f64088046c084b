"""The oracle: a plain, slow, obviously correct CPU implementation of what the
mining path computes.  TEST INFRASTRUCTURE ONLY: the product library and its
binding never import, link or call anything here; only tests, the smoke check
and the benchmark's CPU-baseline leg do.

* ``patterns``  - automorphisms, Algorithm 1, Theorem 2, Algorithms 2 and 3,
                  the analytic performance model, motif enumeration (Python).
* ``brute``     - brute force over k-subsets with isomorphism tests (Python).
* ``count_oracle.c`` - normalisation, degree reindex and the restricted
                  nested-loop enumeration in plain single-threaded C, loaded
                  here through ctypes.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from collections import namedtuple

import numpy as np

from . import patterns

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "count_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None

Graph = namedtuple("Graph", "n rowptr col new_of_old")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, no vector intrinsics)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_normalize.restype = ctypes.c_int64
        lib.oracle_normalize.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, P, P]
        lib.oracle_reindex.restype = None
        lib.oracle_reindex.argtypes = [ctypes.c_int32, P, P, P, P, P]
        lib.oracle_count.restype = ctypes.c_int
        lib.oracle_count.argtypes = [ctypes.c_int32, P, P, ctypes.c_int, P,
                                     ctypes.c_int, P, ctypes.c_int, P, P, P,
                                     ctypes.c_int64, P, P, P]
        lib.oracle_instrument.restype = ctypes.c_int
        lib.oracle_instrument.argtypes = [ctypes.c_int32, P, P, ctypes.c_int, P,
                                          ctypes.c_int, P, P, P, ctypes.c_int64,
                                          P, P, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


# ------------------------------------------------------------------ graphs


def normalize(src, dst, n):
    """Simple undirected graph (int64 rowptr, int32 col, sorted rows) from a
    raw edge list."""
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = src.shape[0]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(max(2 * m, 1), dtype=np.int32)
    nnz = lib.oracle_normalize(n, m, _ptr(src), _ptr(dst), _ptr(rowptr), _ptr(col))
    if nnz < 0:
        raise ValueError("edge endpoint out of range")
    return rowptr, col[:nnz].copy()


def reindex(rowptr, col):
    """Degree reindex: decreasing degree, ties by increasing old id."""
    lib = _load()
    n = rowptr.shape[0] - 1
    rowptr2 = np.zeros(n + 1, dtype=np.int64)
    col2 = np.zeros(max(col.shape[0], 1), dtype=np.int32)
    new_of_old = np.zeros(max(n, 1), dtype=np.int32)
    lib.oracle_reindex(n, _ptr(rowptr), _ptr(np.ascontiguousarray(col)),
                       _ptr(rowptr2), _ptr(col2), _ptr(new_of_old))
    return rowptr2, col2[:col.shape[0]].copy(), new_of_old[:n].copy()


def prepare(src, dst, n, reindex_by_degree: bool = True) -> Graph:
    rowptr, col = normalize(src, dst, n)
    if not reindex_by_degree:
        return Graph(n, rowptr, col, np.arange(n, dtype=np.int32))
    r2, c2, perm = reindex(rowptr, col)
    return Graph(n, r2, c2, perm)


def from_edge_tuple(edges, reindex_by_degree: bool = True) -> Graph:
    src, dst, n = edges
    return prepare(src, dst, n, reindex_by_degree)


def lo_end(g: Graph):
    """Per vertex, the number of neighbours with a smaller id."""
    out = np.zeros(g.n, dtype=np.int64)
    for v in range(g.n):
        row = g.col[g.rowptr[v]:g.rowptr[v + 1]]
        out[v] = int(np.searchsorted(row, v))
    return out


# --------------------------------------------------------------- counting


def oracle_schedule(adj):
    """The oracle's own schedule rule (deliberately not the explorer's pick):
    start at a pattern vertex of largest degree, then repeatedly append the
    unscheduled vertex with the most scheduled neighbours; ties go to the
    smallest label."""
    adj = patterns.as_adj(adj)
    k = len(adj)
    deg = [sum(r) for r in adj]
    first = max(range(k), key=lambda v: (deg[v], -v))
    sched = [first]
    while len(sched) < k:
        rest = [v for v in range(k) if v not in sched]
        nxt = max(rest, key=lambda v: (sum(adj[v][w] for w in sched), -v))
        sched.append(nxt)
    return tuple(sched)


def _u128(lo, hi):
    return int(lo.value) | (int(hi.value) << 64)


def count(g: Graph, adj, induced: bool = True, order=None,
          relations="alg1", roots=None, per_root: bool = False):
    """Exact count of pattern instances.

    relations: "alg1" (every relation of Algorithm 1: each instance once),
    "thm2" (one bound per position), "none" (every automorphic mapping), or
    an explicit list of (a, b) schedule-position pairs.
    roots: optional array of v0 values; with ``per_root`` the per-root counts
    are returned as well.  Returns a Python int (exact, up to 2^128)."""
    lib = _load()
    adj = patterns.as_adj(adj)
    k = len(adj)
    if order is None:
        order = oracle_schedule(adj)
    order = tuple(order)
    if relations == "alg1":
        rel = patterns.relations_as_positions(adj, order)
    elif relations == "thm2":
        b = patterns.reduced_bounds(adj, order)
        rel = [(b[i], i) for i in range(k) if b[i] >= 0]
    elif relations == "none":
        rel = []
    else:
        rel = list(relations)
    A = np.array([[adj[i][j] for j in range(k)] for i in range(k)], dtype=np.uint8).ravel()
    O = np.array(order, dtype=np.int8)
    RA = np.array([a for a, _ in rel] or [0], dtype=np.int8)
    RB = np.array([b for _, b in rel] or [0], dtype=np.int8)
    R = None if roots is None else np.ascontiguousarray(roots, dtype=np.int32)
    nr = 0 if R is None else R.shape[0]
    pr = np.zeros(max(nr, 1), dtype=np.uint64) if (per_root and R is not None) else None
    lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib.oracle_count(g.n, _ptr(g.rowptr), _ptr(g.col), k, _ptr(A),
                          int(bool(induced)), _ptr(O), len(rel), _ptr(RA), _ptr(RB),
                          _ptr(R), nr, ctypes.byref(lo), ctypes.byref(hi), _ptr(pr))
    if rc:
        raise ValueError(f"oracle_count failed with code {rc}")
    total = _u128(lo, hi)
    if per_root:
        return total, pr[:nr].copy()
    return total


def instrument(g: Graph, adj, induced, order, bound, roots=None):
    """(algorithmic bytes, count) of the schedule ``order`` restricted by the
    one-bound-per-position list ``bound``."""
    lib = _load()
    adj = patterns.as_adj(adj)
    k = len(adj)
    A = np.array([[adj[i][j] for j in range(k)] for i in range(k)], dtype=np.uint8).ravel()
    O = np.array(order, dtype=np.int8)
    B = np.array(bound, dtype=np.int8)
    R = None if roots is None else np.ascontiguousarray(roots, dtype=np.int32)
    nr = 0 if R is None else R.shape[0]
    blo, bhi, clo, chi = (ctypes.c_uint64() for _ in range(4))
    rc = lib.oracle_instrument(g.n, _ptr(g.rowptr), _ptr(g.col), k, _ptr(A),
                               int(bool(induced)), _ptr(O), _ptr(B), _ptr(R), nr,
                               ctypes.byref(blo), ctypes.byref(bhi),
                               ctypes.byref(clo), ctypes.byref(chi))
    if rc:
        raise ValueError(f"oracle_instrument failed with code {rc}")
    return _u128(blo, bhi), _u128(clo, chi)

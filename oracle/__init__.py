"""CPU oracle for per-vertex directed 3-, 4- and 5-motif counts.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_2201_11655_amd``): it has its own class table, its own graph
normalisation and its own enumeration, and it never imports the product package.

Contents
--------
* ``vdmc_oracle.c`` (plain C, pthreads): the class table from the definition of the
  motif index (Sec. 4.1, Fig. 1) by trying all k! relabellings; Wernicke's ESU
  enumeration of connected k-sets with per-vertex crediting (Sec. 4.2); a
  per-vertex mode that yields one row exactly.
* ``exhaustive.py`` (pure Python): the plain definition over all k-subsets, for
  tiny graphs, with its own canonicalisation.  It pins the C oracle.

Pins (tests/test_oracle_*.py): Fig. 1 (53 -> 30), the CSR example of Sec. 4.2, the
class counts 13/199/9364 and the labelled counts 54/3834/1027080 (known sequence
values; k = 5 is the extension Sec. 11 names), closed forms on cliques, transitive
tournaments, cycles and stars, brute force on tiny graphs (k = 5 keyed by minimal
index), the column-sum invariant and the G(n,p) expectation of Sec. 7, Eq. 4.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vdmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

NUM_CLASSES = {3: 13, 4: 199, 5: 9364}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64, i32, p = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        lib.oracle_class_table.argtypes = [i32, p, p, p]
        lib.oracle_class_table.restype = i32
        lib.oracle_count.argtypes = [i64, i64, p, p, i32, i32, p, p]
        lib.oracle_count.restype = i32
        lib.oracle_count_rows.argtypes = [i64, i64, p, p, i32, i32, p, i64, p]
        lib.oracle_count_rows.restype = i32
        lib.oracle_count_edges.argtypes = [i64, i64, p, p, i32, i32, i64, p, p, p]
        lib.oracle_count_edges.restype = i32
        lib.oracle_graph_size.argtypes = [i64, i64, p, p, p]
        lib.oracle_graph_size.restype = i32
        lib.oracle_graph_csr.argtypes = [i64, i64, p, p, p, p, p]
        lib.oracle_graph_csr.restype = i32
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def class_table(k: int):
    """Returns (canon[2^(k(k-1))], cls[2^(k(k-1))] (-1 = disconnected), class_codes[C])."""
    lib = _load()
    ncode = 1 << (k * (k - 1))
    canon = np.zeros(ncode, np.uint32)
    cls = np.zeros(ncode, np.int32)
    codes = np.zeros(ncode, np.uint32)
    nc = lib.oracle_class_table(k, _ptr(canon), _ptr(cls), _ptr(codes))
    if nc <= 0:
        raise RuntimeError("oracle_class_table failed")
    return canon, cls, codes[:nc].copy()


def _arcs(src, dst):
    return (np.ascontiguousarray(src, dtype=np.int32), np.ascontiguousarray(dst, dtype=np.int32))


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)


def count(n: int, src, dst, k: int, threads: int | None = None):
    """Per-vertex counts ``uint64[n][C]`` (row = vertex id, column = class id) and the
    per-class totals ``uint64[C]`` (each connected k-set once)."""
    lib = _load()
    s, d = _arcs(src, dst)
    C = NUM_CLASSES[k]
    out = np.zeros((max(n, 0), C), np.uint64)
    tot = np.zeros(C, np.uint64)
    rc = lib.oracle_count(int(n), int(s.shape[0]), _ptr(s), _ptr(d), int(k),
                          int(threads or default_threads()), _ptr(out), _ptr(tot))
    if rc != 0:
        raise ValueError(f"oracle_count failed with {rc}")
    return out, tot


def count_rows(n: int, src, dst, k: int, rows, threads: int | None = None):
    """The rows of the given vertices only: ``uint64[len(rows)][C]``."""
    lib = _load()
    s, d = _arcs(src, dst)
    r = np.ascontiguousarray(rows, dtype=np.int32)
    C = NUM_CLASSES[k]
    out = np.zeros((r.shape[0], C), np.uint64)
    rc = lib.oracle_count_rows(int(n), int(s.shape[0]), _ptr(s), _ptr(d), int(k),
                               int(threads or default_threads()), _ptr(r), int(r.shape[0]), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_count_rows failed with {rc}")
    return out


def undirected_classes(k: int) -> np.ndarray:
    """Class ids (of ``class_table``) whose every vertex pair carries both arcs, ascending.
    With every arc reciprocated, each connected k-set of G_U lands in exactly one of them,
    so they are the undirected classes (connected graphs on k vertices; the paper's
    undirected runs, Fig. 3 caption): 2 for k = 3, 6 for k = 4."""
    from . import exhaustive
    _, cls, _ = class_table(k)
    pairs = [(i, j) for i in range(k) for j in range(i + 1, k)]
    found = set()
    for mask in range(1 << len(pairs)):
        A = [[0] * k for _ in range(k)]
        for b, (i, j) in enumerate(pairs):
            if (mask >> b) & 1:
                A[i][j] = A[j][i] = 1
        c = int(cls[exhaustive.motif_index(A)])
        if c >= 0:
            found.add(c)
    return np.array(sorted(found), np.int64)


def count_undirected(n: int, src, dst, k: int, threads: int | None = None):
    """Per-vertex undirected counts ``uint64[n][U]`` and totals ``uint64[U]``: the directed
    count of the graph with every arc reciprocated (that graph is G_U), restricted to the
    ``undirected_classes`` columns (every other column is zero there)."""
    s, d = _arcs(src, dst)
    out, tot = count(n, np.concatenate([s, d]), np.concatenate([d, s]), k, threads)
    cols = undirected_classes(k)
    return out[:, cols].copy(), tot[cols].copy()


def count_edges(n: int, src, dst, k: int, threads: int | None = None):
    """Per-edge counts (Sec. 11): ``(lo[P], hi[P], uint64[P][C])`` for the P vertex pairs
    {lo < hi} joined in G_U, in ascending (lo, hi) order; row p counts, per class, the
    connected k-sets containing both lo and hi."""
    lib = _load()
    s, d = _arcs(src, dst)
    e = np.zeros(1, np.int64)
    rc = lib.oracle_graph_size(int(n), int(s.shape[0]), _ptr(s), _ptr(d), _ptr(e))
    if rc:
        raise ValueError(rc)
    P = int(e[0]) // 2
    C = NUM_CLASSES[k]
    out = np.zeros((P, C), np.uint64)
    lo = np.zeros(max(P, 1), np.int32)
    hi = np.zeros(max(P, 1), np.int32)
    rc = lib.oracle_count_edges(int(n), int(s.shape[0]), _ptr(s), _ptr(d), int(k),
                                int(threads or default_threads()), P, _ptr(out), _ptr(lo), _ptr(hi))
    if rc != 0:
        raise ValueError(f"oracle_count_edges failed with {rc}")
    return lo[:P].copy(), hi[:P].copy(), out


def simple_graph(n: int, src, dst):
    """The oracle's normalised graph: (off[n+1], nbr, dir) with dir bit0 = row->nbr,
    bit1 = nbr->row."""
    lib = _load()
    s, d = _arcs(src, dst)
    e = np.zeros(1, np.int64)
    rc = lib.oracle_graph_size(int(n), int(s.shape[0]), _ptr(s), _ptr(d), _ptr(e))
    if rc:
        raise ValueError(rc)
    off = np.zeros(n + 1, np.int64)
    nbr = np.zeros(int(e[0]), np.int32)
    dr = np.zeros(int(e[0]), np.uint8)
    rc = lib.oracle_graph_csr(int(n), int(s.shape[0]), _ptr(s), _ptr(d), _ptr(off), _ptr(nbr), _ptr(dr))
    if rc:
        raise ValueError(rc)
    return off, nbr, dr

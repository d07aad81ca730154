"""CPU oracle for cover-edge triangle counting — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The GPU library never calls it, and it never calls the GPU library:
the two share no code (the seeded input generators in ``graphgen`` serve both and hold no
counting arithmetic).

The arithmetic lives in ``cetc_oracle.c`` (plain C, one function per step of the paper's
CETC-Seq, CETC-Seq-S and CETC-SM algorithms, Sections 4.2 to 4.4).  This module builds it with gcc
and marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cetc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

UNVISITED = 0xFFFFFFFF

CHECK_CODES = {
    0: "ok",
    -1: "bad rowptr",
    -2: "neighbour index out of range",
    -3: "row not strictly increasing",
    -4: "self-loop",
    -5: "not symmetric",
}


def build(force: bool = True) -> str:
    """Compile liboracle.so (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", _SRC,
                               "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Stats(ctypes.Structure):
    _fields_ = [("triangles", ctypes.c_uint64), ("cover_edges", ctypes.c_uint64),
                ("probes_min", ctypes.c_uint64), ("probes_merge", ctypes.c_uint64)]


def _bind(lib):
    vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
    lib.orc_check_csr.argtypes = [vp, vp, u32, u64]
    lib.orc_check_csr.restype = ctypes.c_int
    lib.orc_bfs_levels.argtypes = [vp, vp, u32, vp]
    lib.orc_bfs_levels.restype = ctypes.c_int64
    lib.orc_cetc_seq.argtypes = [vp, vp, u32, vp, ctypes.POINTER(_Stats), vp]
    lib.orc_cetc_seq.restype = None
    lib.orc_cetc_sm.argtypes = [vp, vp, u32, vp, ctypes.c_int, ctypes.POINTER(u64),
                                ctypes.POINTER(u64)]
    lib.orc_cetc_sm.restype = u64
    lib.orc_cetc_sm_range.argtypes = [vp, vp, u32, vp, u32, u32, ctypes.c_int,
                                      ctypes.POINTER(u64), ctypes.POINTER(u64)]
    lib.orc_cetc_sm_range.restype = u64
    lib.orc_cetc_split.argtypes = [vp, vp, u32, vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]
    lib.orc_cetc_split.restype = u64
    lib.orc_local_clustering.argtypes = [vp, vp, u32, vp]
    lib.orc_local_clustering.restype = None
    lib.orc_cover_edges.argtypes = [vp, vp, u32, vp]
    lib.orc_cover_edges.restype = u64
    lib.orc_max_threads.restype = ctypes.c_int
    return lib


_override = None


def _load():
    global _lib
    if _override is not None:
        return _override
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


class use_library:
    """Context manager that routes this module's functions to another build of the
    oracle source (used by the mutation tests, which compile deliberately broken copies).
    """

    def __init__(self, path: str):
        self.lib = _bind(ctypes.CDLL(path))

    def __enter__(self):
        global _override
        self.prev = _override
        _override = self.lib
        return self

    def __exit__(self, *exc):
        global _override
        _override = self.prev
        return False


def _arrs(g):
    rowptr = np.ascontiguousarray(g.rowptr, dtype=np.uint32)
    colidx = np.ascontiguousarray(g.colidx, dtype=np.uint32)
    if colidx.size == 0:
        colidx = np.zeros(1, dtype=np.uint32)  # valid pointer for an edgeless graph
    return rowptr, colidx


def check_csr(g) -> int:
    """0 if g is a valid symmetric, sorted, loop-free CSR; else a negative code."""
    rowptr, colidx = _arrs(g)
    return int(_load().orc_check_csr(rowptr.ctypes.data, colidx.ctypes.data, g.n, g.nnz))


def bfs_levels(g):
    """(level uint32[n], depth): BFS restarted from each unvisited vertex in ascending ID."""
    rowptr, colidx = _arrs(g)
    level = np.empty(max(g.n, 1), dtype=np.uint32)
    depth = int(_load().orc_bfs_levels(rowptr.ctypes.data, colidx.ctypes.data, g.n,
                                       level.ctypes.data))
    if depth < 0:
        raise MemoryError("oracle BFS queue allocation failed")
    return level[: g.n], depth


@dataclass
class Result:
    triangles: int
    cover_edges: int
    probes_min: int
    probes_merge: int
    depth: int
    level: np.ndarray
    per_vertex: np.ndarray | None = None

    @property
    def covering_ratio(self) -> float:
        return self.cover_edges / self.num_edges if self.num_edges else 0.0

    num_edges: int = 0


def cetc_seq(g, level=None, per_vertex: bool = False) -> Result:
    """CETC-Seq (Section 4.2): BFS levels, then the horizontal-edge counting loop."""
    rowptr, colidx = _arrs(g)
    depth = -1
    if level is None:
        level, depth = bfs_levels(g)
    level = np.ascontiguousarray(level, dtype=np.uint32)
    lv = level if level.size else np.zeros(1, np.uint32)
    st = _Stats()
    t = np.zeros(max(g.n, 1), dtype=np.uint64) if per_vertex else None
    _load().orc_cetc_seq(rowptr.ctypes.data, colidx.ctypes.data, g.n, lv.ctypes.data,
                         ctypes.byref(st), t.ctypes.data if t is not None else None)
    return Result(int(st.triangles), int(st.cover_edges), int(st.probes_min),
                  int(st.probes_merge), depth, level,
                  t[: g.n] if t is not None else None, g.nnz // 2)


def cetc_sm(g, level=None, nthreads: int = 0):
    """CETC-SM (Section 4.4): (T, c1, c2) with T = c1 + c2 / 3, OpenMP over vertices."""
    rowptr, colidx = _arrs(g)
    if level is None:
        level, _ = bfs_levels(g)
    lv = np.ascontiguousarray(level, dtype=np.uint32)
    if lv.size == 0:
        lv = np.zeros(1, np.uint32)
    c1, c2 = ctypes.c_uint64(0), ctypes.c_uint64(0)
    T = _load().orc_cetc_sm(rowptr.ctypes.data, colidx.ctypes.data, g.n, lv.ctypes.data,
                            int(nthreads), ctypes.byref(c1), ctypes.byref(c2))
    return int(T), int(c1.value), int(c2.value)


def cetc_sm_range(g, level, u_begin: int, u_end: int, nthreads: int = 0):
    """CETC-SM restricted to first endpoints u in [u_begin, u_end): (T, c1, c2)."""
    rowptr, colidx = _arrs(g)
    lv = np.ascontiguousarray(level, dtype=np.uint32)
    if lv.size == 0:
        lv = np.zeros(1, np.uint32)
    c1, c2 = ctypes.c_uint64(0), ctypes.c_uint64(0)
    T = _load().orc_cetc_sm_range(rowptr.ctypes.data, colidx.ctypes.data, g.n, lv.ctypes.data,
                                  int(u_begin), int(u_end), int(nthreads), ctypes.byref(c1),
                                  ctypes.byref(c2))
    return int(T), int(c1.value), int(c2.value)


def cetc_split(g, level=None):
    """CETC-Seq-S (Section 4.3): (T, t0, t1) with t0 = forward-hashed triangles of the
    horizontal subgraph G0 and t1 = the hashed G1 intersections over horizontal edges."""
    rowptr, colidx = _arrs(g)
    if level is None:
        level, _ = bfs_levels(g)
    lv = np.ascontiguousarray(level, dtype=np.uint32)
    if lv.size == 0:
        lv = np.zeros(1, np.uint32)
    t0, t1 = ctypes.c_uint64(0), ctypes.c_uint64(0)
    T = int(_load().orc_cetc_split(rowptr.ctypes.data, colidx.ctypes.data, g.n, lv.ctypes.data,
                                   ctypes.byref(t0), ctypes.byref(t1)))
    if T == 0xFFFFFFFFFFFFFFFF:
        raise MemoryError("oracle split allocation failed")
    return T, int(t0.value), int(t1.value)


def local_clustering(g) -> np.ndarray:
    """C(v) = 2 t(v) / (d(v) (d(v) - 1)) in float64 (0 for d(v) < 2), from CETC-Seq's
    per-vertex counts."""
    rowptr, _ = _arrs(g)
    t = np.ascontiguousarray(cetc_seq(g, per_vertex=True).per_vertex, dtype=np.uint64)
    if t.size == 0:
        t = np.zeros(1, np.uint64)
    cc = np.empty(max(g.n, 1), dtype=np.float64)
    _load().orc_local_clustering(rowptr.ctypes.data, t.ctypes.data, g.n, cc.ctypes.data)
    return cc[: g.n]


def cover_edges(g, level) -> int:
    """|S|: horizontal edges (same BFS level), each undirected edge once."""
    rowptr, colidx = _arrs(g)
    lv = np.ascontiguousarray(level, dtype=np.uint32)
    if lv.size == 0:
        lv = np.zeros(1, np.uint32)
    return int(_load().orc_cover_edges(rowptr.ctypes.data, colidx.ctypes.data, g.n,
                                       lv.ctypes.data))


def count(g) -> int:
    """Triangle count of g by CETC-Seq."""
    return cetc_seq(g).triangles


def max_threads() -> int:
    return int(_load().orc_max_threads())

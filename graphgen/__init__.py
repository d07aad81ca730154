"""Seeded synthetic inputs: R-MAT, Erdős–Rényi, triangulated grids, closed-form
families and batches of uneven graphs, all as clean uint32 CSR (numpy arrays).

Input generation only: no triangle-counting arithmetic lives here.  The compiled part
(``graphgen.cpp``) is built by :func:`build` into ``libgraphgen.so`` next to this file.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

# The paper's R-MAT initiator (a, b, c, d) = (0.57, 0.19, 0.19, 0.05) (Section 6.2).
RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = True) -> str:
    """Compile libgraphgen.so with g++ -O3 -fopenmp."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["g++", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c++17", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _GgCsr(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
        ("nnz", ctypes.c_uint64),
        ("rowptr", ctypes.POINTER(ctypes.c_uint32)),
        ("colidx", ctypes.POINTER(ctypes.c_uint32)),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_uint64, ctypes.c_int, P(_GgCsr)]
        lib.gg_er.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, P(_GgCsr)]
        lib.gg_grid.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                P(_GgCsr)]
        lib.gg_grid_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        lib.gg_grid_edges.restype = ctypes.c_uint64
        lib.gg_from_edges.argtypes = [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_uint64, P(_GgCsr)]
        lib.gg_free.argtypes = [P(_GgCsr)]
        lib.gg_splitmix.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_void_p]
        lib.gg_permutation.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p]
        lib.gg_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class CSR:
    """Simple undirected graph as symmetric CSR with sorted uint32 neighbour lists."""

    rowptr: np.ndarray  # uint32[n + 1]
    colidx: np.ndarray  # uint32[nnz]
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.colidx.shape[0])

    @property
    def num_edges(self) -> int:
        """Undirected edges after cleaning (= stored entries / 2)."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))


def _take(rc: int, g: _GgCsr, name: str) -> CSR:
    if rc != 0:
        raise RuntimeError(f"graphgen failed ({rc}) for {name}")
    lib = _load()
    try:
        n = int(g.n)
        rowptr = np.ctypeslib.as_array(g.rowptr, shape=(n + 1,)).copy()
        nnz = int(g.nnz)
        colidx = (np.ctypeslib.as_array(g.colidx, shape=(nnz,)).copy() if nnz
                  else np.zeros(0, dtype=np.uint32))
    finally:
        lib.gg_free(ctypes.byref(g))
    return CSR(rowptr.astype(np.uint32, copy=False), colidx.astype(np.uint32, copy=False), name)


def rmat(scale: int, edge_factor: int = 16, seed: int = 1, abc=RMAT_ABC,
         permute: bool = True) -> CSR:
    """R-MAT graph: 2^scale vertices, edge_factor * 2^scale generated edges, cleaned,
    symmetrised and (by default) randomly relabelled."""
    lib = _load()
    g = _GgCsr()
    m = int(edge_factor) << int(scale)
    rc = lib.gg_rmat(int(scale), m, abc[0], abc[1], abc[2], seed & (2**64 - 1), int(permute),
                     ctypes.byref(g))
    return _take(rc, g, f"rmat{scale}_ef{edge_factor}_s{seed}")


def erdos_renyi(n: int, avg_degree: float, seed: int = 1) -> CSR:
    """G(n, M) with M = round(n * avg_degree / 2) uniform pairs, cleaned."""
    lib = _load()
    g = _GgCsr()
    m = int(round(n * avg_degree / 2))
    rc = lib.gg_er(int(n), m, seed & (2**64 - 1), ctypes.byref(g))
    return _take(rc, g, f"er{n}_d{avg_degree}_s{seed}")


def grid_edges(rows: int, cols: int) -> int:
    return int(_load().gg_grid_edges(rows, cols))


def tri_grid(rows: int, cols: int, delete_frac: float = 0.0, seed: int = 1) -> CSR:
    """Triangulated rows x cols grid (one diagonal per cell), row-major IDs, with
    round(delete_frac * |E|) edges removed by a seeded shuffle."""
    lib = _load()
    g = _GgCsr()
    ndel = int(round(delete_frac * grid_edges(rows, cols)))
    rc = lib.gg_grid(int(rows), int(cols), ndel, seed & (2**64 - 1), ctypes.byref(g))
    return _take(rc, g, f"grid{rows}x{cols}_del{delete_frac}_s{seed}")


def from_edges(n: int, edges, name: str = "") -> CSR:
    """Clean CSR from an iterable/array of (u, v) pairs: loops dropped, duplicates merged."""
    lib = _load()
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size and (e.min() < 0 or e.max() >= n):
        raise ValueError("edge endpoint out of range")
    u = np.ascontiguousarray(e[:, 0], dtype=np.uint32)
    v = np.ascontiguousarray(e[:, 1], dtype=np.uint32)
    g = _GgCsr()
    rc = lib.gg_from_edges(int(n), u.ctypes.data, v.ctypes.data, int(u.shape[0]), ctypes.byref(g))
    return _take(rc, g, name)


def splitmix(seed: int, start: int, count: int) -> np.ndarray:
    """Raw SplitMix64 outputs start .. start+count-1 of the sequence seeded by `seed`."""
    out = np.empty(count, dtype=np.uint64)
    _load().gg_splitmix(seed & (2**64 - 1), start, count, out.ctypes.data)
    return out


def permutation(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    _load().gg_permutation(n, seed & (2**64 - 1), out.ctypes.data)
    return out


def relabel(g: CSR, perm: np.ndarray) -> CSR:
    """The same graph with vertex x renamed perm[x]."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    e = np.stack([perm[rows], perm[g.colidx.astype(np.int64)]], axis=1)
    return from_edges(g.n, e, g.name + "_perm")


def disjoint_union(graphs) -> CSR:
    edges, base = [], 0
    for g in graphs:
        rows = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
        edges.append(np.stack([rows + base, g.colidx.astype(np.int64) + base], axis=1))
        base += g.n
    e = np.concatenate(edges) if edges else np.zeros((0, 2), np.int64)
    return from_edges(base, e, "union")


# --------------------------------------------------------------------------------------
# Closed-form families (small; built in Python then cleaned by the C routine).
# --------------------------------------------------------------------------------------

def complete(n: int) -> CSR:
    e = [(i, j) for i in range(n) for j in range(i + 1, n)]
    return from_edges(n, e, f"K{n}")


def cycle(n: int) -> CSR:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], f"C{n}")


def path(n: int) -> CSR:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], f"P{n}")


def star(n: int) -> CSR:
    return from_edges(n, [(0, i) for i in range(1, n)], f"S{n}")


def random_tree(n: int, seed: int) -> CSR:
    r = splitmix(seed, 0, max(n, 1))
    e = [(i, int(r[i] % np.uint64(i))) for i in range(1, n)]
    return from_edges(n, e, f"tree{n}")


def complete_bipartite(a: int, b: int) -> CSR:
    return from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)], f"K{a},{b}")


def complete_tripartite(a: int, b: int, c: int) -> CSR:
    parts = [range(0, a), range(a, a + b), range(a + b, a + b + c)]
    e = []
    for p in range(3):
        for q in range(p + 1, 3):
            e += [(i, j) for i in parts[p] for j in parts[q]]
    return from_edges(a + b + c, e, f"K{a},{b},{c}")


def hypercube(d: int) -> CSR:
    n = 1 << d
    e = [(x, x ^ (1 << k)) for x in range(n) for k in range(d) if x < x ^ (1 << k)]
    return from_edges(n, e, f"Q{d}")


def wheel(k: int) -> CSR:
    """Hub 0 joined to every vertex of the cycle 1..k."""
    e = [(0, i) for i in range(1, k + 1)] + [(i, i % k + 1) for i in range(1, k + 1)]
    return from_edges(k + 1, e, f"W{k}")


def clique_union(parts, book_pages: int = 0, chunk_entries: int = 1 << 26) -> CSR:
    """Disjoint union of `count` copies of K_k for each (k, count) in `parts`, in that order
    with consecutive IDs, then (if book_pages >= 1) one book K_{1,1,q}: vertices r, h
    joined to each other and to q pages (r first, then h, then the pages).  Built directly
    as CSR with vectorised fills, so it scales to billions of stored entries."""
    parts = [(int(k), int(c)) for k, c in parts if c > 0]
    assert all(k >= 1 for k, _ in parts)
    deg_groups = [(k - 1, k * c) for k, c in parts]
    n_cl = sum(k * c for k, c in parts)
    q = int(book_pages)
    n = n_cl + (q + 2 if q else 0)
    m = sum(k * (k - 1) * c for k, c in parts) + (4 * q + 2 if q else 0)
    assert m < (1 << 32) and n < (1 << 31)
    deg = np.empty(n, dtype=np.uint64)
    pos = 0
    for d, cnt in deg_groups:
        deg[pos:pos + cnt] = d
        pos += cnt
    if q:
        deg[pos:pos + 2] = q + 1
        deg[pos + 2:] = 2
    rowptr = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(deg, out=rowptr[1:])
    colidx = np.empty(m, dtype=np.uint32)
    vbase, ebase = 0, 0
    for k, c in parts:
        kk = k * (k - 1)
        j = np.arange(k - 1, dtype=np.uint32)
        pat = (j[None, :] + (j[None, :] >= np.arange(k, dtype=np.uint32)[:, None])).ravel()
        per = max(1, chunk_entries // max(kk, 1))
        for c0 in range(0, c, per):
            cc = min(per, c - c0)
            if kk:
                bases = (vbase + (c0 + np.arange(cc, dtype=np.uint64)) * k).astype(np.uint32)
                out = colidx[ebase + c0 * kk: ebase + (c0 + cc) * kk].reshape(cc, kk)
                np.add(pat[None, :], bases[:, None], out=out)
        vbase += k * c
        ebase += kk * c
    if q:
        r, h = vbase, vbase + 1
        pages = np.arange(vbase + 2, vbase + 2 + q, dtype=np.uint32)
        colidx[ebase] = h
        colidx[ebase + 1: ebase + 1 + q] = pages
        colidx[ebase + 1 + q] = r
        colidx[ebase + 2 + q: ebase + 2 + 2 * q] = pages
        pr = colidx[ebase + 2 + 2 * q:].reshape(q, 2)
        pr[:, 0] = r
        pr[:, 1] = h
    return CSR(rowptr.astype(np.uint32), colidx, f"cliques{len(parts)}+B{q}")


def friendship(k: int) -> CSR:
    """k triangles sharing vertex 0."""
    e = []
    for t in range(k):
        a, b = 1 + 2 * t, 2 + 2 * t
        e += [(0, a), (0, b), (a, b)]
    return from_edges(2 * k + 1, e, f"F{k}")


def empty_graph(n: int) -> CSR:
    return from_edges(n, np.zeros((0, 2), np.int64), f"empty{n}")


def gnp_small(n: int, p: float, seed: int) -> CSR:
    """Small dense-ish G(n, p) for brute-force cross-checks."""
    r = splitmix(seed, 0, n * n).reshape(n, n)
    thr = np.uint64(min(int(p * 2.0**64), 2**64 - 1))
    iu, ju = np.triu_indices(n, 1)
    mask = r[iu, ju] < thr
    return from_edges(n, np.stack([iu[mask], ju[mask]], axis=1), f"gnp{n}_{p}_{seed}")


# --------------------------------------------------------------------------------------
# Workloads with the shapes of the measured configurations.
# --------------------------------------------------------------------------------------

def config_seed(k: int) -> int:
    return 1000 + k


@dataclass
class Batch:
    """Concatenated CSRs: graph g owns rowptr_cat[row_off[g]:row_off[g+1]] (its n_g + 1
    local offsets, starting at 0) and colidx_cat[col_off[g]:col_off[g+1]] (local IDs)."""

    rowptr_cat: np.ndarray  # uint32
    colidx_cat: np.ndarray  # uint32
    row_off: np.ndarray  # int64[G + 1]
    col_off: np.ndarray  # int64[G + 1]
    kinds: list

    @property
    def num_graphs(self) -> int:
        return int(self.row_off.shape[0] - 1)

    def graph(self, g: int) -> CSR:
        r = self.rowptr_cat[self.row_off[g]:self.row_off[g + 1]]
        c = self.colidx_cat[self.col_off[g]:self.col_off[g + 1]]
        return CSR(r, c, self.kinds[g])

    @property
    def total_edges(self) -> int:
        return int(self.colidx_cat.shape[0]) // 2


def pack(graphs) -> Batch:
    row_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    col_off = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        row_off[i + 1] = row_off[i] + g.n + 1
        col_off[i + 1] = col_off[i] + g.nnz
    rowptr_cat = (np.concatenate([g.rowptr for g in graphs]) if graphs
                  else np.zeros(0, np.uint32))
    colidx_cat = (np.concatenate([g.colidx for g in graphs]) if graphs
                  else np.zeros(0, np.uint32))
    return Batch(rowptr_cat.astype(np.uint32), colidx_cat.astype(np.uint32), row_off, col_off,
                 [g.name for g in graphs])


def batch_member(g: int, base_seed: int, log2_min: int = 8, log2_max: int = 16):
    """Parameters of batch member g: half R-MAT (scale uniform in [log2_min, log2_max],
    edge factor uniform 8..32), half Erdős–Rényi (n log-uniform in [2^log2_min,
    2^log2_max], average degree uniform in [4, 64])."""
    r = splitmix(base_seed ^ (g * 0x9E3779B97F4A7C15 & (2**64 - 1)), 0, 4)
    seed = int(r[3])
    if g % 2 == 0:
        scale = log2_min + int(r[0] % np.uint64(log2_max - log2_min + 1))
        ef = 8 + int(r[1] % np.uint64(25))
        return ("rmat", scale, ef, seed)
    u = float(r[0] >> np.uint64(11)) / float(1 << 53)
    n = int(math.floor(2.0 ** (log2_min + u * (log2_max - log2_min))))
    d = 4.0 + 60.0 * float(r[1] >> np.uint64(11)) / float(1 << 53)
    return ("er", n, d, seed)


def make_batch(num_graphs: int, base_seed: int, log2_min: int = 8, log2_max: int = 16) -> Batch:
    graphs = []
    for g in range(num_graphs):
        kind, a, b, seed = batch_member(g, base_seed, log2_min, log2_max)
        if kind == "rmat":
            graphs.append(rmat(a, b, seed))
        else:
            graphs.append(erdos_renyi(a, b, seed))
    return pack(graphs)

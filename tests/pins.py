"""Independent counters used to pin the oracle (test helpers; no oracle code).

Each one is a different route to the plain definition of the triangle count in Section 2
of the paper: a triangle is a set of three distinct, pairwise-adjacent vertices.
  - brute_force_triples: the Triples algorithm of Section 3.1 (every ordered triple of
    vertices, divided by 6), written as plain Python loops;
  - trace_count: the trace identity of Section 3.1, T = trace(A^3) / 6, via numpy;
  - sparse_count: sum((A @ A) .* A) / 6 via scipy.sparse (the same identity, a different
    library routine);
  - per_vertex_trace: diag(A^3) / 2, the triangles through each vertex (Section 3.1).
"""
from __future__ import annotations

from collections import deque

import numpy as np
import scipy.sparse as sp


def dense_adjacency(g) -> np.ndarray:
    A = np.zeros((g.n, g.n), dtype=np.int64)
    rows = np.repeat(np.arange(g.n), g.degrees())
    A[rows, g.colidx.astype(np.int64)] = 1
    return A


def sparse_adjacency(g):
    rows = np.repeat(np.arange(g.n), g.degrees())
    data = np.ones(g.nnz, dtype=np.int64)
    return sp.csr_matrix((data, (rows, g.colidx.astype(np.int64))), shape=(g.n, g.n))


def brute_force_triples(g) -> int:
    adj = [set(g.colidx[g.rowptr[u]:g.rowptr[u + 1]].tolist()) for u in range(g.n)]
    t = 0
    for u in range(g.n):
        for v in range(g.n):
            for w in range(g.n):
                if v in adj[u] and w in adj[v] and w in adj[u]:
                    t += 1
    assert t % 6 == 0
    return t // 6


def trace_count(g) -> int:
    A = dense_adjacency(g)
    t = int(np.trace(A @ A @ A))
    assert t % 6 == 0
    return t // 6


def sparse_count(g) -> int:
    A = sparse_adjacency(g)
    t = int((A @ A).multiply(A).sum())
    assert t % 6 == 0
    return t // 6


def per_vertex_trace(g) -> np.ndarray:
    A = sparse_adjacency(g)
    d = np.asarray((A @ A).multiply(A).sum(axis=1)).ravel()
    assert np.all(d % 2 == 0)
    return (d // 2).astype(np.int64)


def triangles(g):
    """All triangles {a < b < c} by brute enumeration over sorted neighbour lists."""
    adj = [set(g.colidx[g.rowptr[u]:g.rowptr[u + 1]].tolist()) for u in range(g.n)]
    out = []
    for a in range(g.n):
        for b in sorted(x for x in adj[a] if x > a):
            for c in sorted(x for x in adj[b] if x > b):
                if c in adj[a]:
                    out.append((a, b, c))
    return out


def bfs_levels_from(g, roots_order) -> np.ndarray:
    """BFS levels where components are searched from the roots in `roots_order` order
    (every vertex must appear); used to check that the count does not depend on roots."""
    lev = np.full(g.n, -1, dtype=np.int64)
    for s in roots_order:
        if lev[s] >= 0:
            continue
        lev[s] = 0
        q = deque([s])
        while q:
            x = q.popleft()
            for y in g.colidx[g.rowptr[x]:g.rowptr[x + 1]]:
                if lev[y] < 0:
                    lev[y] = lev[x] + 1
                    q.append(int(y))
    return lev.astype(np.uint32)

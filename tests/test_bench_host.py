"""Host logic of bench.py: the algorithmic bytes of each intersection class, checked
against a per-edge count written directly from the definitions (no GPU)."""
import numpy as np
import pytest

import bench
import graphgen as gg
import oracle


def brute_class_bytes(g, level, lane_max, wave_max):
    """Cover edges {x, y} (same level, x the larger (degree class, ID) key) per class of
    d(x).  The lane class streams all of N(y) and stages N(x); the other classes stream
    y's neighbours that are on another level or above max(x, y), and stage x's
    neighbours that are on another level or above x.  Each staged x counts once."""
    n = g.n
    rows = [g.colidx[g.rowptr[v]:g.rowptr[v + 1]].tolist() for v in range(n)]
    d = np.diff(g.rowptr.astype(np.int64))
    cls = bench.degree_class(d)
    par = [int(level[v]) & 1 for v in range(n)]
    out = {k: {"cover_edges": 0, "bytes": 0} for k in ("isect_lane", "isect_wave", "isect_block")}
    staged = {k: set() for k in out}
    for u in range(n):
        for v in rows[u]:
            if u < v and par[u] == par[v]:
                if (cls[u], u) > (cls[v], v):
                    x, y = u, v
                else:
                    x, y = v, u
                name = ("isect_lane" if d[x] <= lane_max else
                        "isect_wave" if d[x] <= wave_max else "isect_block")
                out[name]["cover_edges"] += 1
                if name == "isect_lane":
                    streamed = len(rows[y])
                else:
                    streamed = sum(1 for w in rows[y] if par[w] != par[y] or w > max(x, y))
                out[name]["bytes"] += 4 * streamed
                staged[name].add(x)
    for name, xs in staged.items():
        for x in xs:
            if name == "isect_lane":
                out[name]["bytes"] += 4 * len(rows[x])
            else:
                out[name]["bytes"] += 4 * sum(1 for w in rows[x] if par[w] != par[x] or w > x)
    return out


@pytest.mark.parametrize("graph,params", [
    (lambda: gg.rmat(9, 8, seed=7), (4, 24, 4096)),
    (lambda: gg.rmat(8, 16, seed=3), (2, 12, 4096)),
    (lambda: gg.complete(12), (4, 8, 4096)),
])
def test_class_bytes_matches_definition(graph, params):
    g = graph()
    level, _ = oracle.bfs_levels(g)
    got = bench.class_bytes(g, np.asarray(level).astype(np.uint32), params)
    want = brute_class_bytes(g, level, params[0], params[1])
    assert got == want
    assert sum(v["cover_edges"] for v in got.values()) > 0

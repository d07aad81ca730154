"""Host logic of bench.py: the algorithmic bytes of each intersection class and the hub
selection, checked against counts written directly from the definitions (no GPU)."""
import json
import os

import numpy as np
import pytest

import bench
import graphgen as gg
import oracle


def brute_hubs(d, max_hubs, min_degree):
    """No hubs below 1024 * min_degree stored entries.  Else, among the thresholds
    c >= max(class(min_degree), 1), the vertex sets {class >= c} with 1 .. max_hubs
    members; the hubs are the largest of them (none if there is none)."""
    if sum(int(v) for v in d) < 1024 * min_degree:
        return set()
    cls = bench.degree_class(d)
    cmin = max(int(bench.degree_class(np.array([min_degree]))[0]), 1)
    best = set()
    for c in range(cmin, 128):
        s = {v for v in range(len(d)) if cls[v] >= c}
        if 1 <= len(s) <= max_hubs and len(s) > len(best):
            best = s
    return best


def brute_class_bytes(g, level, lane_max, wave_max, hubs=frozenset()):
    """Cover edges {x, y} (same level, x the larger (degree class, ID) key) per class of
    d(x).  The lane class streams all of N(y) and stages N(x); the other classes stream
    y's neighbours that are on another level or above max(x, y), and stage x's
    neighbours that are on another level or above x.  Each staged x counts once.  Edges
    with x a hub go to the hub pass: every partner y of a hub once streams its neighbours
    on another level or above y, looking each up in a mask of nw words, and reads its own
    mask; the masks take every hub's neighbours on another level or above it, and nw
    words per vertex are written."""
    n = g.n
    rows = [g.colidx[g.rowptr[v]:g.rowptr[v + 1]].tolist() for v in range(n)]
    d = np.diff(g.rowptr.astype(np.int64))
    cls = bench.degree_class(d)
    par = [int(level[v]) & 1 for v in range(n)]
    out = {k: {"cover_edges": 0, "bytes": 0, "plan_bytes": 0}
           for k in ("isect_lane", "isect_wave", "isect_block", "isect_hub")}
    staged = {k: set() for k in out}
    touched = {k: set() for k in out}  # vertices of the class's cover edges
    hub_partners = set()

    def pruned(v):
        return sum(1 for w in rows[v] if par[w] != par[v] or w > v)

    for u in range(n):
        for v in rows[u]:
            if u < v and par[u] == par[v]:
                if (cls[u], u) > (cls[v], v):
                    x, y = u, v
                else:
                    x, y = v, u
                if x in hubs:
                    out["isect_hub"]["cover_edges"] += 1
                    out["isect_hub"]["plan_bytes"] += 4 * min(d[x], d[y])
                    touched["isect_hub"] |= {x, y}
                    hub_partners.add(y)
                    continue
                name = ("isect_lane" if d[x] <= lane_max else
                        "isect_wave" if d[x] <= wave_max else "isect_block")
                out[name]["cover_edges"] += 1
                out[name]["plan_bytes"] += 4 * min(d[x], d[y])
                touched[name] |= {x, y}
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
                out[name]["bytes"] += 4 * pruned(x)
    for name, vs in touched.items():
        out[name]["plan_bytes"] += sum(4 * int(d[v]) for v in vs)
    if hubs:
        nw = 4 if len(hubs) <= 128 else 8
        out["isect_hub"]["bytes"] = (sum((4 + 4 * nw) * pruned(y) + 4 * nw for y in hub_partners)
                                     + sum(4 * pruned(h) for h in hubs) + 4 * nw * n)
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


@pytest.mark.parametrize("graph,hubs", [
    (lambda: gg.rmat(9, 8, seed=7), (7, 1)),
    (lambda: gg.rmat(9, 8, seed=7), (200, 1)),
    (lambda: gg.rmat(8, 16, seed=3), (256, 64)),
    (lambda: gg.complete(12), (256, 1)),
    (lambda: gg.complete(12), (5, 1)),
])
def test_hub_class_bytes_match_definition(graph, hubs):
    g = graph()
    level, _ = oracle.bfs_levels(g)
    d = g.degrees()
    hs = brute_hubs(d, *hubs)
    assert set(np.nonzero(bench.hub_set(d, *hubs))[0].tolist()) == hs
    got = bench.class_bytes(g, np.asarray(level).astype(np.uint32), (4, 24, 4096), hubs)
    want = brute_class_bytes(g, level, 4, 24, hs)
    assert got == want


@pytest.mark.parametrize("max_hubs,min_degree", [(1, 1), (7, 1), (128, 1), (129, 1),
                                                 (256, 1), (200, 64), (256, 4096), (0, 0)])
def test_hub_selection_matches_definition(max_hubs, min_degree):
    for g in (gg.rmat(10, 16, seed=5), gg.rmat(9, 8, seed=2), gg.star(40), gg.complete(9),
              gg.complete(40)):
        d = g.degrees()
        assert (set(np.nonzero(bench.hub_set(d, max_hubs, min_degree))[0].tolist())
                == brute_hubs(d, max_hubs, min_degree))


def test_gpu_hub_cases_reach_the_hub_pass():
    """The hub settings of the GPU parity tests do select hubs on their R-MAT cases."""
    for g in (gg.rmat(14, 32, 14), gg.rmat(16, 16, 16)):
        for hubs in [(1, 1), (7, 1), (128, 1), (129, 1), (256, 1), (200, 64)]:
            assert bench.hub_set(g.degrees(), *hubs).sum() > 0, (g.name, hubs)


def brute_plan_bytes(g, level):
    """The measurement plan's bytes written out per edge: BFS 4 (n + 1) + 4 nnz + 4 n,
    extraction 4 (n + 1) + 4 nnz + 8 |S|, intersections 4 min(d_u, d_v) per cover edge
    plus 4 d_x once for every vertex of a cover edge, merge 4 (d_u + d_v) per cover edge."""
    n = g.n
    d = [int(g.rowptr[v + 1] - g.rowptr[v]) for v in range(n)]
    S, short, merge, touched = 0, 0, 0, set()
    for u in range(n):
        for v in g.colidx[g.rowptr[u]:g.rowptr[u + 1]].tolist():
            if u < v and level[u] == level[v]:
                S += 1
                short += min(d[u], d[v])
                merge += d[u] + d[v]
                touched |= {u, v}
    return {"cover_edges": S, "bfs": 4 * (n + 1) + 4 * g.nnz + 4 * n,
            "extract": 4 * (n + 1) + 4 * g.nnz + 8 * S,
            "intersect": 4 * short + 4 * sum(d[x] for x in touched), "merge": 4 * merge}


@pytest.mark.parametrize("graph", [lambda: gg.rmat(9, 8, seed=7), lambda: gg.complete(12),
                                   lambda: gg.tri_grid(9, 13, 0.05, 3), lambda: gg.empty_graph(5)])
def test_plan_bytes_match_definition(graph):
    g = graph()
    level, _ = oracle.bfs_levels(g)
    got = bench.plan_bytes(g.rowptr, g.colidx, np.asarray(level, dtype=np.uint32))
    assert got == brute_plan_bytes(g, level)


def test_batch_plan_bytes_sum_over_members():
    """Members joined into groups (several groups: a tiny group size) give the sum of the
    members' own plan bytes, with 8 output bytes per member."""
    graphs = [gg.rmat(7, 8, seed=1), gg.complete(9), gg.empty_graph(3), gg.tri_grid(6, 7),
              gg.erdos_renyi(300, 6, 2)]
    b = gg.pack(graphs)
    levels = [np.asarray(oracle.bfs_levels(g)[0], dtype=np.uint32) for g in graphs]
    got = bench.batch_plan_bytes(b, levels, chunk_entries=600)
    want = {"cover_edges": 0, "bfs": 0, "extract": 0, "intersect": 0, "merge": 0}
    for g, lv in zip(graphs, levels):
        for k, v in brute_plan_bytes(g, lv).items():
            want[k] += v
    want["output"] = 8 * len(graphs)
    want["total"] = want["bfs"] + want["extract"] + want["intersect"] + want["output"]
    assert got == want


def test_stored_traffic_names_the_reported_kernels():
    # bench.py looks counter traffic up by kernel name; whenever profiles/traffic.json
    # holds records of the current kernel sources for a workload, the kernels bench.py
    # reports for it must be among them (a renamed template would otherwise leave
    # roofline.traffic null without notice)
    rec = json.load(open(os.path.join(bench.PROFILES, "traffic.json")))
    sha = bench.source_sha()
    wanted = {"batch4096": [bench.BATCH_KERNEL],
              "rmat22": [bench.KERNEL_OF_STEP[k] for k in ("isect_block", "isect_wave", "isect_hub")],
              "er22": [bench.KERNEL_OF_STEP["isect_wave"]]}
    for wl, kernels in wanted.items():
        current = {k for k, v in rec.get(wl, {}).items() if v.get("source_sha") == sha}
        if current:
            assert set(kernels) <= current, (wl, sorted(set(kernels) - current))

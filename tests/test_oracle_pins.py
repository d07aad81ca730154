"""Pins of the CPU oracle against things other than itself (CPU only).

- the paper's printed karate row (Table 1): T = 45, c = 35.9 %;
- brute force over all triples (the Triples algorithm, Section 3.1) on tiny graphs;
- trace(A^3) / 6 (Section 3.1) via numpy and scipy on small and medium graphs;
- closed forms (K_n, triangulated grids, trees, bipartite graphs, cycles, wheels,
  complete tripartite and friendship graphs, disjoint unions);
- invariants proven in the paper: every triangle has one or three horizontal edges
  (Lemmas H-E and HE2), T does not depend on the BFS roots (Theorem Correctness holds
  for an arbitrarily rooted BFS), CETC-SM's T = c1 + c2 / 3, per-vertex counts sum to 3T
  and equal diag(A^3) / 2;
- a BFS certificate for the levels (exact distances from the smallest-ID root);
- the cover-edge set size |S| (Theorem Gen-CES): closed forms, networkx BFS distances on
  tiny graphs, and CETC-Seq's own |S|;
- the split variant CETC-Seq-S (Section 4.3): closed forms, both terms against triangle
  enumeration by kind under BFS levels and under arbitrary labels, and t1 = c1,
  3 t0 = c2 of CETC-SM;
- local clustering coefficients: closed forms and networkx's clustering().
"""
import json
import math
import os

import networkx as nx
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def full_check(g):
    """Oracle result plus the checks that hold for every graph."""
    assert oracle.check_csr(g) == 0
    r = oracle.cetc_seq(g, per_vertex=True)
    T_sm, c1, c2 = oracle.cetc_sm(g, r.level)
    assert c2 % 3 == 0
    assert T_sm == r.triangles == c1 + c2 // 3
    assert int(r.per_vertex.sum()) == 3 * r.triangles
    return r


# ---- the paper's printed example -------------------------------------------------------

def test_karate_table1_row():
    ref = json.load(open(os.path.join(GOLDEN, "karate_table1.json")))
    k = nx.karate_club_graph()
    g = gg.from_edges(k.number_of_nodes(), list(k.edges()))
    assert g.n == ref["n"] and g.num_edges == ref["m"]
    r = full_check(g)
    assert r.triangles == ref["triangles"]
    assert round(100.0 * r.cover_edges / g.num_edges, 1) == ref["covering_ratio_percent"]


# ---- brute force and trace identities ------------------------------------------------------

@pytest.mark.parametrize("seed", range(40))
def test_brute_force_tiny(seed):
    n = 3 + seed % 14
    p = [0.1, 0.3, 0.5, 0.8, 1.0][seed % 5]
    g = gg.gnp_small(n, p, seed)
    r = full_check(g)
    assert r.triangles == pins.brute_force_triples(g) == pins.trace_count(g)
    assert np.array_equal(r.per_vertex.astype(np.int64), pins.per_vertex_trace(g))


@pytest.mark.parametrize("seed", range(12))
def test_trace_small(seed):
    n = 50 + 37 * seed
    g = gg.gnp_small(n, [0.02, 0.05, 0.2][seed % 3], 100 + seed)
    r = full_check(g)
    assert r.triangles == pins.trace_count(g)


@pytest.mark.parametrize("scale,ef,seed", [(8, 16, 1), (9, 8, 2), (10, 16, 1001), (11, 32, 3),
                                           (12, 16, 4)])
def test_rmat_against_sparse_trace(scale, ef, seed):
    g = gg.rmat(scale, ef, seed)
    r = full_check(g)
    assert r.triangles == pins.sparse_count(g)
    assert np.array_equal(r.per_vertex.astype(np.int64), pins.per_vertex_trace(g))


@pytest.mark.parametrize("n,d,seed", [(2000, 8, 1), (5000, 32, 2), (3000, 4, 3)])
def test_er_against_sparse_trace(n, d, seed):
    g = gg.erdos_renyi(n, d, seed)
    r = full_check(g)
    assert r.triangles == pins.sparse_count(g)


# ---- closed forms --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 17, 40])
def test_complete_graph(n):
    g = gg.complete(n)
    r = full_check(g)
    assert r.triangles == math.comb(n, 3)
    # root 0 is adjacent to all: every other vertex on level 1, all their edges horizontal
    assert r.cover_edges == math.comb(n - 1, 2)


@pytest.mark.parametrize("R,C", [(1, 1), (1, 5), (2, 2), (3, 7), (16, 16), (40, 25)])
def test_triangulated_grid(R, C):
    g = gg.tri_grid(R, C)
    assert g.num_edges == gg.grid_edges(R, C)
    r = full_check(g)
    assert r.triangles == 2 * (R - 1) * (C - 1)


def grid_cell_count(g, R, C):
    """Triangles of a triangulated grid with deletions, by checking both triangles of
    every cell: {(i,j),(i,j+1),(i+1,j+1)} and {(i,j),(i+1,j),(i+1,j+1)}."""
    adj = [set(g.colidx[g.rowptr[u]:g.rowptr[u + 1]].tolist()) for u in range(g.n)]
    t = 0
    for i in range(R - 1):
        for j in range(C - 1):
            a, b, c, d = i * C + j, i * C + j + 1, (i + 1) * C + j, (i + 1) * C + j + 1
            if d in adj[a]:
                t += (b in adj[a] and d in adj[b]) + (c in adj[a] and d in adj[c])
    return t


@pytest.mark.parametrize("R,C,frac,seed", [(30, 30, 0.01, 1), (20, 45, 0.1, 2), (64, 64, 0.3, 3)])
def test_grid_with_deletions(R, C, frac, seed):
    g = gg.tri_grid(R, C, frac, seed)
    assert g.num_edges == gg.grid_edges(R, C) - round(frac * gg.grid_edges(R, C))
    r = full_check(g)
    assert r.triangles == grid_cell_count(g, R, C)


@pytest.mark.parametrize("make", [
    lambda: gg.path(30), lambda: gg.star(50), lambda: gg.random_tree(200, 7),
    lambda: gg.complete_bipartite(7, 11), lambda: gg.cycle(4), lambda: gg.cycle(10),
    lambda: gg.cycle(5), lambda: gg.cycle(31), lambda: gg.hypercube(6),
    lambda: gg.empty_graph(0), lambda: gg.empty_graph(12),
])
def test_triangle_free(make):
    assert full_check(make()).triangles == 0


def test_single_triangle_and_families():
    assert full_check(gg.cycle(3)).triangles == 1
    for k in (4, 5, 9, 60):
        assert full_check(gg.wheel(k)).triangles == k
    for k in (1, 2, 7, 33):
        assert full_check(gg.friendship(k)).triangles == k
    for a, b, c in [(1, 1, 1), (2, 3, 4), (5, 5, 1), (6, 7, 8)]:
        assert full_check(gg.complete_tripartite(a, b, c)).triangles == a * b * c


def test_disjoint_union_additive():
    parts = [gg.complete(6), gg.wheel(8), gg.rmat(8, 16, 5), gg.empty_graph(3), gg.cycle(3)]
    u = gg.disjoint_union(parts)
    assert full_check(u).triangles == sum(full_check(p).triangles for p in parts)


# ---- the cover-edge set (Theorem Gen-CES, Section 4.1) ------------------------------------
# orc_cover_edges counts the horizontal edges.  Its pins: closed forms of |S| under the
# smallest-ID roots, a count over networkx's own BFS distances on tiny graphs, and the
# separately written edge loop of CETC-Seq (its |S|).

def cover_edges(g):
    level, _ = oracle.bfs_levels(g)
    return oracle.cover_edges(g, level)


def test_cover_edges_karate_table1():
    # Table 1: c = 35.9 % of karate's 78 edges; 28 is the only |S| that rounds to it
    ref = json.load(open(os.path.join(GOLDEN, "karate_table1.json")))
    k = nx.karate_club_graph()
    g = gg.from_edges(k.number_of_nodes(), list(k.edges()))
    S = cover_edges(g)
    assert round(100.0 * S / ref["m"], 1) == ref["covering_ratio_percent"]
    assert S == 28


@pytest.mark.parametrize("n", [1, 2, 3, 4, 9, 30])
def test_cover_edges_complete(n):
    # root 0 is adjacent to every other vertex: levels 0, 1, 1, ...; the level-1 clique
    assert cover_edges(gg.complete(n)) == math.comb(n - 1, 2)


@pytest.mark.parametrize("make", [
    lambda: gg.path(30), lambda: gg.star(12), lambda: gg.random_tree(200, 5),
    lambda: gg.cycle(10), lambda: gg.hypercube(6), lambda: gg.complete_bipartite(5, 9),
    lambda: gg.empty_graph(4)])
def test_cover_edges_bipartite_zero(make):
    # in a bipartite graph the BFS levels alternate sides: no edge joins equal levels
    assert cover_edges(make()) == 0


@pytest.mark.parametrize("k", [3, 5, 9, 21])
def test_cover_edges_odd_cycle(k):
    # the two BFS fronts of an odd cycle meet in exactly one edge on the same level
    assert cover_edges(gg.cycle(k)) == 1


@pytest.mark.parametrize("R,C", [(1, 1), (1, 6), (5, 2), (7, 7), (12, 31)])
def test_cover_edges_triangulated_grid(R, C):
    # from corner 0 with diagonals (i, j)-(i+1, j+1), L(i, j) = max(i, j): a row edge
    # (i, j)-(i, j+1) is horizontal iff j + 1 <= i, a column edge iff i + 1 <= j, a
    # diagonal never
    S = sum(min(i, C - 1) for i in range(R)) + sum(min(j, R - 1) for j in range(C))
    assert cover_edges(gg.tri_grid(R, C)) == S


def test_cover_edges_clique_union_and_book():
    # each K_k: its root alone on level 0, the rest a level-1 clique (C(k-1, 2) edges);
    # the book K_{1,1,q}: r on level 0, the spine h and the q pages on level 1 (q edges)
    parts, q = [(3, 4), (6, 2), (11, 1)], 17
    S = q + sum(c * math.comb(k - 1, 2) for k, c in parts)
    assert cover_edges(gg.clique_union(parts, q)) == S


@pytest.mark.parametrize("seed", range(10))
def test_cover_edges_networkx_bfs(seed):
    # tiny graphs: levels from networkx's shortest paths from each component's smallest
    # vertex, horizontal edges counted over networkx's edge list
    g = gg.gnp_small(8 + 3 * seed, [0.1, 0.25, 0.5][seed % 3], 300 + seed)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from((u, int(v)) for u in range(g.n)
                     for v in g.colidx[g.rowptr[u]:g.rowptr[u + 1]])
    dist = {}
    for comp in nx.connected_components(G):
        dist.update(nx.single_source_shortest_path_length(G, min(comp)))
    S = sum(1 for a, b in G.edges() if dist[a] == dist[b])
    assert cover_edges(g) == S


@pytest.mark.parametrize("make", [lambda: gg.rmat(11, 16, 41), lambda: gg.erdos_renyi(4000, 12, 8),
                                  lambda: gg.tri_grid(30, 40, 0.03, 6)])
def test_cover_edges_match_cetc_seq(make):
    g = make()
    level, _ = oracle.bfs_levels(g)
    assert oracle.cover_edges(g, level) == oracle.cetc_seq(g, level=level).cover_edges


# ---- invariants -------------------------------------------------------------------------

def bfs_certificate(g, level):
    """Levels are exact distances from the smallest ID of each component."""
    n = g.n
    rows = np.repeat(np.arange(n), g.degrees())
    cols = g.colidx.astype(np.int64)
    lv = level.astype(np.int64)
    assert np.all(np.abs(lv[rows] - lv[cols]) <= 1)
    # every non-root has a neighbour one level up
    has_parent = np.zeros(n, dtype=bool)
    has_parent[rows[lv[cols] == lv[rows] - 1]] = True
    roots = lv == 0
    assert np.all(has_parent | roots)
    # one root per component, and it is the component's smallest ID
    comp = np.arange(n)
    changed = True
    while changed:  # label propagation to the minimum
        new = comp.copy()
        np.minimum.at(new, rows, comp[cols])
        changed = not np.array_equal(new, comp)
        comp = new
    assert np.array_equal(np.flatnonzero(roots), np.unique(comp))


@pytest.mark.parametrize("make", [
    lambda: gg.rmat(10, 16, 1001), lambda: gg.erdos_renyi(3000, 3, 9),
    lambda: gg.tri_grid(25, 30, 0.05, 4),
    lambda: gg.disjoint_union([gg.cycle(7), gg.empty_graph(2), gg.rmat(7, 8, 3)]),
])
def test_bfs_levels_certificate(make):
    g = make()
    level, depth = oracle.bfs_levels(g)
    bfs_certificate(g, level)
    assert depth == int(level.max(initial=0))


@pytest.mark.parametrize("seed", range(6))
def test_every_triangle_has_one_or_three_horizontal_edges(seed):
    g = gg.rmat(8, 16, 50 + seed) if seed % 2 else gg.gnp_small(60, 0.15, seed)
    level, _ = oracle.bfs_levels(g)
    tris = pins.triangles(g)
    assert len(tris) == oracle.count(g)
    seen = set()
    for a, b, c in tris:
        h = int(level[a] == level[b]) + int(level[a] == level[c]) + int(level[b] == level[c])
        assert h in (1, 3)
        seen.add(h)
    assert seen == {1, 3}  # both kinds occur on these graphs


@pytest.mark.parametrize("seed", range(8))
def test_count_independent_of_roots(seed):
    g = gg.rmat(9, 16, 70 + seed) if seed % 2 else gg.disjoint_union(
        [gg.gnp_small(40, 0.2, seed), gg.wheel(12), gg.tri_grid(6, 9)])
    T = oracle.count(g)
    order = gg.permutation(g.n, 900 + seed)
    level = pins.bfs_levels_from(g, order)
    r = oracle.cetc_seq(g, level=level)
    assert r.triangles == T
    T_sm, c1, c2 = oracle.cetc_sm(g, level)
    assert T_sm == T and c2 % 3 == 0


@pytest.mark.parametrize("seed", range(4))
def test_relabelling_invariance(seed):
    g = gg.rmat(10, 8, 200 + seed, permute=False)
    h = gg.relabel(g, gg.permutation(g.n, seed))
    assert oracle.count(g) == oracle.count(h)


def test_check_csr_rejects_bad_input():
    g = gg.complete(4)
    assert oracle.check_csr(g) == 0
    bad = gg.CSR(g.rowptr.copy(), g.colidx.copy())
    bad.colidx[0] = 0  # self-loop at vertex 0
    assert oracle.check_csr(bad) == -4
    bad = gg.CSR(g.rowptr.copy(), g.colidx.copy())
    bad.colidx[[0, 1]] = bad.colidx[[1, 0]]
    assert oracle.check_csr(bad) == -3
    s = gg.star(4)
    bad = gg.CSR(s.rowptr.copy(), s.colidx.copy())
    bad.colidx[-1] = 2  # edge 3 -> 2 without 2 -> 3 (and 3 -> 0 dropped)
    assert oracle.check_csr(bad) == -5
    bad = gg.CSR(g.rowptr.copy(), g.colidx.copy())
    bad.rowptr[-1] += 1
    assert oracle.check_csr(bad) == -1


@pytest.mark.parametrize("seed", range(3))
def test_sm_range_partitions_the_edge_loop(seed):
    g = gg.rmat(11, 16, 300 + seed)
    level, _ = oracle.bfs_levels(g)
    T, c1, c2 = oracle.cetc_sm(g, level)
    cut = [0, g.n // 3, g.n // 2, g.n]
    parts = [oracle.cetc_sm_range(g, level, a, b) for a, b in zip(cut[:-1], cut[1:])]
    assert sum(p[1] for p in parts) == c1 and sum(p[2] for p in parts) == c2
    assert T == pins.sparse_count(g)


# ---- CETC-Seq-S: the split into G0 (horizontal edges) and G1 (the rest), Section 4.3 ----

def split_by_enumeration(g, level):
    """(t0, t1) by enumerating every triangle: t0 = triangles whose three vertices share a
    label, t1 = triangles with exactly one same-label edge (the two parts the split
    algorithm counts; a triangle with no same-label edge is in neither)."""
    t0 = t1 = 0
    for a, b, c in pins.triangles(g):
        h = int(level[a] == level[b]) + int(level[a] == level[c]) + int(level[b] == level[c])
        t0 += h == 3
        t1 += h == 1
    return int(t0), int(t1)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 9, 17])
def test_split_complete_graph(n):
    # Root 0 alone on level 0, the other n - 1 vertices on level 1: G0 is K_{n-1}.
    assert oracle.cetc_split(gg.complete(n)) == (
        math.comb(n, 3), math.comb(n - 1, 3), math.comb(n - 1, 2))


def test_split_wheels_friendship_and_triangle_free():
    for k in (4, 5, 9, 60):  # hub 0 is the root; each triangle has one rim edge
        assert oracle.cetc_split(gg.wheel(k)) == (k, 0, k)
    for k in (1, 2, 7):
        assert oracle.cetc_split(gg.friendship(k)) == (k, 0, k)
    for g in (gg.complete_bipartite(7, 11), gg.cycle(5), gg.cycle(31), gg.hypercube(5),
              gg.empty_graph(0), gg.empty_graph(12)):
        assert oracle.cetc_split(g) == (0, 0, 0)


@pytest.mark.parametrize("seed", range(8))
def test_split_terms_by_enumeration(seed):
    g = gg.gnp_small(40 + seed, 0.25, seed) if seed % 2 else gg.rmat(8, 16, 80 + seed)
    level, _ = oracle.bfs_levels(g)
    T, t0, t1 = oracle.cetc_split(g, level)
    assert (t0, t1) == split_by_enumeration(g, level)
    assert T == pins.brute_force_triples(g) if g.n <= 48 else T == pins.sparse_count(g)


@pytest.mark.parametrize("seed", range(4))
def test_split_terms_under_arbitrary_labels(seed):
    # Each step is checked on its own with labels that are not BFS levels: one shared
    # label makes G0 the whole graph (the forward-hashed step alone counts every
    # triangle); random labels give triangles with zero, one and three same-label edges.
    g = gg.rmat(9, 16, 120 + seed)
    T = pins.sparse_count(g)
    assert oracle.cetc_split(g, np.zeros(g.n, np.uint32)) == (T, T, 0)
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, 3, g.n).astype(np.uint32)
    _, t0, t1 = oracle.cetc_split(g, lab)
    assert (t0, t1) == split_by_enumeration(g, lab)


@pytest.mark.parametrize("seed", range(4))
def test_split_matches_cetc_sm_terms_and_any_root(seed):
    # t1 is CETC-SM's c1 (apexes on another level) and 3·t0 its c2; T holds for any roots.
    g = gg.rmat(11, 16, 140 + seed) if seed % 2 else gg.erdos_renyi(4000, 8, seed)
    T = pins.sparse_count(g)
    level, _ = oracle.bfs_levels(g)
    Ts, t0, t1 = oracle.cetc_split(g, level)
    _, c1, c2 = oracle.cetc_sm(g, level)
    assert Ts == T and t1 == c1 and 3 * t0 == c2
    other = pins.bfs_levels_from(g, gg.permutation(g.n, 500 + seed))
    assert oracle.cetc_split(g, other)[0] == T


# ---- local clustering coefficients from the per-vertex counts ---------------------------

def test_clustering_closed_forms():
    for n in (3, 4, 9, 30):
        assert np.all(oracle.local_clustering(gg.complete(n)) == 1.0)
    assert np.all(oracle.local_clustering(gg.complete(2)) == 0.0)
    for k in (4, 5, 9, 60):  # hub 0: k triangles over C(k, 2) pairs; rim: 2 of 3 pairs
        cc = oracle.local_clustering(gg.wheel(k))
        assert cc[0] == 2.0 / (k - 1) and np.all(cc[1:] == 2.0 / 3.0)
    for k in (1, 2, 7):  # centre: k of C(2k, 2) pairs; the others sit in one triangle
        cc = oracle.local_clustering(gg.friendship(k))
        assert cc[0] == 1.0 / (2 * k - 1) and np.all(cc[1:] == 1.0)
    for g in (gg.star(9), gg.path(12), gg.cycle(8), gg.complete_bipartite(4, 6),
              gg.empty_graph(5)):
        assert np.all(oracle.local_clustering(g) == 0.0)
    assert oracle.local_clustering(gg.empty_graph(0)).size == 0


@pytest.mark.parametrize("seed", range(4))
def test_clustering_against_networkx(seed):
    # networkx's clustering() is an independent routine for the same definition.
    if seed == 0:
        k = nx.karate_club_graph()
        g = gg.from_edges(34, list(k.edges()))
    else:
        g = gg.gnp_small(50 + seed, 0.2, seed) if seed % 2 else gg.rmat(9, 16, 160 + seed)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    rows = np.repeat(np.arange(g.n), g.degrees())
    G.add_edges_from(zip(rows.tolist(), g.colidx.tolist()))
    ref = nx.clustering(G)
    assert np.array_equal(oracle.local_clustering(g), np.array([ref[v] for v in range(g.n)]))


def test_full_size_per_vertex_reference_matches_oracle():
    # the full-size GPU test checks sampled t(v) against edges_among_neighbours (the
    # edges between two neighbours of v); on graphs the oracle handles whole, that count
    # equals the oracle's per-vertex counts at every vertex
    from tests.test_parity_full_gpu import edges_among_neighbours
    for g in [gg.rmat(11, 16, 11), gg.wheel(40), gg.complete(15), gg.tri_grid(20, 20, 0.02, 4),
              gg.friendship(9), gg.empty_graph(4)]:
        r = oracle.cetc_seq(g, per_vertex=True)
        got = np.array([edges_among_neighbours(g, v) for v in range(g.n)], dtype=np.int64)
        assert np.array_equal(got, r.per_vertex.astype(np.int64))

"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit-exact.

Compared per graph: T, the BFS level of every vertex (same smallest-ID roots), |S|,
and CETC-SM's c1 and c2.  Graphs span the closed-form families, the karate graph,
R-MAT, Erdős–Rényi and grid workloads at sizes the oracle finishes in seconds, with
ragged tails, isolated vertices, disconnected unions, and hubs large enough for the
chunked workgroup class.
"""
import sys

import networkx as nx
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def book(N):
    """Hubs 0 and 1 joined, both adjacent to 2 .. N+1: exactly N triangles."""
    e = [(0, 1)] + [(0, w) for w in range(2, N + 2)] + [(1, w) for w in range(2, N + 2)]
    return gg.from_edges(N + 2, e, f"book{N}")


def karate():
    k = nx.karate_club_graph()
    return gg.from_edges(34, list(k.edges()), "karate")


CASES = {
    "karate": karate,
    "K40": lambda: gg.complete(40),
    "K1": lambda: gg.complete(1),
    "K2": lambda: gg.complete(2),
    "C3": lambda: gg.cycle(3),
    "wheel500": lambda: gg.wheel(500),
    "friendship100": lambda: gg.friendship(100),
    "tripartite": lambda: gg.complete_tripartite(3, 40, 50),
    "grid64_del": lambda: gg.tri_grid(64, 64, 0.01, 3),
    "grid1x300": lambda: gg.tri_grid(1, 300),
    "path": lambda: gg.path(777),
    "star5000": lambda: gg.star(5000),
    "cycle1001": lambda: gg.cycle(1001),
    "hypercube8": lambda: gg.hypercube(8),
    "edgeless100": lambda: gg.empty_graph(100),
    "book10000": lambda: book(10000),
    "rmat10_c1": lambda: gg.rmat(10, 16, gg.config_seed(0)),
    "rmat12": lambda: gg.rmat(12, 16, 12),
    "rmat14_ef32": lambda: gg.rmat(14, 32, 14),
    "rmat16": lambda: gg.rmat(16, 16, 16),
    "rmat17_ef32": lambda: gg.rmat(17, 32, 17),
    "er16_d32": lambda: gg.erdos_renyi(1 << 16, 32, 5),
    "er14_d4": lambda: gg.erdos_renyi(1 << 14, 4, 6),
    "er14_d256": lambda: gg.erdos_renyi(1 << 14, 256, 7),
    "union": lambda: gg.disjoint_union([gg.rmat(9, 16, 1), gg.empty_graph(5), gg.wheel(30),
                                        gg.tri_grid(10, 13, 0.1, 2), gg.complete(20)]),
    # the smallest vertex with neighbours sits in a triangle, the large component after
    # it: the first search reaches three vertices, the union-find finds the rest
    "small_first": lambda: gg.disjoint_union([gg.empty_graph(3), gg.complete(3),
                                              gg.rmat(12, 16, 21)]),
    # a large first component and many small ones after it (their edges joined alone)
    "big_first": lambda: gg.disjoint_union([gg.erdos_renyi(1 << 12, 16, 8)]
                                           + [gg.complete(4)] * 40 + [gg.empty_graph(7)]
                                           + [gg.path(9)] * 5),
}


def components(g):
    """Connected components (isolated vertices included), via scipy."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    a = sp.csr_matrix((np.ones(g.nnz, dtype=np.int8), g.colidx, g.rowptr), shape=(g.n, g.n))
    return int(connected_components(a, directed=False)[0]) if g.n else 0


_cache = {}


def case(name):
    if name not in _cache:
        g = CASES[name]()
        r = oracle.cetc_seq(g, per_vertex=True)
        T_sm, c1, c2 = oracle.cetc_sm(g, r.level)
        assert T_sm == r.triangles
        _cache[name] = (g, r, c1, c2)
    return _cache[name]


def upload(g, tcm):
    return tcm.to_device(g.rowptr, g.colidx)


@pytest.mark.parametrize("name", list(CASES))
def test_count_matches_oracle(tc_lib, name):
    g, r, c1, c2 = case(name)
    say(f"[parity] tc_count_ex {name}: n={g.n} m={g.nnz}")
    rp, ci = upload(g, tc_lib)
    stats, level = tc_lib.tc_count_ex(rp, ci, want_levels=True)
    assert stats.triangles == r.triangles
    assert stats.cover_edges == r.cover_edges
    assert stats.c1 == c1 and stats.c2 == c2
    assert np.array_equal(level.cpu().numpy().view(np.uint32), r.level)
    assert stats.depth == int(r.level.max(initial=0))
    assert stats.num_roots == components(g)
    assert tc_lib.tc_count(rp, ci) == r.triangles


@pytest.mark.parametrize("name", ["karate", "wheel500", "tripartite", "grid64_del", "rmat12",
                                  "rmat16", "er16_d32", "union"])
def test_split_terms_match_cetc_s(tc_lib, name):
    # CETC-Seq-S (Section 4.3) counts the triangles of the horizontal subgraph G0 by
    # forward-hashing (t0) and the G1 intersections over horizontal edges (t1).  The GPU
    # counts both in one pass: its other-level apexes are t1 and its same-level apexes
    # see each G0 triangle from its three edges.
    g, r, _, _ = case(name)
    T, t0, t1 = oracle.cetc_split(g, r.level)
    say(f"[parity] split terms {name}: n={g.n} m={g.nnz} t0={t0} t1={t1}")
    rp, ci = upload(g, tc_lib)
    stats, _ = tc_lib.tc_count_ex(rp, ci)
    assert T == r.triangles
    assert stats.c1 == t1 and stats.c2 == 3 * t0 and stats.triangles == t0 + t1
    assert tc_lib.tc_count(rp, ci) == t0 + t1


SPLIT_SETTINGS = {
    "default": (None, None),
    "hubs": (None, (16, 1)),            # the hub pass on every graph of >= 1024 entries
    "chunked": ((0, 16, 100, 7), None),  # workgroup class in other/same-level passes
    "wave": ((0, 512, 16384, 1024), None),
}


@pytest.mark.parametrize("setting", list(SPLIT_SETTINGS))
@pytest.mark.parametrize("name", ["karate", "wheel500", "tripartite", "grid64_del", "rmat12",
                                  "rmat16", "er16_d32", "union", "book10000", "K40"])
def test_pruned_split_terms_match_cetc_s(tc_lib, name, setting):
    # tc_count_split tallies the apexes of tc_count's own pruned pass by the level of the
    # streamed entry: same-level ones are the triangles inside G0 (t0, the forward-hashed
    # term of CETC-Seq-S, Section 4.3), other-level ones the G1 intersections (t1).
    g, r, _, _ = case(name)
    T, t0, t1 = oracle.cetc_split(g, r.level)
    isect, hubs = SPLIT_SETTINGS[setting]
    say(f"[parity] pruned split terms {name} ({setting}): t0={t0} t1={t1}")
    rp, ci = upload(g, tc_lib)
    saved_i, saved_h = tc_lib.tc_get_isect_params(), tc_lib.tc_get_hub_params()
    try:
        if isect:
            tc_lib.tc_set_isect_params(*isect)
        if hubs:
            tc_lib.tc_set_hub_params(*hubs)
        got = tc_lib.tc_count_split(rp, ci)
        info = tc_lib.tc_last_call_info()
        pruned = tc_lib.tc_count(rp, ci)
    finally:
        tc_lib.tc_set_isect_params(*saved_i)
        tc_lib.tc_set_hub_params(*saved_h)
    assert T == r.triangles
    assert got == (t0, t1)
    assert pruned == t0 + t1
    if hubs and name in ("rmat12", "rmat16"):
        assert info["hubs"] > 0  # the hub pass took part


FE_GRAPHS = ["karate", "K40", "tripartite", "rmat12", "er14_d256", "rmat16", "er16_d32",
             "union", "book10000", "grid64_del"]


@pytest.mark.parametrize("name", FE_GRAPHS)
def test_forward_dispatch_matches_oracle(tc_lib, name):
    # CETC-Seq-FE (Section 4.3): tc_count switches to the forward ordering (every vertex
    # on one level) when c = |S| / |E| reaches the threshold (the paper's 0.7 here; the
    # library's default 2.0 never switches).  The oracle's split with one shared label is
    # the forward-hashed count of every triangle.
    g, r, _, _ = case(name)
    c = r.cover_edges / g.num_edges
    T_fwd, t0, t1 = oracle.cetc_split(g, np.zeros(g.n, dtype=np.uint32))
    assert (T_fwd, t0, t1) == (r.triangles, r.triangles, 0)
    say(f"[parity] forward dispatch {name}: c={c:.3f}")
    rp, ci = upload(g, tc_lib)
    saved = tc_lib.tc_get_forward_threshold()
    assert saved == 2.0
    try:
        assert tc_lib.tc_count(rp, ci) == r.triangles
        assert tc_lib.tc_last_call_info()["forward"] == 0  # off by default
        tc_lib.tc_set_forward_threshold(0.7)  # the paper's setting
        assert tc_lib.tc_count(rp, ci) == r.triangles
        info = tc_lib.tc_last_call_info()
        assert info["forward"] == (1 if c >= 0.7 else 0)
        assert info["cover_edges"] == r.cover_edges  # the BFS |S| that decided
        tc_lib.tc_set_forward_threshold(0.0)  # always the forward ordering
        assert tc_lib.tc_count(rp, ci) == T_fwd
        assert tc_lib.tc_last_call_info()["forward"] == 1
        tc_lib.tc_set_forward_threshold(2.0)  # never
        assert tc_lib.tc_count(rp, ci) == r.triangles
        assert tc_lib.tc_last_call_info()["forward"] == 0
        # the statistics and the split terms keep the BFS levels
        tc_lib.tc_set_forward_threshold(0.0)
        stats, _ = tc_lib.tc_count_ex(rp, ci)
        assert stats.triangles == r.triangles and tc_lib.tc_last_call_info()["forward"] == 0
        assert sum(tc_lib.tc_count_split(rp, ci)) == r.triangles
        assert tc_lib.tc_last_call_info()["forward"] == 0
    finally:
        tc_lib.tc_set_forward_threshold(saved)


@pytest.mark.parametrize("setting", ["hubs", "chunked", "wave"])
@pytest.mark.parametrize("name", ["K40", "rmat12", "er14_d256", "rmat16", "book10000"])
def test_forward_ordering_under_class_and_hub_settings(tc_lib, name, setting):
    g, r, _, _ = case(name)
    isect, hubs = SPLIT_SETTINGS[setting]
    say(f"[parity] forward ordering {name} ({setting})")
    rp, ci = upload(g, tc_lib)
    saved = (tc_lib.tc_get_forward_threshold(), tc_lib.tc_get_isect_params(),
             tc_lib.tc_get_hub_params())
    try:
        tc_lib.tc_set_forward_threshold(0.0)
        if isect:
            tc_lib.tc_set_isect_params(*isect)
        if hubs:
            tc_lib.tc_set_hub_params(*hubs)
        got = tc_lib.tc_count(rp, ci)
        fwd = tc_lib.tc_last_call_info()["forward"]
    finally:
        tc_lib.tc_set_forward_threshold(saved[0])
        tc_lib.tc_set_isect_params(*saved[1])
        tc_lib.tc_set_hub_params(*saved[2])
    assert got == r.triangles and fwd == 1


@pytest.mark.parametrize("name", ["karate", "K40", "star5000", "wheel500", "rmat12", "er14_d4",
                                  "book10000", "grid64_del", "union", "small_first", "rmat16",
                                  "rmat14_ef32", "er16_d32"])
def test_per_vertex_matches_oracle(tc_lib, name):
    # book10000's two hubs stage more than 4096 keys each, which the per-vertex pass
    # takes in several hash chunks
    g, r, _, _ = case(name)
    say(f"[parity] tc_count_per_vertex {name}")
    rp, ci = upload(g, tc_lib)
    t = tc_lib.as_u64(tc_lib.tc_count_per_vertex(rp, ci))
    assert np.array_equal(t, r.per_vertex)


@pytest.mark.parametrize("setting", ["chunked", "wave", "hubs"])
@pytest.mark.parametrize("name", ["rmat16", "book10000", "er16_d32", "union", "K40"])
def test_per_vertex_under_isect_settings(tc_lib, name, setting):
    # chunked: every vertex above 16 entries in the workgroup class, 100-key chunks and
    # 7-partner items; wave: the wavefront class up to 512 entries, chunks of up to
    # 16384 keys asked for (the per-vertex pass caps them at 4096); hubs: the hub pass
    # (its triangles attributed per hub bit) on every graph of at least 1024 entries
    g, r, _, _ = case(name)
    isect, hubs = SPLIT_SETTINGS[setting]
    say(f"[parity] tc_count_per_vertex {name} ({setting})")
    rp, ci = upload(g, tc_lib)
    saved_i, saved_h = tc_lib.tc_get_isect_params(), tc_lib.tc_get_hub_params()
    try:
        if isect:
            tc_lib.tc_set_isect_params(*isect)
        if hubs:
            tc_lib.tc_set_hub_params(*hubs)
        t = tc_lib.as_u64(tc_lib.tc_count_per_vertex(rp, ci))
        info = tc_lib.tc_last_call_info()
    finally:
        tc_lib.tc_set_isect_params(*saved_i)
        tc_lib.tc_set_hub_params(*saved_h)
    assert np.array_equal(t, r.per_vertex)
    if hubs and name in ("rmat16", "book10000"):
        assert info["hubs"] > 0  # the hub pass took part


@pytest.mark.parametrize("name", ["karate", "K40", "K2", "K1", "wheel500", "friendship100", "star5000",
                                  "edgeless100", "rmat12", "er14_d4", "union"])
def test_local_clustering_matches_oracle(tc_lib, name):
    # Both sides divide exact doubles once (2 t / (d (d - 1)) here, t / pairs in the
    # oracle), so the coefficients agree bit for bit.
    g, _, _, _ = case(name)
    say(f"[parity] tc_local_clustering {name}")
    rp, ci = upload(g, tc_lib)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tri = tc_lib.tc_count_per_vertex(rp, ci, stream=s)
        cc = tc_lib.tc_local_clustering(rp, tri, stream=s)
    s.synchronize()
    assert cc.dtype == torch.float64 and cc.numel() == g.n
    assert np.array_equal(cc.cpu().numpy(), oracle.local_clustering(g))


PARAMS = [(0, 0, 4096, 256), (64, 64, 256, 16), (16, 512, 16384, 1024), (0, 512, 64, 1),
          (512, 512, 4096, 256), (4, 32, 1024, 64), (0, 16, 100, 1000), (16, 128, 16384, 3)]


@pytest.mark.parametrize("params", PARAMS)
@pytest.mark.parametrize("name", ["rmat14_ef32", "book10000", "er16_d32", "union"])
def test_every_class_setting_gives_the_same_count(tc_lib, name, params):
    g, r, _, _ = case(name)
    say(f"[parity] isect params {params} on {name}")
    rp, ci = upload(g, tc_lib)
    saved = tc_lib.tc_get_isect_params()
    try:
        tc_lib.tc_set_isect_params(*params)
        stats, _ = tc_lib.tc_count_ex(rp, ci)
        pruned = tc_lib.tc_count(rp, ci)
    finally:
        tc_lib.tc_set_isect_params(*saved)
    assert stats.triangles == r.triangles and stats.cover_edges == r.cover_edges
    assert pruned == r.triangles


@pytest.mark.parametrize("name", ["rmat14_ef32", "book10000", "er16_d32", "grid64_del"])
def test_unaligned_colidx(tc_lib, name):
    """colidx not 16-byte aligned: the streaming kernels take their scalar-load path."""
    g, r, _, _ = case(name)
    say(f"[parity] unaligned colidx {name}")
    rp, ci = upload(g, tc_lib)
    buf = torch.zeros(ci.numel() + 1, dtype=torch.int32, device="cuda")
    buf[1:] = ci
    shifted = buf[1:]
    assert shifted.data_ptr() % 16 != 0
    saved = tc_lib.tc_get_isect_params()
    try:
        for params in [saved, (0, 16, 100, 7)]:
            tc_lib.tc_set_isect_params(*params)
            stats, _ = tc_lib.tc_count_ex(rp, shifted)
            assert stats.triangles == r.triangles and stats.cover_edges == r.cover_edges
            assert tc_lib.tc_count(rp, shifted) == r.triangles
            t = tc_lib.as_u64(tc_lib.tc_count_per_vertex(rp, shifted))
            assert np.array_equal(t, r.per_vertex)
    finally:
        tc_lib.tc_set_isect_params(*saved)


def test_empty_inputs(tc_lib):
    say("[parity] empty inputs")
    rp = torch.zeros(1, dtype=torch.int32, device="cuda")
    ci = torch.zeros(0, dtype=torch.int32, device="cuda")
    assert tc_lib.tc_count(rp, ci) == 0
    g = gg.empty_graph(17)
    rp, ci = upload(g, tc_lib)
    stats, level = tc_lib.tc_count_ex(rp, ci, want_levels=True)
    assert stats.triangles == 0 and stats.num_roots == 17
    assert int(level.abs().sum()) == 0


def test_repeat_calls_are_identical(tc_lib):
    g, r, _, _ = case("rmat16")
    say("[parity] repeated tc_count rmat16")
    rp, ci = upload(g, tc_lib)
    assert [tc_lib.tc_count(rp, ci) for _ in range(5)] == [r.triangles] * 5


def test_validate_accepts_and_rejects(tc_lib):
    say("[parity] tc_validate_csr")
    for name in ("karate", "rmat12", "union", "edgeless100"):
        g, _, _, _ = case(name)
        assert tc_lib.tc_validate_csr(*upload(g, tc_lib)) == 0
    g = gg.complete(6)
    bad = []
    x = g.colidx.copy(); x[0] = 0; bad.append((g.rowptr, x))            # self-loop
    x = g.colidx.copy(); x[[0, 1]] = x[[1, 0]]; bad.append((g.rowptr, x))  # unsorted
    x = g.colidx.copy(); x[0] = 6; bad.append((g.rowptr, x))            # ID out of range
    s = gg.star(5)
    x = s.colidx.copy(); x[-1] = 2; bad.append((s.rowptr, x))           # asymmetric
    r2 = g.rowptr.copy(); r2[3] = r2[2] - 1; bad.append((r2, g.colidx))  # not monotone
    r3 = g.rowptr.copy(); r3[-1] -= 1; bad.append((r3, g.colidx))        # rowptr[n] != m
    for rp, ci in bad:
        assert tc_lib.tc_validate_csr(*tc_lib.to_device(rp, ci)) == -4


def test_count_reports_same_level_asymmetry(tc_lib):
    """Star centre 0 with leaves 1..4, the entry 0 of leaf 4's row replaced by 2: 4 lists 2
    as a same-level partner, 2 does not list 4, so 4's partner records stay short and the
    count stops with TC_ERR_INVALID_GRAPH before any intersection."""
    say("[parity] asymmetric same-level entry")
    s = gg.star(5)
    x = s.colidx.copy()
    x[-1] = 2
    with pytest.raises(tc_lib.TCError) as e:
        tc_lib.tc_count(*tc_lib.to_device(s.rowptr, x))
    assert e.value.status == -4


# ---- hub pass (tc_set_hub_params) -------------------------------------------------------
# (max_hubs, min_degree): a single hub, hub sets either side of the 4- / 8-word mask
# boundary (128 hubs), the default, and settings that leave some graphs without hubs.
HUB_PARAMS = [(1, 1), (7, 1), (128, 1), (129, 1), (256, 1), (200, 64), (256, 4096), (0, 0)]
HUB_CASES = ["rmat14_ef32", "rmat16", "book10000", "er16_d32", "union", "wheel500", "K40",
             "star5000", "friendship100", "tripartite", "karate"]


@pytest.mark.parametrize("hubs", HUB_PARAMS)
@pytest.mark.parametrize("name", HUB_CASES)
def test_hub_pass_gives_the_same_count(tc_lib, name, hubs):
    import bench
    g, r, _, _ = case(name)
    nh = int(bench.hub_set(g.degrees(), *hubs).sum())
    say(f"[parity] hub params {hubs} on {name}: {nh} hubs")
    rp, ci = upload(g, tc_lib)
    saved = tc_lib.tc_get_hub_params()
    try:
        tc_lib.tc_set_hub_params(*hubs)
        got = [tc_lib.tc_count(rp, ci) for _ in range(2)]
        stats, _ = tc_lib.tc_count_ex(rp, ci)  # never uses the hub pass
    finally:
        tc_lib.tc_set_hub_params(*saved)
    assert got == [r.triangles] * 2
    assert stats.triangles == r.triangles and stats.cover_edges == r.cover_edges


def test_hub_partner_asymmetry_is_reported(tc_lib):
    """Vertex 1 (leaves 4..599, the only hub with max_hubs = 1; the graph's 1200 stored
    entries reach the pass's size floor of 1024 * min_degree) and vertex 2 sit on level 1
    under root 0; vertex 3 hangs off 2 on level 2.  Row 2 lists 1 but row 1 lists 3 in
    place of 2 (a level-2 entry, no partner), so hub 1's cursor ends one past its own
    partner count and the count stops with TC_ERR_INVALID_GRAPH."""
    say("[parity] asymmetric hub partner")
    e = [(0, 1), (0, 2), (1, 2), (2, 3)] + [(1, w) for w in range(4, 600)]
    g = gg.from_edges(600, e, "hub_asym")
    assert g.nnz >= 1024
    x = g.colidx.copy()
    lo, hi = int(g.rowptr[1]), int(g.rowptr[2])
    row = x[lo:hi]
    assert list(row[:3]) == [0, 2, 4]
    row[1] = 3
    x[lo:hi] = row
    saved = tc_lib.tc_get_hub_params()
    try:
        tc_lib.tc_set_hub_params(1, 1)
        assert tc_lib.tc_count(*upload(g, tc_lib)) == 1  # the symmetric graph: one triangle
        with pytest.raises(tc_lib.TCError) as err:
            tc_lib.tc_count(*tc_lib.to_device(g.rowptr, x))
    finally:
        tc_lib.tc_set_hub_params(*saved)
    assert err.value.status == -4


def test_concurrent_counts_on_two_streams(tc_lib):
    """Two host threads count graphs of more than 2^22 entries at once, each on its own
    stream (each call forks and joins its own side stream): every result is exact."""
    import threading
    cases = [case("rmat17_ef32"), case("rmat17_ef32")]
    for g, _, _, _ in cases:
        assert g.nnz >= 1 << 22
    say("[parity] concurrent tc_count on two streams")
    dev = [upload(g, tc_lib) for g, _, _, _ in cases]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    got = [[], []]
    errors = []

    def work(i):
        try:
            with torch.cuda.stream(streams[i]):
                for _ in range(6):
                    got[i].append(tc_lib.tc_count(*dev[i], stream=streams[i]))
        except Exception as e:  # reported below
            errors.append(e)

    th = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not errors, errors
    for i, (g, r, _, _) in enumerate(cases):
        assert got[i] == [r.triangles] * 6, (g.name, got[i])


def test_concurrent_long_searches_on_four_streams(tc_lib):
    """Four host threads count high-diameter graphs at once, each on its own stream, so
    that several calls reach the cooperative BFS launch together: every result is exact."""
    import threading
    names = ["path", "cycle1001", "grid64_del", "grid1x300"]
    cases = [case(nm) for nm in names]
    say("[parity] concurrent long searches on four streams")
    dev = [upload(g, tc_lib) for g, _, _, _ in cases]
    streams = [torch.cuda.Stream() for _ in names]
    got = [[] for _ in names]
    errors = []

    def work(i):
        try:
            with torch.cuda.stream(streams[i]):
                for _ in range(8):
                    got[i].append(tc_lib.tc_count(*dev[i], stream=streams[i]))
        except Exception as e:  # reported below
            errors.append(e)

    th = [threading.Thread(target=work, args=(i,)) for i in range(len(names))]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not errors, errors
    for i, (g, r, _, _) in enumerate(cases):
        assert got[i] == [r.triangles] * 8, (names[i], got[i])


@pytest.mark.parametrize("hubs", [(1, 1), (7, 1), (129, 1), (256, 1), (0, 0)])
@pytest.mark.parametrize("name", ["rmat14_ef32", "rmat17_ef32", "union"])
def test_device_picks_the_hubs_of_the_host_rule(tc_lib, name, hubs):
    """The device's hub selection (class histogram, threshold, numbering) yields exactly
    as many hubs as the host rule of bench.hub_set, the pass has work items when it has
    hubs, tc_count_ex never runs it, and the side stream is used from 2^22 entries on."""
    import bench
    g, r, _, _ = case(name)
    want = int(bench.hub_set(g.degrees(), *hubs).sum())
    say(f"[parity] device hub selection {hubs} on {name}: {want} hubs expected")
    rp, ci = upload(g, tc_lib)
    saved = tc_lib.tc_get_hub_params()
    try:
        tc_lib.tc_set_hub_params(*hubs)
        assert tc_lib.tc_count(rp, ci) == r.triangles
        info = tc_lib.tc_last_call_info()
        tc_lib.tc_count_ex(rp, ci)
        info_ex = tc_lib.tc_last_call_info()
    finally:
        tc_lib.tc_set_hub_params(*saved)
    assert info["hubs"] == want
    assert (info["hub_items"] > 0) == (want > 0)
    assert info["cover_edges"] == r.cover_edges == info_ex["cover_edges"]
    assert info_ex["hubs"] == 0 and info_ex["hub_items"] == 0
    assert info["side_stream"] == (1 if g.nnz >= 1 << 22 else 0)
    assert info_ex["side_stream"] == (1 if g.nnz >= 1 << 22 else 0)


def test_last_call_info_of_an_empty_graph(tc_lib):
    g, r, _, _ = case("rmat12")
    tc_lib.tc_count(*upload(g, tc_lib))
    assert tc_lib.tc_last_call_info()["cover_edges"] == r.cover_edges
    e = gg.empty_graph(5)
    tc_lib.tc_count(*upload(e, tc_lib))
    assert all(v == 0 for v in tc_lib.tc_last_call_info().values())


def test_step_timed_calls_match_and_stay_on_one_stream(tc_lib):
    """With step timing on, tc_count runs every class on the caller's stream one after
    another (no side stream); the count is the same as in the overlapped call."""
    g, r, _, _ = case("rmat17_ef32")
    say("[parity] step-timed tc_count on rmat17_ef32")
    rp, ci = upload(g, tc_lib)
    assert tc_lib.tc_count(rp, ci) == r.triangles
    assert tc_lib.tc_last_call_info()["side_stream"] == 1
    tc_lib.tc_profile_read(reset=True)
    tc_lib.tc_profile_enable(True)
    try:
        got = tc_lib.tc_count(rp, ci)
        info = tc_lib.tc_last_call_info()
    finally:
        tc_lib.tc_profile_enable(False)
    steps, calls = tc_lib.tc_profile_read(reset=True)
    assert got == r.triangles
    assert info["side_stream"] == 0 and info["hubs"] > 0
    assert calls == 1 and steps["isect_block"] > 0 and steps["isect_hub"] > 0

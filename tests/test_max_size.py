"""Counting near the size limit: a graph of more than 2^31 stored entries, the range where
32-bit entry offsets have their top bit set, counted on the GPU against closed forms.

The graph is a disjoint union of complete graphs K_k and one book K_{1,1,q} (vertices r
and h joined to each other and to q pages).  Rooted at its smallest ID, K_k puts one
vertex on level 0 and k - 1 on level 1, so it has C(k-1, 2) horizontal edges, C(k-1, 2)
apexes on another level (the root, once per cover edge) and C(k-1, 3) same-level
triangles, each seen from its three edges.  The book's root r is alone on level 0; h and
the pages share level 1, so the q edges {h, page} are horizontal, each with r as its
only apex.  The closed forms are pinned to the oracle on a small member of the same
family (CPU); the large one puts the lane, wavefront and workgroup classes and the hub
pass (r and h form the top degree class; h stages the q cover edges) beyond entry 2^31.
Per-vertex counts are left out at that size: they add three atomics per triangle (about
6.7e10 here).
"""
import math
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

# K_64 bulk first (2.18e9 entries), then K_1, K_2, K_17 (lane class), K_700 (workgroup
# class) and a book whose r and h (degree 100 001) are the only hubs, all past entry 2^31.
PARTS_BIG = [(64, 540_000), (1, 1000), (2, 1000), (17, 20_000), (700, 200)]
PAGES_BIG = 100_000
PARTS_SMALL = [(64, 3), (1, 5), (2, 4), (17, 6), (40, 2), (5, 7), (3, 2)]
PAGES_SMALL = 30


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def closed_forms(parts, q):
    T = sum(c * math.comb(k, 3) for k, c in parts) + q
    S = sum(c * math.comb(k - 1, 2) for k, c in parts) + q
    c2 = sum(c * 3 * math.comb(k - 1, 3) for k, c in parts)
    roots = sum(c for _, c in parts) + (1 if q else 0)
    depth = 1 if q or any(k >= 2 and c for k, c in parts) else 0
    return dict(T=T, S=S, c1=S, c2=c2, roots=roots, depth=depth)


def closed_form_levels(parts, q):
    chunks = []
    for k, c in parts:
        one = np.ones(k, dtype=np.uint32)
        one[0] = 0
        chunks.append(np.tile(one, c))
    if q:
        b = np.ones(q + 2, dtype=np.uint32)
        b[0] = 0
        chunks.append(b)
    return np.concatenate(chunks)


def closed_form_per_vertex(parts, q):
    chunks = [np.full(k * c, math.comb(k - 1, 2), dtype=np.uint64) for k, c in parts]
    if q:
        b = np.ones(q + 2, dtype=np.uint64)
        b[:2] = q
        chunks.append(b)
    return np.concatenate(chunks)


def test_clique_union_equals_edge_list_construction():
    # The vectorised builder gives the same CSR as the generic edge-list builder.
    parts, q = [(4, 3), (1, 2), (2, 2), (6, 1)], 5
    edges, base = [], 0
    for k, c in parts:
        for _ in range(c):
            edges += [(base + i, base + j) for i in range(k) for j in range(i + 1, k)]
            base += k
    r, h = base, base + 1
    edges += [(r, h)] + [(r, base + 2 + i) for i in range(q)] + [(h, base + 2 + i) for i in range(q)]
    ref = gg.from_edges(base + 2 + q, edges)
    got = gg.clique_union(parts, q, chunk_entries=7)  # several fill chunks per part
    assert np.array_equal(got.rowptr, ref.rowptr) and np.array_equal(got.colidx, ref.colidx)


def test_closed_forms_match_oracle():
    g = gg.clique_union(PARTS_SMALL, PAGES_SMALL)
    assert oracle.check_csr(g) == 0
    r = oracle.cetc_seq(g, per_vertex=True)
    _, c1, c2 = oracle.cetc_sm(g, r.level)
    f = closed_forms(PARTS_SMALL, PAGES_SMALL)
    assert (r.triangles, r.cover_edges, c1, c2) == (f["T"], f["S"], f["c1"], f["c2"])
    assert np.array_equal(r.level, closed_form_levels(PARTS_SMALL, PAGES_SMALL))
    assert r.depth == f["depth"]
    assert np.array_equal(r.per_vertex, closed_form_per_vertex(PARTS_SMALL, PAGES_SMALL))
    # the split variant: G0 holds each K_k's level-1 clique K_{k-1} (t0 = C(k-1, 3)); every
    # other triangle has the root as its apex (t1 = C(k-1, 2), and q in the book)
    t0 = sum(c * math.comb(k - 1, 3) for k, c in PARTS_SMALL)
    assert oracle.cetc_split(g, r.level) == (f["T"], t0, f["S"])


def test_big_instance_crosses_2_31_before_its_small_parts():
    entries_bulk = 64 * 63 * PARTS_BIG[0][1]
    assert entries_bulk > (1 << 31)
    total = sum(k * (k - 1) * c for k, c in PARTS_BIG) + 4 * PAGES_BIG + 2
    assert total < (1 << 32) - (1 << 20)


def test_big_instance_hubs_are_the_book_spine():
    # The default hub rule (256 hubs, degree class >= class(4096)) on the large instance's
    # degrees picks exactly r and h, the two vertices of degree q + 1.
    import bench
    d = np.concatenate([np.full(k * c, k - 1, np.int64) for k, c in PARTS_BIG]
                       + [np.full(2, PAGES_BIG + 1), np.full(PAGES_BIG, 2)])
    hubs = np.flatnonzero(bench.hub_set(d, 256, 4096))
    spine = sum(k * c for k, c in PARTS_BIG)
    assert hubs.tolist() == [spine, spine + 1]


@pytest.mark.gpu
def test_more_than_2_31_entries(tc_lib):
    import torch

    say(f"[max-size] building K_k union + book of {PAGES_BIG} pages")
    g = gg.clique_union(PARTS_BIG, PAGES_BIG)
    f = closed_forms(PARTS_BIG, PAGES_BIG)
    say(f"[max-size] n={g.n} m={g.nnz} (2^31 = {1 << 31}); uploading")
    assert g.nnz > (1 << 31)
    rp = torch.from_numpy(g.rowptr.view(np.int32)).to("cuda")
    ci = torch.from_numpy(g.colidx.view(np.int32)).to("cuda")
    torch.cuda.synchronize()
    del g

    say("[max-size] tc_validate_csr")
    assert tc_lib.tc_validate_csr(rp, ci) == 0

    say("[max-size] tc_count (pruned, hub pass)")
    assert tc_lib.tc_count(rp, ci) == f["T"]
    info = tc_lib.tc_last_call_info()
    assert info["hubs"] == 2 and info["hub_items"] > 0 and info["cover_edges"] == f["S"]

    say("[max-size] tc_count_ex (full form, levels)")
    stats, level = tc_lib.tc_count_ex(rp, ci, want_levels=True)
    assert stats.triangles == f["T"] and stats.cover_edges == f["S"]
    assert stats.c1 == f["c1"] and stats.c2 == f["c2"]
    assert stats.depth == f["depth"] and stats.num_roots == f["roots"]
    expect = closed_form_levels(PARTS_BIG, PAGES_BIG)
    assert np.array_equal(level.cpu().numpy().view(np.uint32), expect)
    say(f"[max-size] ok: T={stats.triangles} |S|={stats.cover_edges}")

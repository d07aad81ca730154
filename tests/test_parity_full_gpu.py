"""GPU parity at the full measured sizes, in the launch configuration bench.py times.

For R-MAT scale 22, the triangulated 4096 x 4096 grid with 1% deletions, Erdős–Rényi
2^22 and R-MAT scale 10, the GPU's T, c1, c2 and |S| must equal the oracle's stored
results (tests/golden/full_size_counts.json, written by make_full_counts.py from the
oracle alone), and the GPU's BFS level of every vertex must equal the oracle's BFS run
here on the host.  For the 4096-graph batch, every member's count, from the batched
launch and from its own tc_count call, must equal the oracle's stored count
(tests/golden/batch4096_counts.json).  Per-vertex counts at full size sum to 3 T and
agree, on the largest-degree vertex and a seeded sample, with a count of the edges among
each sampled vertex's neighbours.
"""
import json
import os
import sys

import numpy as np
import pytest
import torch

import oracle
from tests.workloads import BATCH_BASE_SEED, WORKLOADS, batch4096

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "full_size_counts.json")))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def edges_among_neighbours(g, v):
    """Edges between two neighbours of v (the triangles through v): every entry of a
    neighbour's row that is itself a neighbour of v, halved."""
    rp = g.rowptr.astype(np.int64)
    nb = g.colidx[rp[v]:rp[v + 1]].astype(np.int64)
    mark = np.zeros(g.n, dtype=bool)
    mark[nb] = True
    starts, lens = rp[nb], rp[nb + 1] - rp[nb]
    total = int(lens.sum())
    if total == 0:
        return 0
    idx = np.repeat(starts - np.concatenate(([0], np.cumsum(lens)[:-1])), lens) + np.arange(total)
    hits = int(mark[g.colidx[idx]].sum())
    assert hits % 2 == 0
    return hits // 2


@pytest.mark.parametrize("name", ["rmat10", "er22", "grid4096", "rmat22"])
def test_full_size_matches_oracle(tc_lib, name):
    ref = GOLDEN[name]
    say(f"[full] generating {name}")
    g = WORKLOADS[name]()
    assert (g.n, g.nnz) == (ref["n"], ref["nnz"])
    say(f"[full] tc_count_ex {name}: n={g.n} m={g.nnz}")
    rp, ci = tc_lib.to_device(g.rowptr, g.colidx)
    stats, level = tc_lib.tc_count_ex(rp, ci, want_levels=True)
    assert stats.triangles == ref["triangles"]
    assert stats.c1 == ref["c1"] and stats.c2 == ref["c2"]
    assert stats.cover_edges == ref["cover_edges"]
    assert stats.depth == ref["depth"]
    say(f"[full] oracle BFS {name}")
    lv_ref, depth = oracle.bfs_levels(g)
    assert np.array_equal(level.cpu().numpy().view(np.uint32), lv_ref)
    assert oracle.cover_edges(g, lv_ref) == ref["cover_edges"]
    assert tc_lib.tc_count(rp, ci) == ref["triangles"]
    # the split's two terms from the pruned pass: t1 = c1 and 3 t0 = c2 of CETC-SM (both
    # identities pinned on the CPU against the oracle's own CETC-Seq-S)
    t0, t1 = tc_lib.tc_count_split(rp, ci)
    assert t1 == ref["c1"] and 3 * t0 == ref["c2"]
    # per-vertex counts at full size: they sum to 3 T, and the largest-degree vertex and
    # 31 seeded others have t(v) = the edges among their neighbours, counted here from
    # that definition
    say(f"[full] tc_count_per_vertex {name}")
    tri = tc_lib.as_u64(tc_lib.tc_count_per_vertex(rp, ci))
    assert int(tri.sum()) == 3 * ref["triangles"]
    deg = np.diff(g.rowptr.astype(np.int64))
    rng = np.random.default_rng(2403)
    cand = np.flatnonzero(deg >= 2)
    sample = [int(np.argmax(deg))] + [int(v) for v in rng.choice(cand, 31, replace=False)]
    for v in sample:
        assert int(tri[v]) == edges_among_neighbours(g, v), f"vertex {v} (degree {deg[v]})"


def test_batch4096_every_member(tc_lib):
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "batch4096_counts.json")))
    say("[full] generating the 4096-graph batch")
    b = batch4096()
    assert b.num_graphs == ref["num_graphs"] and ref["base_seed"] == BATCH_BASE_SEED
    assert [g.num_edges for g in (b.graph(i) for i in range(b.num_graphs))] == ref["input_edges"]
    rp, ci = tc_lib.to_device(b.rowptr_cat, b.colidx_cat)
    ro = torch.from_numpy(b.row_off).cuda()
    co = torch.from_numpy(b.col_off).cuda()
    rows = int(b.rowptr_cat.shape[0])
    ws = torch.empty(tc_lib.tc_count_batch_workspace_size(b.num_graphs, rows,
                                                              int(b.colidx_cat.shape[0])),
                     dtype=torch.uint8, device="cuda")
    say("[full] tc_count_batch 4096 graphs")
    counts = tc_lib.as_u64(tc_lib.tc_count_batch(rp, ci, ro, co, total_rows=rows, workspace=ws))
    want = np.array(ref["triangles"], dtype=np.uint64)
    bad = np.flatnonzero(counts != want)
    assert bad.size == 0, f"{bad.size} members differ from the oracle, first {bad[:8].tolist()}"
    say("[full] every member through tc_count against the oracle")
    for i in range(b.num_graphs):
        gi = b.graph(i)
        r1, c1 = tc_lib.to_device(gi.rowptr, gi.colidx)
        assert tc_lib.tc_count(r1, c1) == int(want[i]), f"member {i}"

"""GPU parity at the full measured sizes, in the launch configuration bench.py times.

For R-MAT scale 22, the triangulated 4096 x 4096 grid with 1% deletions, Erdős–Rényi
2^22 and R-MAT scale 10, the GPU's T, c1, c2 and |S| must equal the oracle's stored
results (tests/golden/full_size_counts.json, written by make_full_counts.py from the
oracle alone), and the GPU's BFS level of every vertex must equal the oracle's BFS run
here on the host.  For the 4096-graph batch, a seeded sample of members is checked one
by one against the oracle and every member against tc_count.
"""
import json
import os
import sys

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
from tests.workloads import WORKLOADS

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "full_size_counts.json")))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


def test_batch4096_sampled_members(tc_lib):
    say("[full] generating the 4096-graph batch")
    b = gg.make_batch(4096, gg.config_seed(3))
    rp, ci = tc_lib.to_device(b.rowptr_cat, b.colidx_cat)
    ro = torch.from_numpy(b.row_off).cuda()
    co = torch.from_numpy(b.col_off).cuda()
    rows = int(b.rowptr_cat.shape[0])
    ws = torch.empty(tc_lib.tc_count_batch_workspace_size(b.num_graphs, rows,
                                                              int(b.colidx_cat.shape[0])),
                     dtype=torch.uint8, device="cuda")
    say("[full] tc_count_batch 4096 graphs")
    counts = tc_lib.as_u64(tc_lib.tc_count_batch(rp, ci, ro, co, total_rows=rows, workspace=ws))
    rng = np.random.default_rng(4096)
    sample = sorted(set(rng.choice(b.num_graphs, 48, replace=False).tolist()) |
                    {int(np.argmax(np.diff(b.col_off)))})  # plus the largest member
    for i in sample:
        assert int(counts[i]) == oracle.count(b.graph(i)), f"member {i}"
    say("[full] every member against tc_count")
    for i in range(b.num_graphs):
        gi = b.graph(i)
        r1, c1 = tc_lib.to_device(gi.rowptr, gi.colidx)
        assert tc_lib.tc_count(r1, c1) == int(counts[i]), f"member {i}"

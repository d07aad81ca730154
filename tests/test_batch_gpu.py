"""GPU parity of the batched path: tc_count_batch against the oracle per graph, with
empty and one-vertex graphs inside the batch, a caller workspace, and replays of a
captured HIP graph (each replay checked against the eager result)."""
import sys

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed_graphs():
    gs = [gg.empty_graph(0), gg.complete(12), gg.empty_graph(1), gg.wheel(700),
          gg.tri_grid(20, 31, 0.02, 1), gg.empty_graph(9), gg.rmat(13, 32, 77),
          gg.friendship(40), gg.erdos_renyi(3000, 6, 4)]
    b = gg.make_batch(48, 4004, log2_min=6, log2_max=12)
    gs += [b.graph(i) for i in range(b.num_graphs)]
    return gg.pack(gs)


def upload_batch(b):
    import paper_2403_02997_amd as tcm
    rp, ci = tcm.to_device(b.rowptr_cat, b.colidx_cat)
    ro = torch.from_numpy(b.row_off).cuda()
    co = torch.from_numpy(b.col_off).cuda()
    return rp, ci, ro, co


_expected = {}


def expected(b, key):
    if key not in _expected:
        _expected[key] = np.array([oracle.count(b.graph(i)) for i in range(b.num_graphs)],
                                  dtype=np.uint64)
    return _expected[key]


def test_batch_matches_oracle(tc_lib):
    b = mixed_graphs()
    say(f"[batch] {b.num_graphs} graphs, {b.total_edges} edges, library workspace")
    exp = expected(b, "mixed")
    rp, ci, ro, co = upload_batch(b)
    counts = tc_lib.tc_count_batch(rp, ci, ro, co, total_rows=b.rowptr_cat.shape[0])
    torch.cuda.synchronize()
    assert np.array_equal(tc_lib.as_u64(counts), exp)


def test_batch_caller_workspace_and_repeat(tc_lib):
    b = mixed_graphs()
    say("[batch] caller workspace, 3 calls")
    exp = expected(b, "mixed")
    rp, ci, ro, co = upload_batch(b)
    rows = b.rowptr_cat.shape[0]
    ws = torch.empty(tc_lib.tc_count_batch_workspace_size(b.num_graphs, rows,
                                                              int(b.colidx_cat.shape[0])),
                     dtype=torch.uint8, device="cuda")
    for _ in range(3):
        counts = tc_lib.tc_count_batch(rp, ci, ro, co, total_rows=rows, workspace=ws)
        torch.cuda.synchronize()
        assert np.array_equal(tc_lib.as_u64(counts), exp)


def test_batch_workspace_too_small_is_refused(tc_lib):
    b = gg.pack([gg.complete(5), gg.wheel(6)])
    rp, ci, ro, co = upload_batch(b)
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(tc_lib.TCError):
        tc_lib.tc_count_batch(rp, ci, ro, co, total_rows=b.rowptr_cat.shape[0], workspace=ws)


def test_batch_single_graph_equals_tc_count(tc_lib):
    g = gg.rmat(15, 16, 9)
    say("[batch] one-graph batch vs tc_count")
    b = gg.pack([g])
    rp, ci, ro, co = upload_batch(b)
    counts = tc_lib.tc_count_batch(rp, ci, ro, co, total_rows=b.rowptr_cat.shape[0])
    torch.cuda.synchronize()
    r1, c1 = tc_lib.to_device(g.rowptr, g.colidx)
    assert int(tc_lib.as_u64(counts)[0]) == tc_lib.tc_count(r1, c1) == oracle.count(g)


def test_batch_hip_graph_replays(tc_lib):
    b = mixed_graphs()
    say("[batch] captured graph, 4 replays")
    exp = expected(b, "mixed")
    rp, ci, ro, co = upload_batch(b)
    rows = b.rowptr_cat.shape[0]
    ws = torch.empty(tc_lib.tc_count_batch_workspace_size(b.num_graphs, rows,
                                                              int(b.colidx_cat.shape[0])),
                     dtype=torch.uint8, device="cuda")
    counts = torch.zeros(b.num_graphs, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside capture
        tc_lib.tc_count_batch(rp, ci, ro, co, total_rows=rows, workspace=ws, counts=counts)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        tc_lib.tc_count_batch(rp, ci, ro, co, total_rows=rows, workspace=ws, counts=counts)
    for rep in range(4):
        counts.fill_(0)
        ws.fill_(255)  # scramble the scratch between replays: nothing may depend on it
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(tc_lib.as_u64(counts), exp), f"replay {rep}"
        # eager work between replays
        eager = tc_lib.tc_count_batch(rp, ci, ro, co, total_rows=rows)
        torch.cuda.synchronize()
        assert np.array_equal(tc_lib.as_u64(eager), exp)

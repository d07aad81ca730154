"""The allocation-free batched entry point (tc_count_batch_noalloc, workspace in the
library's fixed per-device array) against tc_count_batch with a library-allocated
workspace and against the oracle, on two calls in a row, the second with a smaller
batch (the array keeps the first call's contents)."""
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


def upload(b):
    import paper_2403_02997_amd as tcm
    rp, ci = tcm.to_device(b.rowptr_cat, b.colidx_cat)
    return rp, ci, torch.from_numpy(b.row_off).cuda(), torch.from_numpy(b.col_off).cuda()


def check_batch(tc_lib, b, label):
    rows, cols = int(b.rowptr_cat.shape[0]), int(b.colidx_cat.shape[0])
    need = tc_lib.tc_count_batch_workspace_size(b.num_graphs, rows, cols)
    say(f"[noalloc] {label}: {b.num_graphs} graphs, {b.total_edges} edges, workspace {need} B")
    assert need <= tc_lib.NOALLOC_SCRATCH_BYTES
    exp = np.array([oracle.count(b.graph(i)) for i in range(b.num_graphs)], dtype=np.uint64)
    rp, ci, ro, co = upload(b)
    ref = tc_lib.tc_count_batch(rp, ci, ro, co, total_rows=rows)
    got = torch.full((b.num_graphs,), -1, dtype=torch.int64, device="cuda")
    tc_lib.tc_count_batch_noalloc(rp, ci, ro, co, got, total_rows=rows)
    torch.cuda.synchronize()
    assert np.array_equal(tc_lib.as_u64(ref), exp)
    assert np.array_equal(tc_lib.as_u64(got), tc_lib.as_u64(ref))


def test_noalloc_matches_allocating_batch_twice(tc_lib):
    big = gg.make_batch(120, 5005, log2_min=8, log2_max=12)
    extra = [gg.empty_graph(0), gg.complete(40), gg.empty_graph(1), gg.wheel(900),
             gg.tri_grid(30, 41, 0.02, 3), gg.rmat(12, 24, 91), gg.friendship(60)]
    first = gg.pack(extra + [big.graph(i) for i in range(big.num_graphs)])
    check_batch(tc_lib, first, "first call")
    # a smaller second batch: every count must come from this call, not the previous one
    second = gg.pack([big.graph(i) for i in range(0, big.num_graphs, 7)] + [gg.complete(9)])
    check_batch(tc_lib, second, "second call, smaller")


def test_noalloc_refuses_a_batch_beyond_the_array(tc_lib):
    g = gg.rmat(16, 32, 17)
    b = gg.pack([g] * 6)
    rows, cols = int(b.rowptr_cat.shape[0]), int(b.colidx_cat.shape[0])
    assert tc_lib.tc_count_batch_workspace_size(b.num_graphs, rows, cols) > \
        tc_lib.NOALLOC_SCRATCH_BYTES
    rp, ci, ro, co = upload(b)
    got = torch.full((b.num_graphs,), -1, dtype=torch.int64, device="cuda")
    with pytest.raises(tc_lib.TCError):
        tc_lib.tc_count_batch_noalloc(rp, ci, ro, co, got, total_rows=rows)
    torch.cuda.synchronize()
    assert (got == -1).all()  # untouched on error

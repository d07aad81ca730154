"""The autotuner on the GPU: it measures, applies a valid setting under which the count
is unchanged (equal to the oracle's), and a second call reuses the cached setting."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture
def restore_params(tc_lib):
    saved = tc_lib.tc_get_isect_params()
    saved_hubs = tc_lib.tc_get_hub_params()
    yield
    tc_lib.tc_set_isect_params(*saved)
    tc_lib.tc_set_hub_params(*saved_hubs)


def test_autotune_single_graph(tc_lib, restore_params, tmp_path):
    from paper_2403_02997_amd import autotune as at
    g = gg.rmat(13, 16, 21)
    T = oracle.count(g)
    rp, ci = tc_lib.to_device(g.rowptr, g.colidx)
    cache = str(tmp_path / "at.json")
    r = at.autotune(rp, ci, reps=1, cache=cache)
    assert r["measured"] > 1 and at.valid(r["params"]) and len(r["params"]) == 5
    assert tc_lib.tc_get_isect_params() == tuple(r["params"][:4])
    assert tc_lib.tc_get_hub_params()[0] == r["params"][4]
    assert tc_lib.tc_count(rp, ci) == T
    tc_lib.tc_set_isect_params(16, 512, 4096, 1024)
    tc_lib.tc_set_hub_params(0, 4096)
    r2 = at.autotune(rp, ci, reps=1, cache=cache)
    assert r2["measured"] == 0 and tuple(r2["params"]) == tuple(r["params"])
    assert tc_lib.tc_get_isect_params() == tuple(r["params"][:4])
    assert tc_lib.tc_get_hub_params()[0] == r["params"][4]


def test_autotune_batch(tc_lib, restore_params, tmp_path):
    from paper_2403_02997_amd import autotune as at
    b = gg.pack([gg.rmat(8 + (i % 4), 16, 100 + i) for i in range(12)] + [gg.wheel(600)])
    want = np.array([oracle.count(b.graph(i)) for i in range(b.num_graphs)], dtype=np.uint64)
    rp, ci = tc_lib.to_device(b.rowptr_cat, b.colidx_cat)
    ro = torch.from_numpy(b.row_off).cuda()
    co = torch.from_numpy(b.col_off).cuda()
    r = at.autotune_batch(rp, ci, ro, co, reps=1, cache=str(tmp_path / "at.json"))
    assert r["measured"] > 1 and at.valid(r["params"])
    got = tc_lib.as_u64(tc_lib.tc_count_batch(rp, ci, ro, co))
    torch.cuda.synchronize()
    assert np.array_equal(got, want)

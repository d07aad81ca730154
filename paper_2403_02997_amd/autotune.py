"""Autotuner for the intersection class thresholds of the counting kernels.

The staged endpoint x of a cover edge goes to the lane class when d(x) <= lane_max, to
the wavefront class when d(x) <= wave_max, else to the workgroup class, which stages
x's entries in chunks of `chunk` keys and takes `seg` partners per work item
(tc_set_isect_params); for a single graph, the cover edges staged under the up to
max_hubs vertices of the top degree classes go to the hub pass instead
(tc_set_hub_params).  The best setting depends on the degree distribution and on the
device, so this module measures candidates on the caller's own graph (or batch) by
coordinate descent: one parameter at a time over its candidate values, the others held
at the best setting so far.  A setting changes only how the work is divided, never the
result: every candidate must return the counts of the first run, and a mismatch raises.

The chosen setting is cached in a JSON file keyed by the device and a size class of the
workload (log2 of its graphs, rows and stored entries), so that a later call on an input
of the same class reuses it without measuring.  The setting is process-wide; tune only
while no other count is running.
"""
from __future__ import annotations

import json
import math
import os
import time

import torch

from . import tc as _tc

# Settings are tuples in NAMES order: the four class thresholds, then (single graphs
# only) the hub count.
NAMES = ("lane_max", "wave_max", "chunk", "seg", "max_hubs")
CANDIDATES = {
    "lane_max": (4, 8, 16, 32),
    "wave_max": (128, 256, 512),
    "chunk": (2048, 4096, 8192),
    "seg": (256, 512, 1024),
    "max_hubs": (0, 32, 128, 256),
}
ORDER = ("max_hubs", "wave_max", "lane_max", "chunk", "seg")
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2403_02997_amd",
                             "autotune.json")


def valid(p) -> bool:
    """The range tc_set_isect_params (and tc_set_hub_params) accept."""
    lane_max, wave_max, chunk, seg = p[:4]
    hubs_ok = len(p) < 5 or 0 <= p[4] <= 256
    return (0 <= lane_max <= wave_max <= 512 and 0 < chunk <= 16384 and 0 < seg <= 1024
            and hubs_ok)


def apply(p) -> None:
    """Sets the library to setting p (4 values, or 5 with the hub count)."""
    _tc.tc_set_isect_params(*p[:4])
    if len(p) > 4:
        _tc.tc_set_hub_params(int(p[4]), _tc.tc_get_hub_params()[1])


def current(with_hubs: bool) -> tuple:
    p = tuple(_tc.tc_get_isect_params())
    return p + (_tc.tc_get_hub_params()[0],) if with_hubs else p


def device_key() -> str:
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{props.name}|{getattr(props, 'gcnArchName', '')}|{props.multi_processor_count}"


def workload_key(kind: str, rows: int, cols: int, graphs: int = 1) -> str:
    def lg(v):
        return int(math.log2(v)) if v > 0 else -1
    return f"{kind}:g{lg(graphs)}:n{lg(rows)}:m{lg(cols)}"


def load_cache(path: str | None) -> dict:
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            db = json.load(f)
        return db if isinstance(db, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(path: str | None, db: dict) -> None:
    if not path:
        return
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


MIN_GAIN = 0.02  # a candidate must beat the best time so far by this fraction


def descend(measure, start, order=ORDER, candidates=CANDIDATES, min_gain=MIN_GAIN):
    """Coordinate descent.  measure(params) -> (result, seconds); params are tuples in
    NAMES order, as long as `start` (the names past its length are not tuned).  A
    candidate replaces the best setting only when it is faster by more than min_gain
    (a relative margin: run-to-run noise of a few tenths of a percent must not move the
    setting).  Returns (best params, best seconds, number of settings measured).  Raises
    RuntimeError when a setting's result differs from the first one's."""
    best = tuple(int(v) for v in start)
    ref, best_t = measure(best)
    tried = {best}
    for name in order:
        i = NAMES.index(name)
        if i >= len(best):
            continue
        for v in candidates[name]:
            cand = best[:i] + (int(v),) + best[i + 1:]
            if cand in tried or not valid(cand):
                continue
            tried.add(cand)
            res, t = measure(cand)
            if res != ref:
                raise RuntimeError(f"setting {cand} changed the result: {res!r} != {ref!r}")
            if t < best_t * (1.0 - min_gain):
                best, best_t = cand, t
    return best, best_t, len(tried)


def _tune(key: str, run, reps: int, cache: str | None, refresh: bool,
          with_hubs: bool) -> dict:
    db = load_cache(cache)
    hit = db.get(key)
    if (hit and not refresh and valid(tuple(hit["params"]))
            and len(hit["params"]) == (5 if with_hubs else 4)):
        apply(tuple(hit["params"]))
        return {"params": tuple(hit["params"]), "ms": hit["ms"], "measured": 0, "key": key}

    def measure(p):
        apply(p)
        res, _ = run()  # warm-up (and the result)
        times = []
        for _ in range(max(reps, 1)):
            r, t = run()
            if r != res:
                raise RuntimeError(f"setting {p} is not repeatable: {r!r} != {res!r}")
            times.append(t)
        return res, min(times)

    start = current(with_hubs)
    try:
        best, best_t, n = descend(measure, start)
    except BaseException:
        apply(start)
        raise
    apply(best)
    db[key] = {"params": list(best), "ms": round(best_t * 1e3, 4)}
    store_cache(cache, db)
    return {"params": best, "ms": best_t * 1e3, "measured": n, "key": key}


def autotune(rowptr: torch.Tensor, colidx: torch.Tensor, reps: int = 2,
             cache: str | None = DEFAULT_CACHE, refresh: bool = False) -> dict:
    """Tunes and applies the thresholds and the hub count for tc_count on this graph
    (device CSR tensors).  Returns {"params": (lane_max, wave_max, chunk, seg, max_hubs),
    "ms", "measured", "key"}."""
    def run():
        t0 = time.perf_counter()
        c = _tc.tc_count(rowptr, colidx)  # blocking
        return c, time.perf_counter() - t0

    key = device_key() + "|" + workload_key("single", rowptr.numel() - 1, colidx.numel())
    return _tune(key, run, reps, cache, refresh, with_hubs=True)


def autotune_batch(rowptr_cat: torch.Tensor, colidx_cat: torch.Tensor, row_off: torch.Tensor,
                   col_off: torch.Tensor, workspace: torch.Tensor | None = None, reps: int = 2,
                   cache: str | None = DEFAULT_CACHE, refresh: bool = False) -> dict:
    """Tunes and applies the thresholds for tc_count_batch on this batch (the batched
    kernel has no hub pass)."""
    G = row_off.numel() - 1
    counts = torch.empty(max(G, 0), dtype=torch.int64, device=rowptr_cat.device)

    def run():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _tc.tc_count_batch(rowptr_cat, colidx_cat, row_off, col_off, workspace=workspace,
                           counts=counts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return tuple(counts.cpu().tolist()), dt

    key = device_key() + "|" + workload_key("batch", rowptr_cat.numel(), colidx_cat.numel(), G)
    return _tune(key, run, reps, cache, refresh, with_hubs=False)

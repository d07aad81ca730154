#!/usr/bin/env python3
"""Throughput of cover-edge triangle counting on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--gpus 1]

Default workload: batch4096, the headline configuration (input edges/s, batched vs
per-graph launch).  One step is one replay of a captured tc_count_batch over 4096
uneven graphs already resident in HBM (component roots, level BFS, cover-edge
extraction, intersections and the per-graph totals, all inside one persistent kernel);
the timed region brackets exactly K replays with device synchronisations, and value =
input edges of the whole batch (undirected, after cleaning) x K / elapsed seconds.
The same graphs then go through one tc_count call each (on one stream, and spread over
four host threads with a stream each): per_graph_launch and batched_over_per_graph.
Every batched count must equal its per-graph count.

Alongside, per JSON line:
  roofline     : the batched kernel's algorithmic bytes per launch (per member: the BFS,
                 extraction and intersection bytes of the measurement plan, the last the
                 short list of every cover edge plus every list touched by a cover edge
                 once; summed over the 4096 members) over its average launch time, from
                 HIP events recorded on the stream the replays run on, against 8 TB/s
                 HBM.  traffic is the counter-measured HBM bytes per launch stored under
                 profiles/ for the current kernel sources, else null.
  cpu_baseline : the CPU oracle timed on this host on a bounded sample of the batch's
                 members (single-thread CETC-Seq and CETC-SM on every host thread,
                 several runs each, mean and median).
  single_graph : the same figures for one tc_count call on R-MAT scale 22 (the
                 single-graph configuration), unless --no-single-graph.

Single-graph workloads (--workload rmat22 | rmat10 | grid4096 | er22): one step is one
whole tc_count call on a graph already resident in HBM (including the call's own
workspace allocation: the paper charges auxiliary arrays to the algorithm).  Their
roofline is the dominant intersection kernel's bytes over its launch time from step-timed
calls; frac is taken on the measurement plan's intersection bytes for that kernel's
cover edges, with the bytes the pruned kernel streams beside it.  serve: a Poisson
stream of requests through the tc_serve_* server (p50/p99 latency and input edges/s,
every result checked against the oracle's stored count).

--autotune picks the intersection thresholds (tc_set_isect_params) and, for a single
graph, the hub count (tc_set_hub_params) on the workload itself before the warm-up, by
the package's coordinate-descent autotuner; the settings are in config.isect_params and
config.hub_params of every line either way.

Counter helpers (no bench line):
  --calibrate-copy MIB  runs a plain device-to-device copy of MIB MiB three times, the
                        known-size kernel that FETCH_SIZE / WRITE_SIZE are scaled by;
  --traffic-summary     reads the four rocprofv3 --pmc CSVs (bench FETCH_SIZE and
                        WRITE_SIZE passes, copy FETCH_SIZE and WRITE_SIZE passes) and
                        stores the per-launch HBM bytes of each counting kernel in
                        profiles/traffic.json under the current kernel source hash.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "input edges/s for cover-edge TC (bit-exact u64), batched vs per-graph launch"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2403_02997_amd", "csrc")
# The kernel instance tc_count launches for each intersection step (16-byte aligned
# colidx, no per-vertex attribution; the workgroup class in its pruned form).
# the kernel instantiations of the counting call (the fourth template argument, false,
# leaves out the split-term tallies of tc_count_split)
BATCH_KERNEL = "k_batch_main<true>"
KERNEL_OF_STEP = {"isect_lane": "k_isect_lane<false>",
                  "isect_wave": "k_isect_wave<false, true, true, false>",
                  "isect_block": "k_isect_block<false, true, true, false>",
                  "isect_hub": "k_hub_count<8u, false, false>"}

WORKLOAD_TEXT = {
    "rmat10": "R-MAT scale 10, edge factor 16, initiator (0.57,0.19,0.19,0.05), seed 1000",
    "rmat22": "R-MAT scale 22, edge factor 16, initiator (0.57,0.19,0.19,0.05), seed 1001",
    "grid4096": "triangulated 4096x4096 grid, 1% of edges deleted, seed 1002",
    "er22": "Erdos-Renyi G(n=2^22, average degree 32), seed 1003",
    "er14_d256": "Erdos-Renyi G(n=2^14, average degree 256), seed 1004",
    "batch4096": "4096 graphs: half R-MAT (scale 8-16, edge factor 8-32), half Erdos-Renyi "
                 "(n log-uniform in [2^8, 2^16], average degree 4-64), seed 1003",
    "serve": "Poisson request stream: 90% R-MAT scale 12-18, 10% R-MAT scale 22-24, one "
             "R-MAT scale 26 request, edge factor 16, seed 1005",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha() -> str:
    """Hash of every source that defines a counting kernel or its launch shape (all of csrc
    but the host-side call orchestration of api.hip, serve.hip and host_api.h, and the
    clustering-coefficient kernel of cluster.hip, which no counting step runs, and the
    allocation-free entry point of noalloc.hip, which only hands over a workspace): any change
    to how the work is divided or done makes a stored traffic record stale."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".h")) and f not in ("api.hip", "serve.hip", "host_api.h",
                                                    "cluster.hip", "noalloc.hip"):
            h.update(f.encode())
            h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


# ---- algorithmic bytes of the intersection classes ------------------------------------

def degree_class(d: np.ndarray) -> np.ndarray:
    """Monotone quantised log2 of the degree (4 steps per octave), 0 for d = 0."""
    d = d.astype(np.int64)
    out = np.zeros_like(d)
    nz = d > 0
    lg = np.floor(np.log2(d[nz])).astype(np.int64)
    frac = np.where(lg >= 2, (d[nz] >> np.maximum(lg - 2, 0)) & 3, (d[nz] << (2 - np.minimum(lg, 2))) & 3)
    out[nz] = np.minimum(1 + 4 * lg + frac, 127)
    return out


def hub_set(d: np.ndarray, max_hubs: int, min_degree: int) -> np.ndarray:
    """The hubs of tc_count's hub pass (tc_set_hub_params): none on graphs of fewer than
    1024 * min_degree stored entries; else the vertices of degree class >= c*, c* the
    smallest class >= max(class(min_degree), 1) whose vertices and those of the classes
    above number between 1 and max_hubs (no hubs if there is none)."""
    cls = degree_class(d)
    if max_hubs == 0 or len(d) == 0 or int(np.sum(d, dtype=np.int64)) < 1024 * min_degree:
        return np.zeros(len(d), dtype=bool)
    suf = np.cumsum(np.bincount(cls, minlength=128)[::-1])[::-1]
    cmin = max(int(degree_class(np.array([min_degree]))[0]), 1)
    for c in range(cmin, 128):
        if 0 < suf[c] <= max_hubs:
            return cls >= c
    return np.zeros(len(d), dtype=bool)


def class_bytes(g, level: np.ndarray, params, hubs=(0, 0)) -> dict:
    """Per intersection class of tc_count: cover edges and the bytes its kernel has to
    read at least once.  A cover edge {x, y} is staged under x (larger degree class, then
    ID) and streams y's list.  The lane class streams all of N(y) and stages N(x); the
    wavefront and workgroup classes stream only y's other-level neighbours and its
    same-level neighbours above max(x, y), and stage x's other-level neighbours and its
    same-level neighbours above x.  Each staged list counts once.  Cover edges staged
    under a hub (hubs = tc_get_hub_params()) go to the hub pass: each partner y of a hub
    streams N'(y) (its other-level neighbours and its same-level neighbours above y) once,
    looks every entry up in a mask of NW words (4 for at most 128 hubs, else 8) and reads
    its own mask H(y); building the masks reads every hub's S list (its other-level
    neighbours and same-level neighbours above it) and writes NW words per vertex."""
    lane_max, wave_max = params[0], params[1]
    d = g.degrees().astype(np.int64)
    hub = hub_set(d, hubs[0], hubs[1])
    rp = g.rowptr.astype(np.int64)
    rows = np.repeat(np.arange(g.n, dtype=np.int64), d)
    cols = g.colidx.astype(np.int64)
    par = (level & 1).astype(np.int8)
    same_entry = par[rows] == par[cols]
    cs = np.concatenate([[0], np.cumsum(same_entry, dtype=np.int64)])
    del same_entry
    m = (par[rows] == par[cols]) & (rows < cols)
    u, v = rows[m], cols[m]
    del m
    key = rows * (1 << 32) + cols  # sorted: rows ascending, columns ascending within
    del rows, cols
    cls_d = degree_class(d)
    key_u = cls_d[u] * (1 << 32) + u
    key_v = cls_d[v] * (1 << 32) + v
    x = np.where(key_u > key_v, u, v)
    y = np.where(key_u > key_v, v, u)
    del u, v, key_u, key_v
    dx = d[x]
    hx = hub[x]
    out = {}
    for name, sel in (("isect_lane", (dx <= lane_max) & ~hx),
                      ("isect_wave", (dx > lane_max) & (dx <= wave_max) & ~hx),
                      ("isect_block", (dx > wave_max) & ~hx)):
        xs = np.unique(x[sel])
        ys = y[sel]
        if name == "isect_lane":
            streamed = int(d[ys].sum())
            staged = int(d[xs].sum())
        else:
            vmax = np.maximum(x[sel], ys)
            pos = np.searchsorted(key, ys * (1 << 32) + vmax, side="right")
            skip = cs[pos] - cs[rp[ys]]
            streamed = int((d[ys] - skip).sum())
            same_x = cs[rp[xs + 1]] - cs[rp[xs]]
            above = cs[rp[xs + 1]] - cs[np.searchsorted(key, xs * (1 << 32) + xs, side="right")]
            staged = int((d[xs] - same_x + above).sum())
        # the measurement plan's intersection bytes for these cover edges: the shorter
        # list of each once, every list they touch once
        xe, ye = x[sel], y[sel]
        touched = np.unique(np.concatenate([xe, ye]))
        b_int = 4 * int(np.minimum(d[xe], d[ye]).sum()) + 4 * int(d[touched].sum())
        out[name] = {"cover_edges": int(sel.sum()), "bytes": 4 * (streamed + staged),
                     "plan_bytes": b_int}
    nh = int(hub.sum())
    hb = 0
    if nh:
        nw = 4 if nh <= 128 else 8
        vs = np.arange(g.n, dtype=np.int64)
        same_v = cs[rp[1:]] - cs[rp[:-1]]
        above_v = cs[rp[1:]] - cs[np.searchsorted(key, vs * (1 << 32) + vs, side="right")]
        nprime = d - same_v + above_v  # N'(v), also S(v)
        ys = np.unique(y[hx])
        hb = int((4 + 4 * nw) * nprime[ys].sum() + 4 * nw * len(ys)
                 + 4 * nprime[hub].sum() + 4 * nw * g.n)
    xe, ye = x[hx], y[hx]
    touched = np.unique(np.concatenate([xe, ye]))
    out["isect_hub"] = {"cover_edges": int(hx.sum()), "bytes": hb,
                        "plan_bytes": 4 * int(np.minimum(d[xe], d[ye]).sum())
                        + 4 * int(d[touched].sum())}
    return out


def plan_bytes(rowptr: np.ndarray, colidx: np.ndarray, level: np.ndarray) -> dict:
    """Algorithmic bytes of the counting path on one graph, or on a disjoint union of
    graphs with global IDs (each term is a sum over vertices or edges): the BFS reads the
    CSR once and writes the levels, 4 (n + 1) + 4 nnz + 4 n; the extraction reads the CSR
    once and writes the cover edges, 4 (n + 1) + 4 nnz + 8 |S|; the intersections read
    the shorter list of every cover edge once and every list that a cover edge touches
    once, B_int = 4 sum_S min(d_u, d_v) + 4 sum_{x in V(S)} d_x (B_merge = 4 sum_S
    (d_u + d_v), the two-pointer merge, beside it); the output is 8 bytes per graph
    (added by the caller)."""
    n = int(rowptr.shape[0]) - 1
    d = np.diff(rowptr.astype(np.int64))
    rows = np.repeat(np.arange(n, dtype=np.int64), d)
    cols = colidx.astype(np.int64)
    lv = level.astype(np.int64)
    h = (rows < cols) & (lv[rows] == lv[cols])
    u, v = rows[h], cols[h]
    del rows, cols, h
    touched = np.zeros(n, dtype=bool)
    touched[u] = True
    touched[v] = True
    nnz = int(colidx.shape[0])
    S = int(u.shape[0])
    short = int(np.minimum(d[u], d[v]).sum())
    merge = int((d[u] + d[v]).sum())
    return {"cover_edges": S, "bfs": 4 * (n + 1) + 4 * nnz + 4 * n,
            "extract": 4 * (n + 1) + 4 * nnz + 8 * S,
            "intersect": 4 * short + 4 * int(d[touched].sum()), "merge": 4 * merge}


def stored_traffic(workload: str, kernel: str, settings: dict):
    """Counter-measured HBM bytes per launch of `kernel` on `workload`, if recorded for the
    current kernel sources and the same class and hub settings, else None."""
    path = os.path.join(PROFILES, "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(workload, {}).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha") != source_sha():
        return None
    if any(rec.get(k) != v for k, v in settings.items()):
        return None
    return rec.get("hbm_bytes_per_launch")


def current_settings(tcm) -> dict:
    return {"isect_params": list(tcm.tc_get_isect_params()),
            "hub_params": list(tcm.tc_get_hub_params())}


# ---- CPU baseline: the oracle on a bounded sample ----------------------------------------

def cpu_baseline(g, target_s: float):
    import oracle

    t0 = time.perf_counter()
    level, _ = oracle.bfs_levels(g)
    t_bfs = time.perf_counter() - t0
    d = g.degrees()
    rows = np.repeat(np.arange(g.n, dtype=np.int64), d)
    cols = g.colidx.astype(np.int64)
    m = (level[rows] == level[cols]) & (rows < cols)
    work_u = np.bincount(rows[m], weights=(d[rows[m]] + d[cols[m]]).astype(np.float64),
                         minlength=g.n)
    del rows, cols, m
    cum = np.cumsum(work_u)
    W = float(cum[-1]) if g.n else 0.0
    threads = oracle.max_threads()
    if W == 0:
        return None

    def run(a, b):
        t = time.perf_counter()
        oracle.cetc_sm_range(g, level, a, b)
        return time.perf_counter() - t

    # calibrate on ~0.2 % of the merge work, then size the sample to ~target_s
    b0 = int(np.searchsorted(cum, 0.002 * W)) + 1
    t_cal = run(0, b0)
    rate = (cum[b0 - 1] / max(t_cal, 1e-6))
    want = min(W - cum[b0 - 1], rate * target_s)
    b1 = int(np.searchsorted(cum, cum[b0 - 1] + want)) + 1
    b1 = min(max(b1, b0 + 1), g.n)
    t_s = run(b0, b1)
    w_s = float(cum[b1 - 1] - cum[b0 - 1])
    t_full = t_bfs + W * t_s / max(w_s, 1.0)
    return {
        "value": g.num_edges / t_full,
        "unit": "input edges/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle BFS restart loop on the whole graph (1 thread, {t_bfs:.2f} s) + "
                   f"CETC-SM edge loop over first endpoints [{b0}, {b1}) = "
                   f"{100.0 * w_s / W:.1f}% of the merge work ({t_s:.2f} s, {threads} threads), "
                   f"extrapolated linearly in merge work to {t_full:.1f} s for the whole graph"),
    }


# ---- single-graph workloads ----------------------------------------------------------------

def bench_single(args, tcm, torch):
    from tests.workloads import WORKLOADS

    t = time.perf_counter()
    g = WORKLOADS[args.workload]()
    log(f"[bench] generated {args.workload}: n={g.n} input edges={g.num_edges} "
        f"({time.perf_counter() - t:.1f}s)")
    rp, ci = tcm.to_device(g.rowptr, g.colidx)
    torch.cuda.synchronize()
    tuned = None
    if args.autotune:
        from paper_2403_02997_amd import autotune as at
        t = time.perf_counter()
        tuned = at.autotune(rp, ci, reps=2, cache=None)
        log(f"[bench] autotune: {tuned['params']} after {tuned['measured']} settings "
            f"({time.perf_counter() - t:.1f}s)")
    for i in range(args.warmup):
        tcm.tc_count(rp, ci)
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = None
    for _ in range(args.steps):
        T = tcm.tc_count(rp, ci)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    forward = tcm.tc_last_call_info()["forward"]
    elapsed = t1 - t0
    log(f"[bench] timed {args.steps} steps: {elapsed * 1e3 / args.steps:.3f} ms/step")
    # Step breakdown and roofline: further calls with step timing on.  The library then
    # runs the intersection classes one after another on the caller's stream (in the
    # timed steps the wavefront class and the hub pass run beside the workgroup class),
    # so each step's events bracket its own kernels.
    tcm.tc_profile_read(reset=True)
    tcm.tc_profile_enable(True)
    for _ in range(args.profile_steps):
        assert tcm.tc_count(rp, ci) == T
    tcm.tc_profile_enable(False)
    prof, calls = tcm.tc_profile_read(reset=True)
    log(f"[bench] {calls} step-timed calls")

    stats, level = tcm.tc_count_ex(rp, ci, want_levels=True)
    assert stats.triangles == T
    level_np = level.cpu().numpy().view(np.uint32)
    params = tcm.tc_get_isect_params()
    hubs = tcm.tc_get_hub_params()
    # the forward ordering runs the same kernels with every vertex on one level
    cb = class_bytes(g, np.zeros_like(level_np) if forward else level_np, params, hubs)
    steps_ms = {k: v / max(calls, 1) for k, v in prof.items()}
    isect = {k: steps_ms.get(k, 0.0) for k in KERNEL_OF_STEP}
    dom = max(isect, key=isect.get)
    dom_ms = isect[dom]
    achieved = cb[dom]["plan_bytes"] / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else 0.0
    streamed = cb[dom]["bytes"] / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else 0.0
    traffic = stored_traffic(args.workload, KERNEL_OF_STEP[dom], current_settings(tcm))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "kernel": KERNEL_OF_STEP[dom], "avg_launch_ms": round(dom_ms, 4),
                "timed_in": f"{calls} step-timed calls (intersection classes one after another)",
                "algorithmic_bytes_per_launch": cb[dom]["plan_bytes"],
                "algorithmic_bytes": "shorter list of each of the kernel's cover edges once "
                                     "plus every list they touch once",
                "pruned_bytes_per_launch": cb[dom]["bytes"],
                "pruned_gbs": round(streamed, 1),
                "traffic_gbs": (round(traffic / (dom_ms * 1e-3) / 1e9, 1)
                                if traffic and dom_ms > 0 else None)}
    out = {
        "metric": METRIC,
        "value": g.num_edges * args.steps / elapsed,
        "unit": "input edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "graph": WORKLOAD_TEXT[args.workload],
                   "n": g.n, "input_edges": g.num_edges, "triangles": T,
                   "cover_edges": stats.cover_edges,
                   "covering_ratio": round(stats.cover_edges / max(g.num_edges, 1), 4),
                   "bfs_depth": stats.depth, "components": stats.num_roots,
                   "isect_params": list(params), "hub_params": list(hubs),
                   "forward_threshold": tcm.tc_get_forward_threshold(),
                   "forward_ordering": bool(forward),
                   "hubs": int(hub_set(g.degrees(), *hubs).sum()),
                   "autotuned": tuned is not None},
        "triangles_per_s": T * args.steps / elapsed,
        "steps_ms": {k: round(v, 4) for k, v in steps_ms.items()},
        "isect_classes": {k: {"cover_edges": v["cover_edges"], "pruned_bytes": v["bytes"],
                              "plan_bytes": v["plan_bytes"],
                              "ms": round(isect.get(k, 0.0), 4)} for k, v in cb.items()},
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_seconds)
    if args.per_vertex:
        out["per_vertex"] = bench_per_vertex(args, tcm, torch, rp, ci, g, T)
    isect_ms = sum(isect.values())
    out["isect_classes"]["isect_all"] = {
        "plan_bytes": sum(v["plan_bytes"] for v in cb.values()),
        "ms": round(isect_ms, 4)}
    return out


def bench_per_vertex(args, tcm, torch, rp, ci, g, T) -> dict:
    """t(v) for every vertex (tc_count_per_vertex) and C(v) from it (tc_local_clustering):
    one untimed call, then --per-vertex calls timed like the count's steps."""
    tri = tcm.tc_count_per_vertex(rp, ci)
    assert int(tri.sum().item()) == 3 * T
    torch.cuda.synchronize()
    k = args.per_vertex
    t0 = time.perf_counter()
    for _ in range(k):
        tri = tcm.tc_count_per_vertex(rp, ci)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(k):
        cc = tcm.tc_local_clustering(rp, tri)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    assert int(tri.sum().item()) == 3 * T and cc.numel() == g.n
    ms = (t1 - t0) * 1e3 / k
    log(f"[bench] per-vertex counts: {ms:.3f} ms/call")
    # step breakdown: the same calls with step timing on (classes one after another)
    tcm.tc_profile_read(reset=True)
    tcm.tc_profile_enable(True)
    for _ in range(k):
        tcm.tc_count_per_vertex(rp, ci)
    tcm.tc_profile_enable(False)
    prof, calls = tcm.tc_profile_read(reset=True)
    return {"calls": k, "ms_per_call": round(ms, 4),
            "input_edges_per_s": g.num_edges / (ms * 1e-3),
            "counted_triangles": T, "attributions": 3 * T,
            "clustering_ms_per_call": round((t2 - t1) * 1e3 / k, 4),
            "steps_ms": {key: round(v / max(calls, 1), 4) for key, v in prof.items()}}


# ---- batched workload ------------------------------------------------------------------------

def batch_levels(tcm, dev):
    """Levels of every member, from one tc_count_ex call per member (the levels are
    checked against the oracle's BFS in the parity tests)."""
    out = []
    for r, c in dev:
        if c.numel() == 0:
            out.append(np.zeros(r.numel() - 1, dtype=np.uint32))
            continue
        _, lv = tcm.tc_count_ex(r, c, want_levels=True)
        out.append(lv.cpu().numpy().view(np.uint32))
    return out


def batch_plan_bytes(b, levels, chunk_entries: int = 1 << 27) -> dict:
    """plan_bytes summed over the members, computed over groups of members joined into
    one disjoint union with global IDs."""
    tot = {"cover_edges": 0, "bfs": 0, "extract": 0, "intersect": 0, "merge": 0,
           "output": 8 * b.num_graphs}
    g0 = 0
    while g0 < b.num_graphs:
        g1, ent = g0, 0
        while g1 < b.num_graphs and (g1 == g0 or ent + int(b.col_off[g1 + 1] - b.col_off[g1])
                                      <= chunk_entries):
            ent += int(b.col_off[g1 + 1] - b.col_off[g1])
            g1 += 1
        degs, cols, lvs, base = [], [], [], 0
        for i in range(g0, g1):
            gi = b.graph(i)
            degs.append(np.diff(gi.rowptr.astype(np.int64)))
            cols.append(gi.colidx.astype(np.int64) + base)
            lvs.append(levels[i])
            base += gi.n
        d = np.concatenate(degs)
        rp = np.zeros(d.shape[0] + 1, dtype=np.int64)
        np.cumsum(d, out=rp[1:])
        r = plan_bytes(rp, np.concatenate(cols), np.concatenate(lvs))
        # each member has its own n_g + 1 rowptr entries, read by both steps
        r["bfs"] += 4 * (g1 - g0 - 1)
        r["extract"] += 4 * (g1 - g0 - 1)
        for k, v in r.items():
            tot[k] += v
        g0 = g1
    tot["total"] = tot["bfs"] + tot["extract"] + tot["intersect"] + tot["output"]
    return tot


def cpu_baseline_batch(b, target_s: float, reps: int = 3):
    """The oracle on a bounded sample of the batch's members, as it stands: CETC-Seq on
    one thread (BFS restart loop and edge loop) and the BFS restart loop plus CETC-SM on
    every host thread, `reps` runs of each over the same sample; the members are taken
    every k-th in order of size, k sized from a calibration run so that all runs together
    take about target_s."""
    import oracle

    threads = oracle.max_threads()
    ent = np.diff(b.col_off)
    by_size = np.argsort(ent, kind="stable")

    def run_single(ids):
        t = time.perf_counter()
        for i in ids:
            oracle.cetc_seq(b.graph(int(i)))
        return time.perf_counter() - t

    def run_omp(ids):
        t = time.perf_counter()
        for i in ids:
            g = b.graph(int(i))
            lv, _ = oracle.bfs_levels(g)
            oracle.cetc_sm(g, lv)
        return time.perf_counter() - t

    cal = by_size[::256]
    t_cal = run_single(cal) + run_omp(cal)
    per_edge = t_cal / max(int(ent[cal].sum()) // 2, 1)
    want_edges = target_s / (reps * max(per_edge, 1e-12))
    k = max(1, int(np.ceil(b.total_edges / max(want_edges, 1.0))))
    sample = by_size[k // 2::k]
    edges = int(ent[sample].sum()) // 2
    ts = [run_single(sample) for _ in range(reps)]
    to = [run_omp(sample) for _ in range(reps)]
    rate = lambda t: edges / t  # noqa: E731
    return {
        "value": edges / float(np.median(to)),
        "unit": "input edges/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{len(sample)} of {b.num_graphs} members (every {k}th by size, "
                   f"{edges} input edges = {100.0 * edges / b.total_edges:.2f}% of the batch); "
                   f"{reps} runs each of the BFS restart loop + CETC-SM edge loop on "
                   f"{threads} threads (value: median) and of CETC-Seq on one thread"),
        "omp_threads": threads,
        "omp_edges_per_s_median": rate(float(np.median(to))),
        "omp_edges_per_s_mean": edges * reps / float(np.sum(to)),
        "single_thread_edges_per_s_median": rate(float(np.median(ts))),
        "single_thread_edges_per_s_mean": edges * reps / float(np.sum(ts)),
        "runs_s": {"omp": [round(t, 3) for t in to], "single_thread": [round(t, 3) for t in ts]},
    }


def per_graph_streams(tcm, torch, dev, nstreams: int):
    """All members through tc_count, spread round-robin over nstreams host threads, each
    with its own stream (tc_count blocks its caller until its stream is done)."""
    import threading

    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    out = np.zeros(len(dev), dtype=np.uint64)
    errors = []

    def work(k):
        try:
            for i in range(k, len(dev), nstreams):
                out[i] = tcm.tc_count(dev[i][0], dev[i][1], stream=streams[k])
        except Exception as e:  # noqa: BLE001
            errors.append(e)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th = [threading.Thread(target=work, args=(k,)) for k in range(nstreams)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if errors:
        raise errors[0]
    return out, elapsed


def bench_batch(args, tcm, torch):
    from tests import workloads as wl

    t = time.perf_counter()
    b = wl.batch4096()
    log(f"[bench] generated batch: {b.num_graphs} graphs, {b.total_edges} input edges "
        f"({time.perf_counter() - t:.1f}s)")
    rp, ci = tcm.to_device(b.rowptr_cat, b.colidx_cat)
    ro = torch.from_numpy(b.row_off).cuda()
    co = torch.from_numpy(b.col_off).cuda()
    rows = int(b.rowptr_cat.shape[0])
    ws_bytes = tcm.tc_count_batch_workspace_size(b.num_graphs, rows, int(b.colidx_cat.shape[0]))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    counts = torch.zeros(b.num_graphs, dtype=torch.int64, device="cuda")
    tuned = None
    if args.autotune:
        from paper_2403_02997_amd import autotune as at
        t = time.perf_counter()
        tuned = at.autotune_batch(rp, ci, ro, co, workspace=ws, reps=1, cache=None)
        log(f"[bench] autotune: {tuned['params']} after {tuned['measured']} settings "
            f"({time.perf_counter() - t:.1f}s)")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(max(args.warmup, 1)):
            tcm.tc_count_batch(rp, ci, ro, co, total_rows=rows, workspace=ws, counts=counts)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        tcm.tc_count_batch(rp, ci, ro, co, total_rows=rows, workspace=ws, counts=counts)
    torch.cuda.synchronize()
    # the replays run on the current stream: events recorded there bracket each launch
    cur = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(cur)
    for i in range(args.steps):
        graph.replay()
        ev[i + 1].record(cur)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.steps
    launch_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
    batched = tcm.as_u64(counts).copy()
    log(f"[bench] batched: {t_batch * 1e3:.3f} ms per batch (events: "
        f"{np.mean(launch_ms):.3f} ms per launch)")

    if args.no_per_graph:  # counter runs: only the batched launches
        return {"metric": METRIC, "ms_per_step": t_batch * 1e3, "workload": "batch4096",
                "launch_ms": float(np.mean(launch_ms)), "per_graph_launch": None}
    # the same graphs through one tc_count call each
    dev = []
    for i in range(b.num_graphs):
        gi = b.graph(i)
        dev.append(tcm.to_device(gi.rowptr, gi.colidx))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    single = np.array([tcm.tc_count(r, c) for r, c in dev], dtype=np.uint64)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - t0
    log(f"[bench] per-graph: {t_single * 1e3:.3f} ms for {b.num_graphs} calls on one stream")
    assert np.array_equal(single, batched), "batched and per-graph counts differ"
    single4, t_single4 = per_graph_streams(tcm, torch, dev, 4)
    log(f"[bench] per-graph: {t_single4 * 1e3:.3f} ms for {b.num_graphs} calls on 4 streams")
    assert np.array_equal(single4, batched), "batched and per-graph counts differ (4 streams)"

    levels = batch_levels(tcm, dev)
    del dev
    pb = batch_plan_bytes(b, levels)
    del levels
    kern_ms = float(np.mean(launch_ms))
    achieved = pb["total"] / (kern_ms * 1e-3) / 1e9
    traffic = stored_traffic("batch4096", BATCH_KERNEL, current_settings(tcm))
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": BATCH_KERNEL, "avg_launch_ms": round(kern_ms, 4),
                "timed_in": f"HIP events around {args.steps} graph replays on their stream "
                            "(the replay also holds two kernels of a few microseconds)",
                "algorithmic_bytes_per_launch": pb["total"],
                "algorithmic_bytes": {k: pb[k] for k in ("bfs", "extract", "intersect", "output")},
                "intersect_frac": round(pb["intersect"] / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "merge_bytes_per_launch": pb["merge"],
                "traffic_gbs": (round(traffic / (kern_ms * 1e-3) / 1e9, 1) if traffic else None)}
    out = {
        "metric": METRIC,
        "value": b.total_edges / t_batch,
        "unit": "input edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_batch * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "batch4096", "graph": WORKLOAD_TEXT["batch4096"],
                   "num_graphs": b.num_graphs, "input_edges": b.total_edges,
                   "triangles": int(batched.sum()), "cover_edges": pb["cover_edges"],
                   "isect_params": list(tcm.tc_get_isect_params()),
                   "autotuned": tuned is not None, "launch": "hipGraph replay"},
        "triangles_per_s": float(batched.sum()) / t_batch,
        "per_graph_launch": {"value": b.total_edges / t_single, "unit": "input edges/s",
                             "ms_total": round(t_single * 1e3, 3), "streams": 1,
                             "four_streams": {"value": b.total_edges / t_single4,
                                              "ms_total": round(t_single4 * 1e3, 3)}},
        "batched_over_per_graph": t_single / t_batch,
        "batched_over_per_graph_four_streams": t_single4 / t_batch,
        "launch_ms": {"mean": round(kern_ms, 4), "median": round(float(np.median(launch_ms)), 4),
                      "min": round(float(np.min(launch_ms)), 4)},
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a sample of the members ...")
        out["cpu_baseline"] = cpu_baseline_batch(b, args.cpu_seconds)
    return out


# ---- continuous-batching server ----------------------------------------------------------

def bench_serve(args, tcm, torch):
    """Requests arrive as a Poisson stream whose offered load is --serve-load (default
    0.8) times the capacity of one-at-a-time standalone processing (pinned upload +
    tc_count); each result is checked against the standalone count of the same graph."""
    from tests import workloads as wl

    rng = np.random.default_rng(wl.SERVE_BASE_SEED)
    small_scales = list(wl.SERVE_SMALL_SCALES)
    large_scales = list(wl.SERVE_LARGE_SCALES)
    specs = wl.serve_pool_specs(args.serve_huge_scale)
    pool = {}
    t = time.perf_counter()
    for key, seed in specs.items():
        pool[key] = wl.serve_graph(key[0], seed)
        if key[0] >= 22:
            log(f"[bench] generated R-MAT scale {key[0]} ({time.perf_counter() - t:.1f}s)")
    # the oracle's counts of the pool, stored by tests/golden/make_full_counts.py
    gold_path = os.path.join(ROOT, "tests", "golden", "serve_pool_counts.json")
    gold = json.load(open(gold_path)) if os.path.exists(gold_path) else {}
    oracle_T = {key: gold.get(wl.rmat_key(key[0], wl.SERVE_EDGE_FACTOR, seed), {}).get("triangles")
                for key, seed in specs.items()}
    # Host CSRs in pinned memory (where a front end would receive them), standalone
    # results, and standalone service times (upload + count).
    host, ref, svc = {}, {}, {}
    for key, g in pool.items():
        hp = []
        for a in (g.rowptr, g.colidx):
            t_ = torch.empty(a.shape[0], dtype=torch.int32, pin_memory=True)
            t_.numpy()[:] = a.view(np.int32)
            hp.append(t_)
        host[key] = tuple(hp)
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rp, ci = hp[0].to("cuda"), hp[1].to("cuda")
            ref[key] = tcm.tc_count(rp, ci)
            svc[key] = time.perf_counter() - t0
            del rp, ci
    torch.cuda.empty_cache()
    log(f"[bench] standalone counts of {len(pool)} pool graphs done")
    nreq = args.serve_requests
    keys = []
    for _ in range(nreq):
        if rng.random() < 0.9:
            keys.append((int(rng.choice(small_scales)), int(rng.integers(0, 3))))
        else:
            keys.append((int(rng.choice(large_scales)), 0))
    if args.serve_huge_scale:
        keys[nreq // 2] = (args.serve_huge_scale, 0)
    mean_svc = float(np.mean([svc[k] for k in keys]))
    rate = args.serve_load / mean_svc
    gaps = rng.exponential(1.0 / rate, size=nreq)
    log(f"[bench] {nreq} requests, mean standalone service {mean_svc * 1e3:.2f} ms, "
        f"arrival rate {rate:.1f}/s")
    srv = tcm.Server(small_max_entries=args.serve_small_max)
    tickets = {}
    results = []
    t_start = time.perf_counter()
    next_t = t_start
    for k, key in enumerate(keys):
        next_t += gaps[k]
        while True:
            results += srv.poll(cap=512, timeout_ms=0)
            dt = next_t - time.perf_counter()
            if dt <= 0:
                break
            time.sleep(min(dt, 0.0005))
        tickets[srv.submit(*host[key])] = key
        if (k + 1) % 100 == 0:
            log(f"[bench] submitted {k + 1}/{nreq}")
    while len(results) < nreq:
        results += srv.poll(cap=512, timeout_ms=500)
    st = srv.stats()
    srv.close()
    bad = [r for r in results if r.status != 0 or r.triangles != ref[tickets[r.ticket]]]
    assert not bad, f"{len(bad)} server results differ from the standalone counts"
    unchecked = sorted({tickets[r.ticket] for r in results if oracle_T[tickets[r.ticket]] is None})
    wrong = [r for r in results
             if oracle_T[tickets[r.ticket]] is not None
             and r.triangles != oracle_T[tickets[r.ticket]]]
    assert not wrong, f"{len(wrong)} server results differ from the oracle's stored counts"
    assert all(ref[k] == oracle_T[k] for k in ref if oracle_T[k] is not None)
    lat = np.array([r.latency_s for r in results])
    first = min(r.submit_s for r in results)
    last = max(r.done_s for r in results)
    edges = sum(r.input_edges for r in results)
    paths = {"batched": sum(r.path == 0 for r in results),
             "single_medium": sum(r.path == 1 for r in results),
             "single_large": sum(r.path == 3 for r in results)}
    # the large path's requests: wait from submission to the start of their job, job
    # time and the standalone service time (the huge request is marked)
    large = sorted((r for r in results if r.path == 3), key=lambda r: r.submit_s)
    huge = (args.serve_huge_scale, 0) if args.serve_huge_scale else None
    large_path = {
        "admit_wait_ms_sum": round(sum(r.admit_s - r.submit_s for r in large) * 1e3, 1),
        "service_ms_sum": round(sum(r.done_s - r.admit_s for r in large) * 1e3, 1),
        "count_ms_sum": round(sum(r.done_s - r.count_s for r in large) * 1e3, 1),
        "standalone_ms_sum": round(sum(svc[tickets[r.ticket]] for r in large) * 1e3, 1),
        "huge": [{"latency_ms": round(r.latency_s * 1e3, 1),
                  "admit_wait_ms": round((r.admit_s - r.submit_s) * 1e3, 1),
                  "standalone_ms": round(svc[tickets[r.ticket]] * 1e3, 1)}
                 for r in large if tickets[r.ticket] == huge],
    }
    if args.serve_trace:
        # one line per request: its graph, path, server times and standalone service
        with open(args.serve_trace, "w") as f:
            for r in sorted(results, key=lambda r: r.submit_s):
                key = tickets[r.ticket]
                f.write(json.dumps({"scale": key[0], "graph": key[1], "path": r.path,
                                    "submit": r.submit_s, "admit": r.admit_s,
                                    "count": r.count_s, "done": r.done_s,
                                    "standalone_ms": round(svc[key] * 1e3, 3)}) + "\n")
    lat_by = {}
    for name, ids in (("batched", (0,)), ("single_medium", (1,)), ("single_large", (3,))):
        v = np.array([r.latency_s for r in results if r.path in ids])
        if v.size:
            lat_by[name] = {"p50": round(float(np.percentile(v, 50)) * 1e3, 3),
                            "p99": round(float(np.percentile(v, 99)) * 1e3, 3)}
    return {
        "metric": METRIC,
        "value": edges / (last - first),
        "unit": "input edges/s",
        "n_gpus": 1,
        "steps": nreq,
        "warmup": 0,
        "ms_per_step": (last - first) * 1e3 / nreq,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "serve", "graph": WORKLOAD_TEXT["serve"], "requests": nreq,
                   "arrival_rate_per_s": round(rate, 2), "offered_load": args.serve_load,
                   "mean_standalone_service_ms": round(mean_svc * 1e3, 3),
                   "huge_scale": args.serve_huge_scale,
                   "small_max_entries": args.serve_small_max},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 3),
                       "mean": round(float(lat.mean()) * 1e3, 3),
                       "max": round(float(lat.max()) * 1e3, 3)},
        "latency_ms_by_path": lat_by,
        "input_edges": int(edges),
        "paths": paths,
        "server": {k: st[k] for k in ("batches", "singles", "hbm_peak", "hbm_budget",
                                      "busy_s", "device_s")},
        "oracle_checked": {"requests": sum(oracle_T[tickets[r.ticket]] is not None
                                           for r in results),
                           "pool_graphs_without_stored_count": [list(k) for k in unchecked]},
        "large_path": large_path,
        "roofline": None,
        "cpu_baseline": None,
    }


# ---- counter-measured HBM traffic ---------------------------------------------------------

def _pmc_per_kernel(path: str, counter: str) -> dict:
    """Mean counter value (KiB) per dispatch, by kernel name with template arguments."""
    import csv
    acc = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("tc::", "")
        acc.setdefault(name, []).append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v), max(v)) for k, v in acc.items()}


def traffic_summary(args, settings: dict):
    mib = args.copy_mib
    copy_bytes = mib * (1 << 20)
    cf = _pmc_per_kernel(args.copy_fetch, "FETCH_SIZE")["__amd_rocclr_copyBuffer"][2]
    cw = _pmc_per_kernel(args.copy_write, "WRITE_SIZE")["__amd_rocclr_copyBuffer"][2]
    f_fetch = cf * 1024 / copy_bytes
    f_write = cw * 1024 / copy_bytes
    fetch = _pmc_per_kernel(args.pmc_fetch, "FETCH_SIZE")
    write = _pmc_per_kernel(args.pmc_write, "WRITE_SIZE")
    path = os.path.join(PROFILES, "traffic.json")
    db = json.load(open(path)) if os.path.exists(path) else {}
    rec = db.setdefault(args.workload, {})
    lines = [f"copy calibration: {mib} MiB device copy reads FETCH_SIZE {cf:.1f} KiB "
             f"(factor {f_fetch:.4f}) and WRITE_SIZE {cw:.1f} KiB (factor {f_write:.4f})"]
    for k in sorted(fetch):
        if not k.startswith(("k_isect", "k_hub_count", "k_batch_main", "k_split_rows")) or \
                k not in write:
            continue
        fb = fetch[k][0] * 1024 / f_fetch
        wb = write[k][0] * 1024 / f_write
        rec[k] = {"source_sha": source_sha(), **settings, "hbm_bytes_per_launch": int(fb + wb),
                  "fetch_bytes": int(fb), "write_bytes": int(wb),
                  "fetch_kib_raw": round(fetch[k][0], 1), "write_kib_raw": round(write[k][0], 1),
                  "dispatches": fetch[k][1], "copy_factor_fetch": round(f_fetch, 5),
                  "copy_factor_write": round(f_write, 5)}
        lines.append(f"{k}: FETCH_SIZE {fetch[k][0]:.1f} KiB, WRITE_SIZE {write[k][0]:.1f} KiB "
                     f"per dispatch ({fetch[k][1]} dispatches) -> {(fb + wb) / 1e9:.3f} GB "
                     f"of HBM traffic per launch")
    json.dump(db, open(path, "w"), indent=1, sort_keys=True)
    print("\n".join(lines))


def calibrate_copy(args, torch):
    n = args.calibrate_copy * (1 << 20)
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch4096", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-per-graph", action="store_true",
                    help="batch4096: skip the per-graph legs and the roofline (profiler runs)")
    ap.add_argument("--no-single-graph", action="store_true",
                    help="batch4096: leave out the nested R-MAT scale 22 single-graph figures")
    ap.add_argument("--single-cpu-seconds", type=float, default=8.0,
                    help="CPU-oracle budget of the nested single-graph figures")
    ap.add_argument("--isect", default="", metavar="LANE,WAVE,CHUNK,SEG",
                    help="intersection class parameters (tc_set_isect_params) for this run")
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="step-timed calls after the timed steps (step breakdown, roofline)")
    ap.add_argument("--forward-threshold", type=float, default=None,
                    help="CETC-Seq-FE covering-ratio threshold (the paper's 0.7; library "
                         "default 2 = never; 0 always counts in the forward ordering)")
    ap.add_argument("--hubs", default="", metavar="MAX_HUBS,MIN_DEGREE",
                    help="hub pass parameters (tc_set_hub_params) for this run; 0,0 turns it off")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the intersection class parameters on the workload first")
    ap.add_argument("--per-vertex", type=int, default=0, metavar="K",
                    help="single-graph workloads: also time K tc_count_per_vertex and "
                         "tc_local_clustering calls")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-huge-scale", type=int, default=26)
    ap.add_argument("--serve-small-max", type=int, default=1 << 18)
    ap.add_argument("--serve-load", type=float, default=0.8)
    ap.add_argument("--serve-trace", default="",
                    help="serve: write one JSON line per request (times, path, graph) here")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB")
    ap.add_argument("--traffic-summary", action="store_true")
    ap.add_argument("--pmc-fetch")
    ap.add_argument("--pmc-write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-mib", type=int, default=1024)
    args = ap.parse_args()
    if args.traffic_summary:
        # the settings of the counter runs: the library defaults unless given here too
        import paper_2403_02997_amd as tcm
        tcm.load()
        if args.isect:
            tcm.tc_set_isect_params(*[int(v) for v in args.isect.split(",")])
        if args.hubs:
            tcm.tc_set_hub_params(*[int(v) for v in args.hubs.split(",")])
        traffic_summary(args, current_settings(tcm))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the counting path here is single-GPU "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2403_02997_amd as tcm

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        calibrate_copy(args, torch)
        return
    tcm.load()
    if args.isect:
        tcm.tc_set_isect_params(*[int(v) for v in args.isect.split(",")])
    if args.hubs:
        tcm.tc_set_hub_params(*[int(v) for v in args.hubs.split(",")])
    if args.forward_threshold is not None:
        tcm.tc_set_forward_threshold(args.forward_threshold)
    if args.workload == "batch4096":
        out = bench_batch(args, tcm, torch)
        torch.cuda.empty_cache()
        if not args.no_single_graph:
            sub = argparse.Namespace(**vars(args))
            sub.workload = "rmat22"
            sub.cpu_seconds = args.single_cpu_seconds
            one = bench_single(sub, tcm, torch)
            out["single_graph"] = {k: one[k] for k in (
                "value", "unit", "ms_per_step", "steps", "config", "triangles_per_s",
                "steps_ms", "isect_classes", "roofline", "cpu_baseline")}
    elif args.workload == "serve":
        out = bench_serve(args, tcm, torch)
    else:
        out = bench_single(args, tcm, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

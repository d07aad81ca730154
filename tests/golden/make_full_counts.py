"""Writes the oracle's results for the full-size workloads:

  full_size_counts.json   the four single graphs (T, c1, c2, |S|, depth);
  batch4096_counts.json   every member of the 4096-graph batch (T, |S|, input edges);
  serve_pool_counts.json  every graph of the serving pool, keyed by generator,
                          parameters and seed (T, |S|, input edges).

Calls only the seeded generators (graphgen) and the CPU oracle (oracle); no value
comes from the GPU path.
Run: python tests/golden/make_full_counts.py [rmat10 rmat22 grid4096 er22 batch4096 serve]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

from tests import workloads as wl  # noqa: E402

OUT = os.path.join(HERE, "full_size_counts.json")
OUT_BATCH = os.path.join(HERE, "batch4096_counts.json")
OUT_SERVE = os.path.join(HERE, "serve_pool_counts.json")
ORACLE_TEXT = "CETC-SM (Section 4.4) after the ascending-ID BFS restart loop"


def count(g):
    """(T, c1, c2, |S|, depth) of g by the oracle."""
    level, depth = oracle.bfs_levels(g)
    S = oracle.cover_edges(g, level)
    T, c1, c2 = oracle.cetc_sm(g, level)
    return T, c1, c2, S, depth


def single(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        t0 = time.time()
        g = wl.WORKLOADS[name]()
        t1 = time.time()
        T, c1, c2, S, depth = count(g)
        t2 = time.time()
        data[name] = {
            "n": g.n, "nnz": g.nnz, "input_edges": g.num_edges, "triangles": T, "c1": c1,
            "c2": c2, "cover_edges": S, "depth": depth, "oracle": ORACLE_TEXT,
            "oracle_seconds": round(t2 - t1, 1), "threads": oracle.max_threads(),
        }
        print(name, data[name], f"gen {t1 - t0:.1f}s", flush=True)
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


def batch():
    t0 = time.time()
    b = wl.batch4096()
    print(f"batch4096 generated ({time.time() - t0:.1f}s)", flush=True)
    tri, cov, edges = [], [], []
    t1 = time.time()
    for i in range(b.num_graphs):
        g = b.graph(i)
        T, _, _, S, _ = count(g)
        tri.append(T)
        cov.append(S)
        edges.append(g.num_edges)
        if (i + 1) % 512 == 0:
            print(f"batch4096: {i + 1} members counted ({time.time() - t1:.1f}s)", flush=True)
    data = {"base_seed": wl.BATCH_BASE_SEED, "num_graphs": b.num_graphs,
            "oracle": ORACLE_TEXT, "triangles": tri, "cover_edges": cov,
            "input_edges": edges}
    json.dump(data, open(OUT_BATCH, "w"), separators=(",", ":"))
    print(f"batch4096: total T {sum(tri)}, {sum(edges)} input edges "
          f"({time.time() - t1:.1f}s)", flush=True)


def serve():
    data = json.load(open(OUT_SERVE)) if os.path.exists(OUT_SERVE) else {}
    specs = sorted(wl.serve_pool_specs().items())
    for (sc, _), seed in specs:
        key = wl.rmat_key(sc, wl.SERVE_EDGE_FACTOR, seed)
        if key in data:
            continue
        t0 = time.time()
        g = wl.serve_graph(sc, seed)
        t1 = time.time()
        T, c1, c2, S, depth = count(g)
        t2 = time.time()
        data[key] = {"scale": sc, "edge_factor": wl.SERVE_EDGE_FACTOR, "seed": seed,
                     "n": g.n, "input_edges": g.num_edges, "triangles": T, "c1": c1,
                     "c2": c2, "cover_edges": S, "depth": depth, "oracle": ORACLE_TEXT,
                     "oracle_seconds": round(t2 - t1, 1), "threads": oracle.max_threads()}
        del g
        print(key, data[key], f"gen {t1 - t0:.1f}s", flush=True)
        json.dump(data, open(OUT_SERVE, "w"), indent=1, sort_keys=True)


def main(names):
    for name in names:
        if name == "batch4096":
            batch()
        elif name == "serve":
            serve()
        else:
            single([name])


if __name__ == "__main__":
    main(sys.argv[1:] or sorted(wl.WORKLOADS) + ["batch4096", "serve"])

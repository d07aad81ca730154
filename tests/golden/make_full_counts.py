"""Writes full_size_counts.json: oracle results for the full-size workloads.

Calls only the seeded generators (graphgen) and the CPU oracle (oracle); no value
comes from the GPU path.  Run: python tests/golden/make_full_counts.py [name ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

from tests.workloads import WORKLOADS  # noqa: E402

OUT = os.path.join(HERE, "full_size_counts.json")


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        t0 = time.time()
        g = WORKLOADS[name]()
        t1 = time.time()
        level, depth = oracle.bfs_levels(g)
        t2 = time.time()
        S = oracle.cover_edges(g, level)
        T, c1, c2 = oracle.cetc_sm(g, level)
        t3 = time.time()
        data[name] = {
            "n": g.n, "nnz": g.nnz, "input_edges": g.num_edges, "triangles": T, "c1": c1,
            "c2": c2, "cover_edges": S, "depth": depth,
            "oracle": "CETC-SM (Section 4.4) after the ascending-ID BFS restart loop",
            "oracle_seconds": round(t3 - t2, 1), "threads": oracle.max_threads(),
        }
        print(name, data[name], f"gen {t1 - t0:.1f}s bfs {t2 - t1:.1f}s", flush=True)
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or sorted(WORKLOADS))

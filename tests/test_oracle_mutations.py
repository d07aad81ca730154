"""The oracle's pins catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of oracle/cetc_oracle.c (a wrong index, a
flipped comparison, a dropped condition, a wrong divisor, a broken merge step, a
cover-edge count over both stored copies of an edge or with the wrong level test, a
different BFS root order, a split pass that adds to the wrong set, leaves marks behind
or drops a term, a clustering coefficient over ordered pairs), builds the copy with gcc
into a temporary directory, and checks that at least one pin from test_oracle_pins
fails against it.  The committed oracle is never modified.
"""
import os
import subprocess

import networkx as nx
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import pins
from tests.test_oracle_pins import bfs_certificate, split_by_enumeration

SRC = os.path.join(os.path.dirname(oracle.__file__), "cetc_oracle.c")

MUTATIONS = {
    "rule_uses_u_not_v": ("if (one_horizontal || w > v) {", "if (one_horizontal || w > u) {"),
    "rule_level_test_flipped": ("const int one_horizontal = level[w] != level[u];",
                                "const int one_horizontal = level[w] == level[u];"),
    "edge_loop_drops_u_lt_v": ("      if (v <= u) continue;                /* the copy in the larger endpoint's row */\n",
                               ""),
    "edge_loop_not_horizontal": ("if (level[v] != level[u]) continue;  /* not horizontal: covers nothing */",
                                 "if (level[v] == level[u]) continue;"),
    "cover_edges_drops_u_lt_v": ("S += (u < colidx[e] && level[colidx[e]] == level[u]) ? 1u : 0u;",
                                 "S += (level[colidx[e]] == level[u]) ? 1u : 0u;"),
    "cover_edges_level_test_flipped": ("S += (u < colidx[e] && level[colidx[e]] == level[u]) ? 1u : 0u;",
                                       "S += (u < colidx[e] && level[colidx[e]] != level[u]) ? 1u : 0u;"),
    "bfs_level_step_two": ("level[y] = level[x] + 1;", "level[y] = level[x] + 2;"),
    "sm_divides_by_two": ("return c1 + c2 / 3;", "return c1 + c2 / 2;"),
    "merge_advances_wrong_list": ("if (colidx[i] < colidx[j]) {\n          ++i;",
                                  "if (colidx[i] < colidx[j]) {\n          ++j;"),
    "split_forward_adds_wrong_end": ("aset[rp0[v] + alen[v]++] = u;",
                                     "aset[rp0[u] + alen[u]++] = v;"),
    "split_cross_drops_u_lt_v": ("      if (!(u < v)) continue;\n      for (uint64_t k = rp1[v];",
                                 "      for (uint64_t k = rp1[v];"),
    "split_forward_marks_not_cleared": (
        "      for (uint64_t k = 0; k < alen[u]; ++k) hash[aset[rp0[u] + k]] = 0;\n", ""),
    "split_total_drops_g0": ("ret = t0 + t1;", "ret = t1;"),
    "clustering_counts_ordered_pairs": ("(double)(d - 1) / 2.0;", "(double)(d - 1);"),
    "bfs_roots_descending": ("for (uint32_t s = 0; s < n; ++s) {\n    if (level[s] != ORC_UNVISITED)",
                             "for (uint32_t s = n; s-- > 0;) {\n    if (level[s] != ORC_UNVISITED)"),
}


def pins_hold() -> bool:
    """True when every pin passes for the oracle currently in use."""
    try:
        k = nx.karate_club_graph()
        g = gg.from_edges(34, list(k.edges()))
        r = oracle.cetc_seq(g)
        if r.triangles != 45 or round(100.0 * r.cover_edges / 78, 1) != 35.9:
            return False
        if oracle.cover_edges(g, r.level) != 28:
            return False
        if oracle.cover_edges(gg.cycle(9), oracle.bfs_levels(gg.cycle(9))[0]) != 1:
            return False
        for seed in range(6):
            g = gg.gnp_small(12 + seed, 0.5, seed)
            r = oracle.cetc_seq(g)
            T_sm, c1, c2 = oracle.cetc_sm(g, r.level)
            if r.triangles != pins.brute_force_triples(g) or T_sm != r.triangles:
                return False
        g = gg.rmat(9, 16, 3)
        r = oracle.cetc_seq(g)
        if r.triangles != pins.sparse_count(g):
            return False
        if oracle.count(gg.complete(9)) != 84 or oracle.count(gg.tri_grid(7, 9)) != 96:
            return False
        bfs_certificate(g, r.level)
        if not np.all(oracle.local_clustering(gg.complete(6)) == 1.0):
            return False
        if oracle.cetc_split(gg.complete(9)) != (84, 56, 28):
            return False
        for seed in range(4):
            g = gg.gnp_small(40 + seed, 0.25, seed)
            level, _ = oracle.bfs_levels(g)
            T, t0, t1 = oracle.cetc_split(g, level)
            if (t0, t1) != split_by_enumeration(g, level) or T != pins.brute_force_triples(g):
                return False
    except AssertionError:
        return False
    return True


def test_unmodified_oracle_passes():
    assert pins_hold()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new, 1))  # first occurrence only
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                           str(mutated), "-o", str(lib)])
    with oracle.use_library(str(lib)):
        assert not pins_hold(), f"planted mistake {name} went unnoticed"

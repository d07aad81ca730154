/*
 * CPU ORACLE for cover-edge triangle counting — TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * this code.  It shares nothing with the GPU library: no headers, helpers, tables or
 * kernels.  It is deliberately plain and slow so that it can be checked against the
 * paper by eye:
 *
 *   Bader, Li, Du et al., "Cover Edge-Based Novel Triangle Counting" (arXiv 2403.02997)
 *     Section 2  : graph, neighbour set N(v), triangle = 3 distinct pairwise-adjacent
 *                  vertices.
 *     Def. BFS-Edge (Section 4.1): level L(v) = BFS distance from the root; an edge whose
 *                  endpoints share a level is horizontal.
 *     Algorithm CETC-Seq (Section 4.2): BFS from every still-unvisited vertex, then for
 *                  every horizontal edge (u,v) with u < v, every w in N(u) ∩ N(v) is
 *                  counted when L(u) != L(w), or when L(u) == L(w) and v < w.
 *     Algorithm CETC-SM (Section 4.4): the same edge loop in parallel; c1 counts apexes
 *                  on another level, c2 apexes on the same level; T = c1 + c2 / 3.
 *     Algorithm CETC-Seq-S (Section 4.3): the edges split into G0 (horizontal) and G1
 *                  (the rest); forward-hashed on G0, plus hashed N_G1(u) ∩ N_G1(v) for
 *                  every horizontal (u,v) with u < v.
 *
 * Readings where the paper is silent (also listed in the design notes):
 *   - the BFS restart loop visits candidate roots in ascending vertex ID, so each
 *     component's root is its smallest vertex ID, and every component starts at level 0;
 *   - the edge loop scans both stored directions of the symmetric CSR and keeps u < v,
 *     so every undirected edge is examined once;
 *   - "c2 / 3" is exact integer division (c2 is a multiple of 3);
 *   - the forward pass of CETC-Seq-S takes G0's edges by first endpoint in ascending ID;
 *   - counts are 64-bit unsigned.
 *
 * Input: symmetric CSR, rowptr[n+1], colidx[nnz] (uint32), neighbour lists strictly
 * increasing, no self-loops.  orc_check_csr verifies exactly that.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_UNVISITED 0xFFFFFFFFu

/* Return codes of orc_check_csr. */
#define ORC_OK 0
#define ORC_BAD_ROWPTR (-1)   /* rowptr[0] != 0, not monotone, or rowptr[n] != nnz */
#define ORC_BAD_INDEX (-2)    /* a neighbour ID >= n                               */
#define ORC_UNSORTED (-3)     /* a row not strictly increasing (or duplicate)       */
#define ORC_SELF_LOOP (-4)    /* v in N(v)                                          */
#define ORC_ASYMMETRIC (-5)   /* v in N(u) but u not in N(v)                        */

/* Binary search for x in the sorted list a[0..len). */
static int orc_contains(const uint32_t* a, uint64_t len, uint32_t x) {
  uint64_t lo = 0, hi = len;
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo < len && a[lo] == x;
}

/* Validate the input contract: the graph of Section 2 stored as a symmetric CSR. */
int orc_check_csr(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n, uint64_t nnz) {
  if (rowptr[0] != 0 || (uint64_t)rowptr[n] != nnz) return ORC_BAD_ROWPTR;
  for (uint32_t u = 0; u < n; ++u)
    if (rowptr[u + 1] < rowptr[u]) return ORC_BAD_ROWPTR;
  for (uint32_t u = 0; u < n; ++u) {
    for (uint64_t i = rowptr[u]; i < rowptr[u + 1]; ++i) {
      uint32_t v = colidx[i];
      if (v >= n) return ORC_BAD_INDEX;
      if (v == u) return ORC_SELF_LOOP;
      if (i > rowptr[u] && colidx[i - 1] >= v) return ORC_UNSORTED;
    }
  }
  for (uint32_t u = 0; u < n; ++u)
    for (uint64_t i = rowptr[u]; i < rowptr[u + 1]; ++i) {
      uint32_t v = colidx[i];
      if (!orc_contains(colidx + rowptr[v], rowptr[v + 1] - rowptr[v], u)) return ORC_ASYMMETRIC;
    }
  return ORC_OK;
}

/*
 * Levels by breadth-first search, restarted from every unvisited vertex (CETC-Seq, the
 * BFS restart loop; Def. BFS-Edge).  Candidate roots are taken in ascending ID; the
 * root of each component gets level 0 and every other vertex its shortest distance to
 * that root.  level[] must hold n entries.  Returns the largest level assigned (0 for an
 * edgeless graph), or -1 if the queue cannot be allocated.
 */
int64_t orc_bfs_levels(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n,
                       uint32_t* level) {
  uint32_t* queue = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
  if (!queue) return -1;
  uint32_t max_level = 0;
  for (uint32_t i = 0; i < n; ++i) level[i] = ORC_UNVISITED;
  for (uint32_t s = 0; s < n; ++s) {
    if (level[s] != ORC_UNVISITED) continue;
    /* BFS(G, s): plain FIFO queue. */
    uint64_t head = 0, tail = 0;
    level[s] = 0;
    queue[tail++] = s;
    while (head < tail) {
      uint32_t x = queue[head++];
      for (uint64_t i = rowptr[x]; i < rowptr[x + 1]; ++i) {
        uint32_t y = colidx[i];
        if (level[y] == ORC_UNVISITED) {
          level[y] = level[x] + 1;
          if (level[y] > max_level) max_level = level[y];
          queue[tail++] = y;
        }
      }
    }
  }
  free(queue);
  return (int64_t)max_level;
}

/*
 * Size of the cover-edge set of Theorem Gen-CES (Section 4.1): the number of horizontal
 * edges, those whose endpoints share a BFS level.  Every undirected edge is stored twice
 * in the CSR; only the copy in the row of its smaller endpoint is counted.
 */
uint64_t orc_cover_edges(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n,
                         const uint32_t* level) {
  uint64_t S = 0;
  for (uint32_t u = 0; u < n; ++u)
    for (uint64_t e = rowptr[u]; e < rowptr[u + 1]; ++e)
      S += (u < colidx[e] && level[colidx[e]] == level[u]) ? 1u : 0u;
  return S;
}

/* Statistics of one CETC-Seq run. */
typedef struct {
  uint64_t triangles;      /* T                                             */
  uint64_t cover_edges;    /* |S| = number of horizontal edges (u < v)      */
  uint64_t probes_min;     /* sum over S of min(d(u), d(v))                 */
  uint64_t probes_merge;   /* sum over S of d(u) + d(v)                     */
} orc_stats;

/*
 * The counting step of CETC-Seq (Section 4.2), after the BFS.  Each undirected edge
 * {u, v} is taken once, from the row of its smaller endpoint u.  When u and v share a
 * level the edge is a cover edge, and every common neighbour w of u and v is the apex of
 * one triangle {u, v, w} that contains it.  Such a triangle has either this one
 * horizontal edge (w on another level) or three (w on the same level; Lemma HE2).  The
 * first kind is counted here at once; the second kind is counted only at its edge of the
 * two smallest IDs, i.e. when w is larger than v (Theorem Correctness).  The common
 * neighbours come from a two-pointer walk over the two sorted rows.
 * `level` comes from orc_bfs_levels.  If tri_per_vertex is not NULL (n entries, zeroed
 * by the caller) every counted triangle {u, v, w} adds 1 to each of its three vertices.
 */
void orc_cetc_seq(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n,
                  const uint32_t* level, orc_stats* st, uint64_t* tri_per_vertex) {
  uint64_t T = 0, S = 0, pmin = 0, pmerge = 0;
  for (uint32_t u = 0; u < n; ++u) {
    const uint64_t ub = rowptr[u], ue = rowptr[u + 1];
    for (uint64_t e = ub; e < ue; ++e) {
      const uint32_t v = colidx[e];
      if (v <= u) continue;                /* the copy in the larger endpoint's row */
      if (level[v] != level[u]) continue;  /* not horizontal: covers nothing */
      S += 1;
      const uint64_t vb = rowptr[v], ve = rowptr[v + 1];
      pmin += (ue - ub) < (ve - vb) ? (ue - ub) : (ve - vb);
      pmerge += (ue - ub) + (ve - vb);
      uint64_t i = ub, j = vb;
      while (i < ue && j < ve) {
        if (colidx[i] < colidx[j]) {
          ++i;
        } else if (colidx[i] > colidx[j]) {
          ++j;
        } else {
          const uint32_t w = colidx[i];
          const int one_horizontal = level[w] != level[u];
          if (one_horizontal || w > v) {
            T += 1;
            if (tri_per_vertex) {
              tri_per_vertex[u] += 1;
              tri_per_vertex[v] += 1;
              tri_per_vertex[w] += 1;
            }
          }
          ++i;
          ++j;
        }
      }
    }
  }
  st->triangles = T;
  st->cover_edges = S;
  st->probes_min = pmin;
  st->probes_merge = pmerge;
}

/*
 * CETC-SM (Section 4.4): the horizontal-edge loop run in parallel with OpenMP over the
 * first endpoint u; for every common neighbour w, c1 counts w on another level and c2
 * counts w on the same level.  Only first endpoints u in [u_begin, u_end) are visited
 * (the whole graph is [0, n)), which lets a caller time a bounded sample.  Writes c1, c2
 * and returns T = c1 + c2 / 3 for the visited edges.  nthreads <= 0 uses the OpenMP
 * default.
 */
uint64_t orc_cetc_sm_range(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n,
                           const uint32_t* level, uint32_t u_begin, uint32_t u_end,
                           int nthreads, uint64_t* c1_out, uint64_t* c2_out) {
  uint64_t c1 = 0, c2 = 0;
  if (u_end > n) u_end = n;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : c1, c2) num_threads(nthreads)
#endif
  for (int64_t uu = (int64_t)u_begin; uu < (int64_t)u_end; ++uu) {
    uint32_t u = (uint32_t)uu;
    for (uint64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
      uint32_t v = colidx[e];
      if (!(level[u] == level[v] && u < v)) continue;
      uint64_t i = rowptr[u], j = rowptr[v];
      while (i < rowptr[u + 1] && j < rowptr[v + 1]) {
        if (colidx[i] < colidx[j]) {
          ++i;
        } else if (colidx[i] > colidx[j]) {
          ++j;
        } else {
          if (level[colidx[i]] != level[u]) c1 += 1;
          else c2 += 1;
          ++i;
          ++j;
        }
      }
    }
  }
  if (c1_out) *c1_out = c1;
  if (c2_out) *c2_out = c2;
  return c1 + c2 / 3;
}

/* CETC-SM over the whole graph. */
uint64_t orc_cetc_sm(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n,
                     const uint32_t* level, int nthreads, uint64_t* c1_out, uint64_t* c2_out) {
  return orc_cetc_sm_range(rowptr, colidx, n, level, 0, n, nthreads, c1_out, c2_out);
}

/*
 * CETC-Seq-S (Section 4.3, the split variant, Algorithm CETC-Seq-S), after the BFS:
 *   1. every edge goes to G0 when its endpoints share a level (horizontal), else to G1;
 *   2. t0 <- TC_forward-hashed(G0) (Section 3, Algorithm Forward-Hashed): for every edge
 *      (u, v) of G0 with u < v, count A(u) ∩ A(v) with a Boolean array, then add u to
 *      A(v); edges are taken by first endpoint in ascending ID, so A(u) already holds
 *      every smaller G0 neighbour of u when u's own edges are taken;
 *   3. t1 <- for every u, mark N_G1(u) in the Boolean array; for every v in N_G0(u) with
 *      u < v, count the w in N_G1(v) that are marked; clear the marks.
 * T = t0 + t1: t0 counts the triangles whose three edges are all horizontal, t1 the
 * others, each at its one horizontal edge.  The Boolean array is indexed by vertex
 * (n entries).  Writes t0 and t1; returns T, or UINT64_MAX if an allocation fails.
 */
uint64_t orc_cetc_split(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n,
                        const uint32_t* level, uint64_t* t0_out, uint64_t* t1_out) {
  size_t rows = (size_t)n + 1;
  uint64_t nnz = rowptr[n];
  uint64_t* rp0 = (uint64_t*)calloc(rows, sizeof(uint64_t));
  uint64_t* rp1 = (uint64_t*)calloc(rows, sizeof(uint64_t));
  uint32_t* ci0 = (uint32_t*)malloc(sizeof(uint32_t) * (nnz ? nnz : 1));
  uint32_t* ci1 = (uint32_t*)malloc(sizeof(uint32_t) * (nnz ? nnz : 1));
  uint32_t* aset = (uint32_t*)malloc(sizeof(uint32_t) * (nnz ? nnz : 1));
  uint64_t* alen = (uint64_t*)calloc(n ? n : 1, sizeof(uint64_t));
  unsigned char* hash = (unsigned char*)calloc(n ? n : 1, 1);
  uint64_t t0 = 0, t1 = 0, ret = UINT64_MAX;
  if (!rp0 || !rp1 || !ci0 || !ci1 || !aset || !alen || !hash) goto done;

  /* Step 1: partition E into E0 (horizontal) and E1, as two symmetric CSRs. */
  for (uint32_t u = 0; u < n; ++u) {
    uint64_t h = 0;
    for (uint64_t e = rowptr[u]; e < rowptr[u + 1]; ++e)
      if (level[colidx[e]] == level[u]) ++h;
    rp0[u + 1] = rp0[u] + h;
    rp1[u + 1] = rp1[u] + (rowptr[u + 1] - rowptr[u] - h);
  }
  for (uint32_t u = 0; u < n; ++u) {
    uint64_t i0 = rp0[u], i1 = rp1[u];
    for (uint64_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
      uint32_t v = colidx[e];
      if (level[v] == level[u]) ci0[i0++] = v;
      else ci1[i1++] = v;
    }
  }

  /* Step 2: forward-hashed on G0.  A(v) lives in aset[rp0[v] .. rp0[v] + alen[v]); it
   * only ever holds G0 neighbours of v, so d_G0(v) slots suffice. */
  for (uint32_t u = 0; u < n; ++u) {
    for (uint64_t e = rp0[u]; e < rp0[u + 1]; ++e) {
      uint32_t v = ci0[e];
      if (!(u < v)) continue;
      for (uint64_t k = 0; k < alen[u]; ++k) hash[aset[rp0[u] + k]] = 1;
      for (uint64_t k = 0; k < alen[v]; ++k)
        if (hash[aset[rp0[v] + k]]) t0 += 1;
      for (uint64_t k = 0; k < alen[u]; ++k) hash[aset[rp0[u] + k]] = 0;
      aset[rp0[v] + alen[v]++] = u;
    }
  }

  /* Step 3: hashed intersections on G1 for every horizontal edge (u, v), u < v. */
  for (uint32_t u = 0; u < n; ++u) {
    for (uint64_t e = rp1[u]; e < rp1[u + 1]; ++e) hash[ci1[e]] = 1;
    for (uint64_t e = rp0[u]; e < rp0[u + 1]; ++e) {
      uint32_t v = ci0[e];
      if (!(u < v)) continue;
      for (uint64_t k = rp1[v]; k < rp1[v + 1]; ++k)
        if (hash[ci1[k]]) t1 += 1;
    }
    for (uint64_t e = rp1[u]; e < rp1[u + 1]; ++e) hash[ci1[e]] = 0;
  }
  if (t0_out) *t0_out = t0;
  if (t1_out) *t1_out = t1;
  ret = t0 + t1;
done:
  free(rp0);
  free(rp1);
  free(ci0);
  free(ci1);
  free(aset);
  free(alen);
  free(hash);
  return ret;
}

/*
 * Local clustering coefficient (Watts and Strogatz; Section 1 lists clustering
 * coefficients among the uses of triangle counts), from the vertex form of the count of
 * Section 2: C(v) = |Delta(v)| / (d(v) choose 2) = 2 t(v) / (d(v) (d(v) - 1)), 0 when
 * d(v) < 2.  tri holds t(v) (orc_cetc_seq's per-vertex counts); cc gets n doubles.
 */
void orc_local_clustering(const uint32_t* rowptr, const uint64_t* tri, uint32_t n, double* cc) {
  for (uint32_t v = 0; v < n; ++v) {
    uint64_t d = rowptr[v + 1] - rowptr[v];
    if (d < 2) {
      cc[v] = 0.0;
    } else {
      double pairs = (double)d * (double)(d - 1) / 2.0; /* neighbour pairs, exact */
      cc[v] = (double)tri[v] / pairs;
    }
  }
}

/* Threads the OpenMP runtime would use by default (1 without OpenMP). */
int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

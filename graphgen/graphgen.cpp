// Seeded synthetic graph generators producing simple, symmetric uint32 CSR graphs
// with strictly increasing neighbour lists.
//
// This module holds input generation only (random draws, cleaning, CSR assembly).
// It contains none of the triangle-counting arithmetic and is shared by the tests,
// the benchmark and the CPU oracle's callers alike.
//
// Randomness: every draw is output i of a SplitMix64 sequence (Steele, Lea & Flood,
// "Fast splittable pseudorandom number generators", OOPSLA 2014), addressed by a
// counter, so each edge's draws depend only on (seed, edge index) and generation is
// deterministic regardless of the number of OpenMP threads.  Bounded integers use the
// multiply-high reduction (Lemire, "Fast random integer generation in an interval",
// TOMACS 2019, without the rejection step; the bias is below 2^-32 for our ranges).
//
// Families:
//   R-MAT / Kronecker (Chakrabarti, Zhan & Faloutsos, SDM 2004): each of `scale` bit
//     levels picks one of four quadrants with probabilities (a, b, c, 1-a-b-c).
//   Erdős–Rényi G(n, M): M uniform vertex pairs.
//   Triangulated R x C grid: 4-neighbour grid plus one diagonal (i,j)-(i+1,j+1) per
//     cell; optionally a seeded fraction of its edges deleted.
// Cleaning (all families): self-loops dropped, duplicates merged, both directions
// stored, rows sorted ascending.
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace {

inline uint64_t sm64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Output number i (0-based) of the SplitMix64 sequence whose state starts at `seed`.
inline uint64_t sm64_at(uint64_t seed, uint64_t i) {
  return sm64_mix(seed + (i + 1) * 0x9E3779B97F4A7C15ULL);
}

inline uint64_t bounded(uint64_t r, uint64_t range) {
  return (uint64_t)(((__uint128_t)r * (__uint128_t)range) >> 64);
}

const uint64_t kPermSalt = 0x5DEECE66DULL;
const uint64_t kDeleteSalt = 0xA5A5A5A5DEADBEEFULL;

// Probability p in [0,1] as a 64-bit threshold: draw r < thr happens with prob ~p.
inline uint64_t prob_threshold(long double p) {
  if (p <= 0) return 0;
  if (p >= 1) return UINT64_MAX;
  long double t = p * 18446744073709551616.0L;
  if (t >= 18446744073709551615.0L) return UINT64_MAX;
  return (uint64_t)t;
}

}  // namespace

extern "C" {

typedef struct {
  uint32_t n;
  uint64_t nnz;  // number of stored entries = 2 * undirected edges
  uint32_t* rowptr;  // n + 1 entries, malloc'd
  uint32_t* colidx;  // nnz entries, malloc'd
} gg_csr;

void gg_free(gg_csr* g) {
  if (!g) return;
  free(g->rowptr);
  free(g->colidx);
  g->rowptr = nullptr;
  g->colidx = nullptr;
}

int gg_num_threads(void) { return omp_get_max_threads(); }

// Build a clean CSR from an edge list (u[i], v[i]), i < m.  Self-loops are dropped,
// duplicate pairs (in either orientation) merged, both directions stored.
// Returns 0, or -1 on bad input / -2 on allocation failure / -3 when the cleaned
// graph has 2^32 or more stored entries.
int gg_from_edges(uint32_t n, const uint32_t* u, const uint32_t* v, uint64_t m, gg_csr* out) {
  if (!out) return -1;
  out->n = n;
  out->nnz = 0;
  out->rowptr = nullptr;
  out->colidx = nullptr;
  for (uint64_t i = 0; i < m; ++i)
    if (u[i] >= n || v[i] >= n) return -1;
  std::vector<uint64_t> deg((size_t)n + 1, 0);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)m; ++i) {
    if (u[i] == v[i]) continue;
#pragma omp atomic
    deg[u[i]]++;
#pragma omp atomic
    deg[v[i]]++;
  }
  std::vector<uint64_t> off((size_t)n + 1, 0);
  for (uint32_t x = 0; x < n; ++x) off[x + 1] = off[x] + deg[x];
  const uint64_t raw = off[n];
  uint32_t* tmp = (uint32_t*)malloc(sizeof(uint32_t) * (raw ? raw : 1));
  if (!tmp) return -2;
  std::vector<uint64_t> cur(off.begin(), off.end() - 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)m; ++i) {
    const uint32_t a = u[i], b = v[i];
    if (a == b) continue;
    uint64_t pa, pb;
#pragma omp atomic capture
    pa = cur[a]++;
#pragma omp atomic capture
    pb = cur[b]++;
    tmp[pa] = b;
    tmp[pb] = a;
  }
  // Sort and deduplicate every row in place; new degree into deg[].
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t x = 0; x < (int64_t)n; ++x) {
    uint32_t* r = tmp + off[x];
    const uint64_t len = off[x + 1] - off[x];
    std::sort(r, r + len);
    uint64_t k = 0;
    for (uint64_t i = 0; i < len; ++i)
      if (k == 0 || r[i] != r[k - 1]) r[k++] = r[i];
    deg[x] = k;
  }
  uint64_t nnz = 0;
  for (uint32_t x = 0; x < n; ++x) nnz += deg[x];
  if (nnz >= (1ULL << 32)) {
    free(tmp);
    return -3;
  }
  uint32_t* rowptr = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)n + 1));
  uint32_t* colidx = (uint32_t*)malloc(sizeof(uint32_t) * (nnz ? nnz : 1));
  if (!rowptr || !colidx) {
    free(tmp);
    free(rowptr);
    free(colidx);
    return -2;
  }
  rowptr[0] = 0;
  for (uint32_t x = 0; x < n; ++x) rowptr[x + 1] = rowptr[x] + (uint32_t)deg[x];
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t x = 0; x < (int64_t)n; ++x)
    memcpy(colidx + rowptr[x], tmp + off[x], sizeof(uint32_t) * deg[x]);
  free(tmp);
  out->nnz = nnz;
  out->rowptr = rowptr;
  out->colidx = colidx;
  return 0;
}

// Seeded random permutation of [0, n): Fisher–Yates driven by the counter RNG.
int gg_permutation(uint32_t n, uint64_t seed, uint32_t* perm) {
  for (uint32_t i = 0; i < n; ++i) perm[i] = i;
  for (uint32_t i = n; i > 1; --i) {
    const uint32_t j = (uint32_t)bounded(sm64_at(seed ^ kPermSalt, i - 1), i);
    std::swap(perm[i - 1], perm[j]);
  }
  return 0;
}

// R-MAT graph with 2^scale vertices and `nedges` generated (pre-cleaning) edges.
// Quadrant probabilities (a, b, c, 1-a-b-c).  With permute != 0 the vertex IDs are
// relabelled by a seeded random permutation.
int gg_rmat(int scale, uint64_t nedges, double a, double b, double c, uint64_t seed,
            int permute, gg_csr* out) {
  if (!out || scale < 1 || scale > 31 || a < 0 || b < 0 || c < 0 || a + b + c > 1.0)
    return -1;
  const uint32_t n = 1u << scale;
  const uint64_t ta = prob_threshold((long double)a);
  const uint64_t tab = prob_threshold((long double)a + b);
  const uint64_t tabc = prob_threshold((long double)a + b + c);
  uint32_t* u = (uint32_t*)malloc(sizeof(uint32_t) * (nedges ? nedges : 1));
  uint32_t* v = (uint32_t*)malloc(sizeof(uint32_t) * (nedges ? nedges : 1));
  if (!u || !v) {
    free(u);
    free(v);
    return -2;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)nedges; ++i) {
    uint32_t x = 0, y = 0;
    for (int lvl = 0; lvl < scale; ++lvl) {
      const uint64_t r = sm64_at(seed, (uint64_t)i * (uint64_t)scale + (uint64_t)lvl);
      uint32_t bx, by;
      if (r < ta) {
        bx = 0; by = 0;
      } else if (r < tab) {
        bx = 0; by = 1;
      } else if (r < tabc) {
        bx = 1; by = 0;
      } else {
        bx = 1; by = 1;
      }
      x = (x << 1) | bx;
      y = (y << 1) | by;
    }
    u[i] = x;
    v[i] = y;
  }
  if (permute) {
    std::vector<uint32_t> perm(n);
    gg_permutation(n, seed, perm.data());
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)nedges; ++i) {
      u[i] = perm[u[i]];
      v[i] = perm[v[i]];
    }
  }
  const int rc = gg_from_edges(n, u, v, nedges, out);
  free(u);
  free(v);
  return rc;
}

// Erdős–Rényi G(n, M): M uniform ordered pairs, then cleaned.
int gg_er(uint32_t n, uint64_t nedges, uint64_t seed, gg_csr* out) {
  if (!out || n == 0) return -1;
  uint32_t* u = (uint32_t*)malloc(sizeof(uint32_t) * (nedges ? nedges : 1));
  uint32_t* v = (uint32_t*)malloc(sizeof(uint32_t) * (nedges ? nedges : 1));
  if (!u || !v) {
    free(u);
    free(v);
    return -2;
  }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)nedges; ++i) {
    u[i] = (uint32_t)bounded(sm64_at(seed, 2 * (uint64_t)i), n);
    v[i] = (uint32_t)bounded(sm64_at(seed, 2 * (uint64_t)i + 1), n);
  }
  const int rc = gg_from_edges(n, u, v, nedges, out);
  free(u);
  free(v);
  return rc;
}

// Number of edges of the triangulated R x C grid before deletions.
uint64_t gg_grid_edges(uint32_t R, uint32_t C) {
  if (R == 0 || C == 0) return 0;
  return (uint64_t)R * (C - 1) + (uint64_t)(R - 1) * C + (uint64_t)(R - 1) * (C - 1);
}

// Triangulated R x C grid, vertex (i, j) = i * C + j (row-major, not permuted).
// Edge list order: all horizontal (i,j)-(i,j+1), then vertical (i,j)-(i+1,j), then
// diagonal (i,j)-(i+1,j+1).  `ndelete` edges are removed, chosen as the first
// `ndelete` positions of a seeded partial Fisher–Yates shuffle of the edge indices.
int gg_grid(uint32_t R, uint32_t C, uint64_t ndelete, uint64_t seed, gg_csr* out) {
  if (!out || R == 0 || C == 0) return -1;
  const uint64_t ne = gg_grid_edges(R, C);
  if (ndelete > ne) return -1;
  const uint64_t nv = (uint64_t)R * C;
  if (nv >= (1ULL << 32)) return -1;
  uint32_t* u = (uint32_t*)malloc(sizeof(uint32_t) * (ne ? ne : 1));
  uint32_t* v = (uint32_t*)malloc(sizeof(uint32_t) * (ne ? ne : 1));
  if (!u || !v) {
    free(u);
    free(v);
    return -2;
  }
  const uint64_t nh = (uint64_t)R * (C - 1), nvt = (uint64_t)(R - 1) * C;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < (int64_t)ne; ++e) {
    uint64_t i, j;
    uint32_t a, b;
    if ((uint64_t)e < nh) {
      i = e / (C - 1); j = e % (C - 1);
      a = (uint32_t)(i * C + j); b = a + 1;
    } else if ((uint64_t)e < nh + nvt) {
      const uint64_t k = e - nh;
      i = k / C; j = k % C;
      a = (uint32_t)(i * C + j); b = a + C;
    } else {
      const uint64_t k = e - nh - nvt;
      i = k / (C - 1); j = k % (C - 1);
      a = (uint32_t)(i * C + j); b = a + C + 1;
    }
    u[e] = a;
    v[e] = b;
  }
  if (ndelete > 0) {
    std::vector<uint32_t> idx(ne);
    for (uint64_t e = 0; e < ne; ++e) idx[e] = (uint32_t)e;
    for (uint64_t k = 0; k < ndelete; ++k) {
      const uint64_t j = k + bounded(sm64_at(seed ^ kDeleteSalt, k), ne - k);
      std::swap(idx[k], idx[j]);
    }
    // A deleted edge becomes a self-loop on its first endpoint; cleaning drops it.
    for (uint64_t k = 0; k < ndelete; ++k) v[idx[k]] = u[idx[k]];
  }
  const int rc = gg_from_edges((uint32_t)nv, u, v, ne, out);
  free(u);
  free(v);
  return rc;
}

// Raw draws of the counter RNG, for determinism tests and for seeding batch members.
void gg_splitmix(uint64_t seed, uint64_t start, uint64_t count, uint64_t* outv) {
  for (uint64_t i = 0; i < count; ++i) outv[i] = sm64_at(seed, start + i);
}

}  // extern "C"

// Preparation kernels: CSR tile map, connected components with smallest-ID roots
// (the root each BFS restart of the paper's CETC-Seq starts from), the per-vertex info
// byte, a device-wide exclusive scan, and the graph-format validator.
#include "tc_device.h"
#include "tc_launch.h"

namespace tc {

static inline u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }

int num_cus() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev >= 0 && dev < 64 && cached[dev]) return cached[dev];
  int v = 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
    v = 256;
  if (dev >= 0 && dev < 64) cached[dev] = v;
  return v;
}

// ---- tile map ----------------------------------------------------------------------
// Every tile start t*kTile lies in exactly one non-empty row; that row writes it.
__global__ void k_tile_rows(const u32* __restrict__ rowptr, u32 n, u32 m, u32 ntiles,
                            u32* __restrict__ tile_row) {
  for (u32 r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
    const u32 lo = rowptr[r], hi = rowptr[r + 1];
    if (lo == hi) continue;
    for (u32 t = (lo + kTile - 1) / kTile; (u64)t * kTile < hi; ++t) tile_row[t] = r;
    if (lo <= m - 1 && m - 1 < hi) tile_row[ntiles] = r;
  }
}

void launch_tile_rows(const u32* rowptr, u32 n, u32 m, u32* tile_row, hipStream_t s) {
  if (m == 0 || n == 0) return;
  const u32 ntiles = cdiv(m, kTile);
  const u32 grid = min(cdiv(n, 256), (u32)num_cus() * 8);
  hipLaunchKernelGGL(k_tile_rows, dim3(grid), dim3(256), 0, s, rowptr, n, m, ntiles, tile_row);
}

// ---- connected components ----------------------------------------------------------
// Union-find over parent[] with the invariant parent[x] <= x: links always go from the
// larger root to the smaller one, so each component's final root is its smallest
// vertex ID.  Initialisation takes the smallest neighbour as the first parent and the
// finds use path halving (both as in ECL-CC, Jaiganesh & Burtscher, HPDC 2018).
__global__ void k_cc_init(const u32* __restrict__ rowptr, const u32* __restrict__ colidx,
                          u32 n, u32* __restrict__ parent) {
  for (u32 v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const u32 lo = rowptr[v], hi = rowptr[v + 1];
    u32 p = v;
    if (lo < hi) p = min(v, colidx[lo]);  // rows are sorted: colidx[lo] is the smallest
    parent[v] = p;
  }
}

// Sampled links (Afforest, Sutton, Ben-Nun & Barak, IPDPS 2018): every vertex links the
// current roots of itself and of its two smallest neighbours (cc_min_link), which
// already assembles most of a dominant component; the links not made here are made by
// k_cc_finish.
__global__ void k_cc_sample(const u32* __restrict__ rowptr, const u32* __restrict__ colidx,
                            u32 n, u32* parent) {
  for (u32 v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const u32 lo = rowptr[v], hi = rowptr[v + 1];
    if (hi - lo >= 1 && colidx[lo] > v) cc_min_link(parent, v, colidx[lo]);
    if (hi - lo >= 2) cc_min_link(parent, v, colidx[lo + 1]);
  }
}

// A second sampling round (the third and fourth smallest neighbours), run only when
// mode[1] says that the first one left too many vertices outside the dominant component
// (many links lost to races, as on graphs without hubs, where every root is contended
// about equally); otherwise it returns at once.
__global__ void k_cc_sample_more(const u32* __restrict__ rowptr, const u32* __restrict__ colidx,
                                 u32 n, u32* parent, const u32* __restrict__ mode) {
  if (mode[1] == 0) return;
  for (u32 v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const u32 lo = rowptr[v], hi = rowptr[v + 1];
    if (hi - lo >= 3) cc_min_link(parent, v, colidx[lo + 2]);
    if (hi - lo >= 4) cc_min_link(parent, v, colidx[lo + 3]);
  }
}

// REDO: only when mode[1] is set (after k_cc_sample_more).
template <bool REDO>
__global__ void k_cc_compress(u32 n, u32* parent, const u32* __restrict__ mode) {
  if (REDO && mode[1] == 0) return;
  for (u32 v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    parent[v] = cc_find(parent, v);
}

// The most frequent root among kModeSamples spread-out vertices (one workgroup) in
// mode[0].  The first pass (REDO = false) also sets mode[1] when fewer than 90 % of the
// sampled vertices with neighbours have that root; the second pass runs only then.
constexpr u32 kModeSamples = 1024;

template <bool REDO>
__global__ void __launch_bounds__(kModeSamples) k_cc_mode(const u32* __restrict__ rowptr, u32 n,
                                                           u32* parent, u32* __restrict__ mode) {
  __shared__ u32 s_root[kModeSamples];
  __shared__ u64 s_best[kModeSamples / kWave];
  __shared__ u32 s_live[kModeSamples / kWave];
  if (REDO && mode[1] == 0) return;  // uniform
  const u32 i = threadIdx.x;
  const u32 v = (u32)(((u64)i * 2654435761ull + 12345u) % n);
  const u32 r = cc_find(parent, v);
  const bool live = rowptr[v + 1] > rowptr[v];
  s_root[i] = live ? r : kInf;  // isolated vertices are their own components
  __syncthreads();
  u32 cnt = 0;
  for (u32 j = 0; j < kModeSamples; ++j) cnt += s_root[j] == r;
  // largest (count, root) pair; ties go to the larger root value, any choice is correct
  u64 key = ((u64)cnt << 32) | r;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const u64 o = __shfl_xor(key, off, kWave);
    key = o > key ? o : key;
  }
  const u32 nlive = (u32)__popcll(__ballot(live));
  if (lane_id() == 0) {
    s_best[i / kWave] = key;
    s_live[i / kWave] = nlive;
  }
  __syncthreads();
  if (i == 0) {
    u64 b = 0;
    u32 tl = 0;
    for (u32 w = 0; w < kModeSamples / kWave; ++w) {
      b = s_best[w] > b ? s_best[w] : b;
      tl += s_live[w];
    }
    mode[0] = (u32)b;
    if (!REDO) mode[1] = (u32)(b >> 32) * 10 < tl * 9 ? 1u : 0u;
  }
}

// Remaining links: every vertex outside the dominant component joins all its
// neighbours.  An edge is skipped only when both endpoints already belong to the
// dominant component, because a vertex skips its list only once it is found inside it.
__global__ void __launch_bounds__(256) k_cc_finish(const u32* __restrict__ rowptr,
                                                   const u32* __restrict__ colidx, u32 n,
                                                   u32* parent, const u32* __restrict__ mode) {
  const u32 c = *mode;
  const u32 lane = lane_id();
  const u32 nr = (n + kWave - 1) / kWave * kWave;
  for (u32 u = blockIdx.x * blockDim.x + threadIdx.x; u < nr; u += gridDim.x * blockDim.x) {
    u32 lo = 0, d = 0;
    if (u < n && load_coherent(&parent[u]) != c) {
      lo = rowptr[u];
      d = rowptr[u + 1] - lo;
    }
    const bool big = d > kWave / 2;
    if (!big)
      for (u32 j = 0; j < d; ++j) cc_union(parent, u, colidx[lo + j]);
    u64 bigmask = __ballot(big);
    while (bigmask) {
      const int b = __ffsll((unsigned long long)bigmask) - 1;
      bigmask &= bigmask - 1;
      const u32 bu = __shfl(u, b, kWave), blo = __shfl(lo, b, kWave), bd = __shfl(d, b, kWave);
      for (u32 j = lane; j < bd; j += kWave) cc_union(parent, bu, colidx[blo + j]);
    }
  }
}

void launch_cc(const u32* rowptr, const u32* colidx, u32 n, u32 m, u32* parent, u32* mode,
               hipStream_t s) {
  if (n == 0) return;
  const u32 gv = min(cdiv(n, 256), (u32)num_cus() * 8);
  hipLaunchKernelGGL(k_cc_init, dim3(gv), dim3(256), 0, s, rowptr, colidx, n, parent);
  if (m > 0) {
    // flatten the initial forest first, so that the sampled links start from short paths
    hipLaunchKernelGGL(k_cc_compress<false>, dim3(gv), dim3(256), 0, s, n, parent, mode);
    hipLaunchKernelGGL(k_cc_sample, dim3(gv), dim3(256), 0, s, rowptr, colidx, n, parent);
    hipLaunchKernelGGL(k_cc_compress<false>, dim3(gv), dim3(256), 0, s, n, parent, mode);
    hipLaunchKernelGGL(k_cc_mode<false>, dim3(1), dim3(kModeSamples), 0, s, rowptr, n, parent,
                       mode);
    // second sampling round, only where the first left the dominant component thin
    hipLaunchKernelGGL(k_cc_sample_more, dim3(gv), dim3(256), 0, s, rowptr, colidx, n, parent,
                       mode);
    hipLaunchKernelGGL(k_cc_compress<true>, dim3(gv), dim3(256), 0, s, n, parent, mode);
    hipLaunchKernelGGL(k_cc_mode<true>, dim3(1), dim3(kModeSamples), 0, s, rowptr, n, parent,
                       mode);
    hipLaunchKernelGGL(k_cc_finish, dim3(gv), dim3(256), 0, s, rowptr, colidx, n, parent, mode);
  }
  hipLaunchKernelGGL(k_cc_compress<false>, dim3(gv), dim3(256), 0, s, n, parent, mode);
}

// ---- the first component and the rest ----------------------------------------------
// The restart loop of CETC-Seq starts its first BFS from the smallest ID; every vertex
// below the smallest one with neighbours is isolated, so that vertex v0 is the smallest
// of its component and roots it.  The first search runs from v0 alone (the isolated
// vertices are their own roots); only the vertices it does not reach need the
// union-find, which then joins just their edges (k_cc_finish with v0 as the dominant
// root).  mode[0] receives v0 (kInf when no vertex has neighbours), mode[2] the number
// of unreached vertices.
__global__ void __launch_bounds__(256) k_first_active(const u32* __restrict__ rowptr, u32 n,
                                                      u32* __restrict__ mode) {
  u32 best = kInf;
  for (u32 v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    if (rowptr[v + 1] > rowptr[v]) {
      best = v;  // the grid-stride order visits this thread's vertices ascending
      break;
    }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) best = min(best, (u32)__shfl_xor(best, off, kWave));
  if (lane_id() == 0 && best != kInf) atomicMin(&mode[0], best);
}

// parent[v] = v for v0 and the isolated vertices (the first search's roots), v0 for
// every other vertex.
__global__ void k_seed_first(const u32* __restrict__ rowptr, u32 n, u32* __restrict__ parent,
                             const u32* __restrict__ mode) {
  const u32 v0 = mode[0];
  for (u32 v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    parent[v] = rowptr[v + 1] == rowptr[v] || v == v0 || v0 == kInf ? v : v0;
}

// After the first search: every vertex it did not reach becomes its own parent and is
// counted in mode[2]; the reached ones keep parent v0.
__global__ void __launch_bounds__(256) k_rest_init(const u32* __restrict__ level, u32 n,
                                                   u32* __restrict__ parent,
                                                   u32* __restrict__ mode) {
  u32 cnt = 0;
  for (u32 v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    if (level[v] == kInf) {
      parent[v] = v;
      ++cnt;
    }
  cnt = wave_sum_u32(cnt);
  if (lane_id() == 0 && cnt) atomicAdd(&mode[2], cnt);
}

void launch_first_root(const u32* rowptr, u32 n, u32* parent, u32* mode, hipStream_t s) {
  if (n == 0) return;
  const u32 gv = min(cdiv(n, 256), (u32)num_cus() * 8);
  hipMemsetAsync(mode, 0xFF, sizeof(u32), s);  // mode[0] = kInf
  hipMemsetAsync(mode + 2, 0, sizeof(u32), s);
  hipLaunchKernelGGL(k_first_active, dim3(gv), dim3(256), 0, s, rowptr, n, mode);
  hipLaunchKernelGGL(k_seed_first, dim3(gv), dim3(256), 0, s, rowptr, n, parent, mode);
}

void launch_rest_init(const u32* level, u32 n, u32* parent, u32* mode, hipStream_t s) {
  if (n == 0) return;
  const u32 gv = min(cdiv(n, 256), (u32)num_cus() * 8);
  hipLaunchKernelGGL(k_rest_init, dim3(gv), dim3(256), 0, s, level, n, parent, mode);
}

void launch_rest_links(const u32* rowptr, const u32* colidx, u32 n, u32* parent, u32* mode,
                       hipStream_t s) {
  if (n == 0) return;
  const u32 gv = min(cdiv(n, 256), (u32)num_cus() * 8);
  hipLaunchKernelGGL(k_cc_finish, dim3(gv), dim3(256), 0, s, rowptr, colidx, n, parent, mode);
  hipLaunchKernelGGL(k_cc_compress<false>, dim3(gv), dim3(256), 0, s, n, parent, mode);
}

// ---- per-vertex info byte ------------------------------------------------------------
__global__ void __launch_bounds__(256) k_vinfo(const u32* __restrict__ rowptr,
                                               const u32* __restrict__ level, u32 n,
                                               uint8_t* __restrict__ vinfo,
                                               u32* __restrict__ hcur,
                                               u32* __restrict__ class_hist, u32 hist_min) {
  __shared__ u32 s_hist[128];
  if (class_hist) {
    if (threadIdx.x < 128) s_hist[threadIdx.x] = 0;
    __syncthreads();
  }
  for (u32 v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const u32 lo = rowptr[v];
    const u32 d = rowptr[v + 1] - lo;
    const u32 c = degree_class(d);
    const u32 par = level ? level[v] & 1u : 0u;  // no levels: every vertex on one level
    vinfo[v] = (uint8_t)((par << 7) | c);
    hcur[v] = lo;
    if (class_hist && c >= hist_min) atomicAdd(&s_hist[c], 1u);
  }
  if (class_hist) {
    __syncthreads();
    if (threadIdx.x < 128 && s_hist[threadIdx.x]) atomicAdd(&class_hist[threadIdx.x],
                                                            s_hist[threadIdx.x]);
  }
}

void launch_vinfo(const u32* rowptr, const u32* level, u32 n, uint8_t* vinfo, u32* hcur,
                  u32* class_hist, u32 hist_min, hipStream_t s) {
  if (n == 0) return;
  const u32 g = min(cdiv(n, 256), (u32)num_cus() * 8);
  hipLaunchKernelGGL(k_vinfo, dim3(g), dim3(256), 0, s, rowptr, level, n, vinfo, hcur,
                     class_hist, hist_min);
}

// ---- device-wide exclusive scan (u32) ------------------------------------------------
// Three phases: per-block sums of kScanChunk elements, a single-block scan of those
// sums, then a per-block scan that adds its block offset.
constexpr u32 kScanThreads = 256;
constexpr u32 kScanPer = 8;
constexpr u32 kScanChunk = kScanThreads * kScanPer;

size_t scan_tmp_words(u32 count) { return (size_t)cdiv(count, kScanChunk) + 1; }

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const u32* __restrict__ in,
                                                              u32 count, u32* __restrict__ sums) {
  __shared__ u32 s_tmp[kScanThreads / kWave];
  const u32 base = blockIdx.x * kScanChunk;
  u32 v = 0;
  for (u32 i = 0; i < kScanPer; ++i) {
    const u32 idx = base + i * kScanThreads + threadIdx.x;
    if (idx < count) v += in[idx];
  }
  u32 tot;
  block_incl_scan(v, s_tmp, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(u32* sums, u32 nb) {
  __shared__ u32 s_tmp[kScanThreads / kWave];
  u32 carry = 0;
  for (u32 base = 0; base < nb; base += kScanThreads) {
    const u32 idx = base + threadIdx.x;
    const u32 v = idx < nb ? sums[idx] : 0;
    u32 tot;
    const u32 incl = block_incl_scan(v, s_tmp, &tot);
    if (idx < nb) sums[idx] = carry + incl - v;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const u32* in, u32* out, u32 count,
                                                             const u32* __restrict__ sums) {
  __shared__ u32 s_tmp[kScanThreads / kWave];
  const u32 base = blockIdx.x * kScanChunk + threadIdx.x * kScanPer;
  u32 vals[kScanPer];
  u32 local = 0;
#pragma unroll
  for (u32 i = 0; i < kScanPer; ++i) {
    const u32 idx = base + i;
    vals[i] = idx < count ? in[idx] : 0;
    local += vals[i];
  }
  u32 tot;
  const u32 incl = block_incl_scan(local, s_tmp, &tot);
  u32 run = sums[blockIdx.x] + incl - local;
#pragma unroll
  for (u32 i = 0; i < kScanPer; ++i) {
    const u32 idx = base + i;
    if (idx < count) out[idx] = run;
    run += vals[i];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[count] = sums[gridDim.x];
}

void launch_scan(const u32* in, u32* out, u32 count, u32* tmp, hipStream_t s) {
  const u32 nb = count ? cdiv(count, kScanChunk) : 1;
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, in, count, tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanThreads), 0, s, in, out, count, tmp);
}

// ---- validator ------------------------------------------------------------------------
// flag bits: 1 bad rowptr, 2 index out of range, 4 unsorted/duplicate, 8 self-loop,
// 16 asymmetric.
__global__ void k_validate_rowptr(const u32* __restrict__ rowptr, u32 n, u32 m,
                                  u32* __restrict__ flag) {
  const u32 tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid == 0 && (rowptr[0] != 0 || rowptr[n] != m)) atomicOr(flag, 1u);
  for (u32 v = tid; v < n; v += gridDim.x * blockDim.x)
    if (rowptr[v + 1] < rowptr[v]) atomicOr(flag, 1u);
}

__device__ __forceinline__ bool sorted_contains(const u32* __restrict__ a, u32 len, u32 x) {
  u32 lo = 0, hi = len;
  while (lo < hi) {
    const u32 mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo < len && a[lo] == x;
}

__global__ void __launch_bounds__(kTileThreads) k_validate_entries(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx,
    const u32* __restrict__ tile_row, u32 n, u32 m, u32* __restrict__ flag) {
  __shared__ u32 s_rp[kTileRowCap];
  const u32 ntiles = (m + kTile - 1) / kTile;
  for (u32 t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const TileInfo ti = tile_begin(rowptr, tile_row, t, m, s_rp);
    for (u32 e = ti.e0 + threadIdx.x; e < ti.e1; e += blockDim.x) {
      const u32 u = tile_row_of(ti, s_rp, rowptr, e);
      const u32 v = colidx[e];
      u32 bad = 0;
      if (v >= n) {
        bad |= 2u;
      } else {
        if (v == u) bad |= 8u;
        if (e > rowptr[u] && colidx[e - 1] >= v) bad |= 4u;
        if (!sorted_contains(colidx + rowptr[v], rowptr[v + 1] - rowptr[v], u)) bad |= 16u;
      }
      if (bad) atomicOr(flag, bad);
    }
    __syncthreads();
  }
}

bool validate_rowptr_ok(const u32* rowptr, u32 n, u32 m, u32* flag, hipStream_t s) {
  const u32 g = min(cdiv(n + 1, 256), (u32)num_cus() * 8);
  hipLaunchKernelGGL(k_validate_rowptr, dim3(g), dim3(256), 0, s, rowptr, n, m, flag);
  u32 h = 0;
  if (hipMemcpyAsync(&h, flag, sizeof(u32), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
  if (hipStreamSynchronize(s) != hipSuccess) return false;
  return h == 0;
}

// Every neighbour ID below n (the bounds half of the contract: with rowptr monotone from
// 0 to m, no kernel then reads outside the graph's arrays).
__global__ void __launch_bounds__(256) k_check_ids(const u32* __restrict__ colidx, u32 n, u32 m,
                                                   u32* __restrict__ flag) {
  u32 bad = 0;
  for (u32 e = blockIdx.x * blockDim.x + threadIdx.x; e < m; e += gridDim.x * blockDim.x)
    bad |= colidx[e] >= n ? 1u : 0u;
  if (__ballot(bad != 0) && lane_id() == 0) atomicOr(flag, 1u);
}

int check_csr_bounds(const u32* rowptr, const u32* colidx, u32 n, u32 m, u32* flag,
                     hipStream_t s) {
  if (hipMemsetAsync(flag, 0, sizeof(u32), s) != hipSuccess) return -3;
  if (m > 0) {
    const u32 g = min(cdiv(m, 256), (u32)num_cus() * 8);
    hipLaunchKernelGGL(k_check_ids, dim3(g), dim3(256), 0, s, colidx, n, m, flag);
  }
  if (hipGetLastError() != hipSuccess) return -3;
  return validate_rowptr_ok(rowptr, n, m, flag, s) ? 0 : (hipGetLastError() != hipSuccess ? -3 : -4);
}

void launch_validate(const u32* rowptr, const u32* colidx, const u32* tile_row, u32 n, u32 m,
                     u32* flag, hipStream_t s) {
  if (m == 0) return;
  const u32 ntiles = cdiv(m, kTile);
  const u32 g = min(ntiles, (u32)num_cus() * 8);
  hipLaunchKernelGGL(k_validate_entries, dim3(g), dim3(kTileThreads), 0, s, rowptr, colidx,
                     tile_row, n, m, flag);
}

}  // namespace tc

// Batched counting: many independent graphs in one persistent launch.
//
// A planner orders the graphs by stored entries, largest power-of-two class first.  Then
// one persistent grid of workgroups pops graphs from that order; the workgroup that
// takes a graph runs the whole method on it without leaving the kernel:
//
//   1. component roots: union-find with smallest-ID roots (the root each restart of
//      the paper's CETC-Seq BFS loop starts from);
//   2. level BFS from all roots, one frontier level per workgroup barrier;
//   3. per-vertex info byte (level parity, degree class);
//   4. cover edges and intersections fused: every vertex x selects its horizontal
//      neighbours y of smaller (degree class, ID) key on the fly, stages N(x) in an LDS
//      hash set (per wavefront when d(x) <= 512, per workgroup in 4096-entry chunks
//      otherwise) and streams the partners' lists through it with the apex rule of
//      CETC-Seq (Section 4.2);
//   5. counts[g] = c1 + t2.
//
// Per-vertex scratch (parent, level, queue, info) lives in the caller's workspace at the
// graph's row offset, so graphs never share memory and the call allocates nothing.
#include "tc_device.h"
#include "tc_launch.h"

namespace tc {

constexpr int kBT = 256;                 // threads per workgroup
constexpr int kBW = kBT / kWave;         // wavefronts per workgroup
constexpr u32 kBSmallMax = 512;          // d(x) staged per wavefront
constexpr int kBWSlots = 1024;           // hash slots per wavefront
constexpr int kBBSlots = 8192;           // hash slots per workgroup
constexpr u32 kBChunk = 4096;            // entries of N(x) per workgroup table
constexpr u32 kBuckets = 40;             // planner cost classes
constexpr u32 kLaneDeg = 32;             // lists up to this length are walked per lane
constexpr int kBUnroll = 4;

struct BatchCtl {
  u32 next;
  u32 status;
  u32 pad[2];
};

size_t batch_ctl_bytes() { return 256; }

// ---- planner ------------------------------------------------------------------------
__device__ __forceinline__ u32 cost_bucket(u64 m) {
  const u32 bl = m ? 64u - (u32)__clzll((long long)m) : 0u;
  return kBuckets - 1 - (bl < kBuckets - 1 ? bl : kBuckets - 1);
}

__global__ void __launch_bounds__(256) k_batch_prepare(const int64_t* __restrict__ col_off,
                                                       u32 G, BatchCtl* __restrict__ ctl,
                                                       u32* __restrict__ order) {
  __shared__ u32 s_hist[kBuckets], s_cur[kBuckets];
  for (u32 i = threadIdx.x; i < kBuckets; i += blockDim.x) s_hist[i] = 0;
  if (threadIdx.x == 0) {
    ctl->next = 0;
    ctl->status = 0;
  }
  __syncthreads();
  for (u32 g = threadIdx.x; g < G; g += blockDim.x)
    atomicAdd(&s_hist[cost_bucket((u64)(col_off[g + 1] - col_off[g]))], 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    u32 run = 0;
    for (u32 b = 0; b < kBuckets; ++b) {
      s_cur[b] = run;
      run += s_hist[b];
    }
  }
  __syncthreads();
  for (u32 g = threadIdx.x; g < G; g += blockDim.x) {
    const u32 b = cost_bucket((u64)(col_off[g + 1] - col_off[g]));
    order[atomicAdd(&s_cur[b], 1u)] = g;
  }
}

// ---- workgroup-wide traversal of adjacency lists -----------------------------------------
// Calls f(u, v, active) for every v in N(u), u = list[i] (or i when list is null),
// i < count.  Short lists are walked one per lane in lockstep, long lists by the whole
// wavefront; f is reached by all lanes of a wavefront together (for wave_append).
template <typename F>
__device__ __forceinline__ void block_for_each_entry(const u32* __restrict__ rp,
                                                     const u32* __restrict__ ci, u32 count,
                                                     const u32* __restrict__ list, F&& f) {
  const u32 lane = lane_id();
  const u32 cr = (count + kWave - 1) / kWave * kWave;
  for (u32 i = threadIdx.x; i < cr; i += blockDim.x) {
    u32 u = 0, lo = 0, d = 0;
    if (i < count) {
      u = list ? list[i] : i;
      lo = rp[u];
      d = rp[u + 1] - lo;
    }
    const bool big = d > kLaneDeg;
    const u32 dl = big ? 0 : d;
    u32 dmax = dl;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dmax = max(dmax, (u32)__shfl_xor(dmax, off, kWave));
    for (u32 j = 0; j < dmax; ++j) {
      const bool act = j < dl;
      const u32 v = act ? ci[lo + j] : 0u;
      f(u, v, act);
    }
    u64 bigmask = __ballot(big);
    while (bigmask) {
      const int b = __ffsll((unsigned long long)bigmask) - 1;
      bigmask &= bigmask - 1;
      const u32 bu = __shfl(u, b, kWave), blo = __shfl(lo, b, kWave), bd = __shfl(d, b, kWave);
      for (u32 j0 = 0; j0 < bd; j0 += kWave) {
        const u32 j = j0 + lane;
        const bool act = j < bd;
        const u32 v = act ? ci[blo + j] : 0u;
        f(bu, v, act);
      }
    }
  }
}

__global__ void __launch_bounds__(kBT) k_batch_main(
    const u32* __restrict__ rowptr_cat, const u32* __restrict__ colidx_cat,
    const int64_t* __restrict__ row_off, const int64_t* __restrict__ col_off, u32 G,
    const u32* __restrict__ order, BatchCtl* __restrict__ ctl, u32* __restrict__ parent_all,
    u32* __restrict__ level_all, u32* __restrict__ queue_all, uint8_t* __restrict__ vinfo_all,
    u64* __restrict__ counts) {
  __shared__ __align__(16) u32 s_tab[kBBSlots];  // 4 wavefront tables, or one workgroup table
  __shared__ u32 s_plist[kBW][kBSmallMax];
  __shared__ u32 s_incl[kBT], s_start[kBT], s_y[kBT];
  __shared__ u32 s_tmp[kBW];
  __shared__ u64 s_red[3 * kBW];
  __shared__ u32 s_g, s_qtail, s_xnext, s_cnt;
  const u32 lane = lane_id(), wid = threadIdx.x / kWave;

  while (true) {
    if (threadIdx.x == 0) {
      const u32 idx = atomicAdd(&ctl->next, 1u);
      s_g = idx < G ? order[idx] : kInf;
      s_qtail = 0;
      s_xnext = 0;
      s_cnt = 0;
    }
    __syncthreads();
    const u32 g = s_g;
    if (g == kInf) break;
    const int64_t rb = row_off[g];
    const u32 n = (u32)(row_off[g + 1] - rb - 1);
    const int64_t cb = col_off[g];
    const u32 m = (u32)(col_off[g + 1] - cb);
    if (n == 0 || m == 0) {
      if (threadIdx.x == 0) counts[g] = 0;
      __syncthreads();
      continue;
    }
    const u32* rp = rowptr_cat + rb;
    const u32* ci = colidx_cat + cb;
    u32* parent = parent_all + rb;
    u32* level = level_all + rb;
    u32* queue = queue_all + rb;
    uint8_t* vinfo = vinfo_all + rb;

    // ---- 1. component roots ----
    for (u32 v = threadIdx.x; v < n; v += kBT) {
      const u32 lo = rp[v], hi = rp[v + 1];
      parent[v] = lo < hi ? min(v, ci[lo]) : v;
    }
    __syncthreads();
    block_for_each_entry(rp, ci, n, nullptr, [&](u32 u, u32 v, bool act) {
      if (act && v < u && load_coherent(&parent[u]) != v) cc_union(parent, u, v);
    });
    __syncthreads();
    for (u32 v = threadIdx.x; v < n; v += kBT) parent[v] = cc_find(parent, v);
    __syncthreads();

    // ---- 2. level BFS from every root ----
    {
      const u32 nr = (n + kWave - 1) / kWave * kWave;
      for (u32 v = threadIdx.x; v < nr; v += kBT) {
        bool push = false;
        if (v < n) {
          const bool root = parent[v] == v;
          level[v] = root ? 0u : kInf;
          push = root && rp[v + 1] > rp[v];
        }
        const u32 pos = wave_append(&s_qtail, push);
        if (push) queue[pos] = v;
      }
    }
    __syncthreads();
    u32 qs = 0, k = 0;
    while (true) {
      const u32 qe = s_qtail;
      if (qs == qe) break;
      __syncthreads();
      const u32 next = k + 1;
      block_for_each_entry(rp, ci, qe - qs, queue + qs, [&](u32 u, u32 v, bool act) {
        (void)u;
        bool claimed = false;
        if (act && load_coherent(&level[v]) == kInf)
          claimed = atomicCAS(&level[v], kInf, next) == kInf;
        const u32 pos = wave_append(&s_qtail, claimed);
        if (claimed) queue[pos] = v;
      });
      __syncthreads();
      qs = qe;
      ++k;
    }

    // ---- 3. per-vertex info ----
    for (u32 v = threadIdx.x; v < n; v += kBT)
      vinfo[v] = (uint8_t)(((level[v] & 1u) << 7) | degree_class(rp[v + 1] - rp[v]));
    __syncthreads();

    // ---- 4a. staged vertices of short lists: one wavefront each ----
    Counts c{0, 0, 0, 0, 0};
    {
      u32* table = s_tab + wid * kBWSlots;
      u32* plist = s_plist[wid];
      u32* incl_w = s_incl + wid * kWave;
      u32* start_w = s_start + wid * kWave;
      u32* y_w = s_y + wid * kWave;
      while (true) {
        u32 x = 0;
        if (lane == 0) x = atomicAdd(&s_xnext, 1u);
        x = __shfl(x, 0, kWave);
        if (x >= n) break;
        const u32 bx = rp[x], dx = rp[x + 1] - bx;
        if (dx < 2 || dx > kBSmallMax) continue;
        const u32 vx = vinfo[x], px = vx & 0x80u, cx = vx & 127u;
        const u32 mask = bucket_mask(dx, kBWSlots);
        for (u32 i = lane; i < (mask + 1) * 4; i += kWave) table[i] = kInf;
        wave_lds_sync();
        u32 np = 0;
        for (u32 i0 = 0; i0 < dx; i0 += kWave) {
          const u32 i = i0 + lane;
          const bool act = i < dx;
          u32 w = 0, vw = 0;
          if (act) {
            w = ci[bx + i];
            vw = vinfo[w];
          }
          const bool same = (vw & 0x80u) == px;
          if (act) hash_insert(table, mask, w, same ? 1u : 0u);
          const bool isp = act && same && key_less(vw & 127u, w, cx, x);
          const u64 pm = __ballot(isp);
          if (isp) plist[np + mask_rank(pm)] = w;
          np += (u32)__popcll(pm);
        }
        wave_lds_sync();
        for (u32 pb = 0; pb < np; pb += kWave) {
          const u32 p = pb + lane;
          u32 y = 0, sy = 0, dy = 0;
          if (p < np) {
            y = plist[p];
            sy = rp[y];
            dy = rp[y + 1] - sy;
          }
          const u32 incl = wave_incl_scan(dy);
          const u32 total = __shfl(incl, kWave - 1, kWave);
          incl_w[lane] = incl;
          start_w[lane] = sy - (incl - dy);
          y_w[lane] = y;
          wave_lds_sync();
          for (u32 k0 = 0; k0 < total; k0 += kWave * kBUnroll) {
            u32 ws[kBUnroll], ls[kBUnroll];
#pragma unroll
            for (int u = 0; u < kBUnroll; ++u) {
              const u32 kk = k0 + u * kWave + lane;
              ls[u] = kInf;
              if (kk < total) {
                u32 lo = 0, hi = kWave - 1;
                while (lo < hi) {
                  const u32 mid = (lo + hi) >> 1;
                  if (incl_w[mid] > kk) hi = mid;
                  else lo = mid + 1;
                }
                ls[u] = lo;
                ws[u] = ci[start_w[lo] + kk];
              }
            }
#pragma unroll
            for (int u = 0; u < kBUnroll; ++u) {
              if (ls[u] != kInf) {
                const u32 r = hash_probe(table, mask, ws[u]);
                if (r) {
                  const u32 y2 = y_w[ls[u]];
                  count_hit<false>(r, ws[u], x, y2, max(x, y2), c, nullptr);
                }
              }
            }
          }
          wave_lds_sync();
        }
      }
    }
    __syncthreads();

    // ---- 4b. staged vertices of long lists: the whole workgroup, chunk by chunk ----
    {
      const u32 nr = (n + kWave - 1) / kWave * kWave;
      for (u32 v = threadIdx.x; v < nr; v += kBT) {
        const bool isl = v < n && rp[v + 1] - rp[v] > kBSmallMax;
        const u32 pos = wave_append(&s_cnt, isl);
        if (isl) queue[pos] = v;  // the BFS queue is free again
      }
      __syncthreads();
      const u32 nl = s_cnt;
      for (u32 li = 0; li < nl; ++li) {
        const u32 x = queue[li];
        const u32 bx = rp[x], dx = rp[x + 1] - bx;
        const u32 vx = vinfo[x], px = vx & 0x80u, cx = vx & 127u;
        const u32 nch = (dx + kBChunk - 1) / kBChunk;
        for (u32 ch = 0; ch < nch; ++ch) {
          const u32 c0 = ch * kBChunk, clen = min(kBChunk, dx - c0);
          const u32 mask = bucket_mask(clen, kBBSlots);
          for (u32 i = threadIdx.x; i < (mask + 1) * 4; i += kBT) s_tab[i] = kInf;
          __syncthreads();
          for (u32 i = threadIdx.x; i < clen; i += kBT) {
            const u32 w = ci[bx + c0 + i];
            const u32 same = ((vinfo[w] & 0x80u) == px) ? 1u : 0u;
            hash_insert(s_tab, mask, w, same);
          }
          const u32 wlo = ci[bx + c0], whi = ci[bx + c0 + clen - 1];
          __syncthreads();
          for (u32 j0 = 0; j0 < dx; j0 += kBT) {
            const u32 j = j0 + threadIdx.x;
            u32 y = 0, sy = 0, dy = 0;
            if (j < dx) {
              y = ci[bx + j];
              const u32 vy = vinfo[y];
              if ((vy & 0x80u) == px && key_less(vy & 127u, y, cx, x)) {
                sy = rp[y];
                u32 ey = rp[y + 1];
                if (nch > 1) {
                  sy = lower_bound_g(ci, sy, ey, wlo);
                  ey = lower_bound_g(ci, sy, ey, whi + 1u);
                }
                dy = ey - sy;
              }
            }
            u32 total;
            const u32 incl = block_incl_scan(dy, s_tmp, &total);
            s_incl[threadIdx.x] = incl;
            s_start[threadIdx.x] = sy - (incl - dy);
            s_y[threadIdx.x] = y;
            __syncthreads();
            for (u32 k0 = 0; k0 < total; k0 += kBT * kBUnroll) {
              u32 ws[kBUnroll], ls[kBUnroll];
#pragma unroll
              for (int u = 0; u < kBUnroll; ++u) {
                const u32 kk = k0 + u * kBT + threadIdx.x;
                ls[u] = kInf;
                if (kk < total) {
                  u32 lo = 0, hi = kBT - 1;
                  while (lo < hi) {
                    const u32 mid = (lo + hi) >> 1;
                    if (s_incl[mid] > kk) hi = mid;
                    else lo = mid + 1;
                  }
                  ls[u] = lo;
                  ws[u] = ci[s_start[lo] + kk];
                }
              }
#pragma unroll
              for (int u = 0; u < kBUnroll; ++u) {
                if (ls[u] != kInf) {
                  const u32 r = hash_probe(s_tab, mask, ws[u]);
                  if (r) {
                    const u32 y2 = s_y[ls[u]];
                    count_hit<false>(r, ws[u], x, y2, max(x, y2), c, nullptr);
                  }
                }
              }
            }
            __syncthreads();
          }
        }
      }
    }

    // ---- 5. per-graph totals ----
    c.c1 = wave_sum_u64(c.c1);
    c.c2 = wave_sum_u64(c.c2);
    c.t2 = wave_sum_u64(c.t2);
    if (lane == 0) {
      s_red[3 * wid] = c.c1;
      s_red[3 * wid + 1] = c.c2;
      s_red[3 * wid + 2] = c.t2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      u64 c1 = 0, c2 = 0, t2 = 0;
      for (int w = 0; w < kBW; ++w) {
        c1 += s_red[3 * w];
        c2 += s_red[3 * w + 1];
        t2 += s_red[3 * w + 2];
      }
      counts[g] = c1 + t2;
      if (c2 != 3 * t2) atomicOr(&ctl->status, 1u);
    }
    __syncthreads();
  }
}

size_t batch_workspace_bytes(u32 G, u64 total_rows) {
  size_t b = batch_ctl_bytes();
  b += ((size_t)G * 4 + 255) / 256 * 256;
  b += (total_rows * 4 + 255) / 256 * 256 * 3;
  b += (total_rows + 255) / 256 * 256;
  return b + 256;
}

int batch_grid() {
  // Two workgroups of ~46 KB LDS per compute unit.
  return num_cus() * 2;
}

void launch_batch(const u32* rowptr_cat, const u32* colidx_cat, const int64_t* row_off,
                  const int64_t* col_off, u32 G, u64 total_rows, void* ws, u64* counts,
                  hipStream_t s) {
  char* base = (char*)(((uintptr_t)ws + 255) / 256 * 256);
  BatchCtl* ctl = (BatchCtl*)base;
  base += batch_ctl_bytes();
  u32* order = (u32*)base;
  base += ((size_t)G * 4 + 255) / 256 * 256;
  const size_t vb = (total_rows * 4 + 255) / 256 * 256;
  u32* parent = (u32*)base;
  base += vb;
  u32* level = (u32*)base;
  base += vb;
  u32* queue = (u32*)base;
  base += vb;
  uint8_t* vinfo = (uint8_t*)base;
  hipLaunchKernelGGL(k_batch_prepare, dim3(1), dim3(256), 0, s, col_off, G, ctl, order);
  const u32 grid = (u32)min((int)G, batch_grid());
  hipLaunchKernelGGL(k_batch_main, dim3(grid), dim3(kBT), 0, s, rowptr_cat, colidx_cat, row_off,
                     col_off, G, order, ctl, parent, level, queue, vinfo, counts);
}

}  // namespace tc

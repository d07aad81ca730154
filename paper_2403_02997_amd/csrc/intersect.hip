// Intersection of neighbour lists over the cover edges, with the apex rule.
//
// For a cover edge {x, y} (x = staged endpoint, y = streamed endpoint) and a common
// neighbour w, the paper's CETC-Seq (Section 4.2) counts w when L(w) != L(u), or when
// L(w) == L(u) and v < w, where u < v are the edge's endpoints in ID order; CETC-SM
// (Section 4.4) counts c1 = apexes on another level and c2 = apexes on the same level.
// Since w is adjacent to x, "L(w) != L(x)" equals "parity(w) != parity(x)".  The
// kernels count c1, c2 and t2 = #{same-level apex with w > max(x, y)}; T = c1 + t2 and,
// independently, T = c1 + c2 / 3.
//
// Three classes by d(x):
//   lane  : d(x) <= lane_max — one lane merges N(x) and N(y) (sorted two-pointer).
//   wave  : d(x) <= wave_max — one wavefront per x stages N(x) in an LDS hash set and
//           streams the concatenated partner lists, 64 lanes wide.
//   block : larger — one workgroup per (x, chunk of N(x), segment of partners); the
//           chunk goes into a 32 KB LDS hash set, each partner list is cut to the
//           chunk's ID range by binary search and streamed by all 256 threads.
#include "tc_device.h"
#include "tc_launch.h"

namespace tc {

static inline u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }

constexpr int kWaveSlots = 1024;   // LDS hash slots per wavefront (d(x) <= 512)
constexpr int kBlockSlots = 8192;  // LDS hash slots per workgroup (chunk <= 4096)
constexpr int kIsectThreads = 256;
constexpr int kUnroll = 4;         // independent list loads in flight per lane

// ---- lane class: one thread per cover edge ---------------------------------------------
template <bool PV>
__global__ void __launch_bounds__(kTileThreads) k_isect_lane(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx,
    const uint8_t* __restrict__ vinfo, const u32* __restrict__ hoff, const u32* __restrict__ hadj,
    const u32* __restrict__ htile_row, u32 nS, u32 lane_max, u64* __restrict__ ctr,
    u64* __restrict__ tri) {
  __shared__ u32 s_rp[kTileRowCap];
  __shared__ u64 s_red[5 * (kTileThreads / kWave)];
  Counts c{0, 0, 0, 0, 0};
  const u32 ntiles = (nS + kTile - 1) / kTile;
  for (u32 t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const TileInfo ti = tile_begin(hoff, htile_row, t, nS, s_rp);
    for (u32 e = ti.e0 + threadIdx.x; e < ti.e1; e += blockDim.x) {
      const u32 x = tile_row_of(ti, s_rp, hoff, e);
      u32 i = rowptr[x];
      const u32 ie = rowptr[x + 1];
      if (ie - i > lane_max) continue;
      const u32 y = hadj[e];
      u32 j = rowptr[y];
      const u32 je = rowptr[y + 1];
      c.probes += je - j;
      c.staged += ie - i;
      const u32 px = vinfo[x] & 0x80u;
      const u32 vmax = max(x, y);
      if (i < ie && j < je) {
        u32 a = colidx[i], b = colidx[j];
        while (true) {
          if (a < b) {
            if (++i == ie) break;
            a = colidx[i];
          } else if (a > b) {
            if (++j == je) break;
            b = colidx[j];
          } else {
            const u32 r = 1u + (((vinfo[a] & 0x80u) == px) ? 1u : 0u);
            count_hit<PV>(r, a, x, y, vmax, c, tri);
            if (++i == ie || ++j == je) break;
            a = colidx[i];
            b = colidx[j];
          }
        }
      }
    }
    __syncthreads();
  }
  block_flush_counts(c, 0, ctr, s_red);
}

// ---- wave class: one wavefront per staged vertex x ---------------------------------------
template <bool PV>
__global__ void __launch_bounds__(kIsectThreads) k_isect_wave(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx,
    const uint8_t* __restrict__ vinfo, const u32* __restrict__ hoff, const u32* __restrict__ hadj,
    const u32* __restrict__ wave_x, u32 nwx, Plan* __restrict__ plan, u64* __restrict__ ctr,
    u64* __restrict__ tri) {
  constexpr int kW = kIsectThreads / kWave;
  __shared__ u32 s_table[kW][kWaveSlots];
  __shared__ u32 s_incl[kW][kWave];
  __shared__ u32 s_start[kW][kWave];
  __shared__ u32 s_y[kW][kWave];
  __shared__ u64 s_red[5 * kW];
  const u32 wid = threadIdx.x / kWave, lane = lane_id();
  u32* table = s_table[wid];
  Counts c{0, 0, 0, 0, 0};
  while (true) {
    u32 idx = 0;
    if (lane == 0) idx = atomicAdd(&plan->next_wave, 1u);
    idx = __shfl(idx, 0, kWave);
    if (idx >= nwx) break;
    const u32 x = wave_x[idx];
    const u32 bx = rowptr[x], dx = rowptr[x + 1] - bx;
    const u32 px = vinfo[x] & 0x80u;
    const u32 mask = table_mask(dx, kWaveSlots);
    c.staged += lane == 0 ? dx : 0;
    for (u32 i = lane; i <= mask; i += kWave) table[i] = kInf;
    wave_lds_sync();
    for (u32 i = lane; i < dx; i += kWave) {
      const u32 w = colidx[bx + i];
      const u32 same = ((vinfo[w] & 0x80u) == px) ? 1u : 0u;
      hash_insert(table, mask, w | (same << 31));
    }
    wave_lds_sync();
    const u32 hs = hoff[x], np = hoff[x + 1] - hs;
    for (u32 pb = 0; pb < np; pb += kWave) {
      const u32 p = pb + lane;
      u32 y = 0, sy = 0, dy = 0;
      if (p < np) {
        y = hadj[hs + p];
        sy = rowptr[y];
        dy = rowptr[y + 1] - sy;
      }
      c.probes += dy;
      const u32 incl = wave_incl_scan(dy);
      const u32 total = __shfl(incl, kWave - 1, kWave);
      s_incl[wid][lane] = incl;
      s_start[wid][lane] = sy - (incl - dy);  // element k of partner l sits at start + k
      s_y[wid][lane] = y;
      wave_lds_sync();
      for (u32 k0 = 0; k0 < total; k0 += kWave * kUnroll) {
        u32 ws[kUnroll], ls[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const u32 k = k0 + u * kWave + lane;
          ls[u] = kInf;
          if (k < total) {
            // partner l: smallest l with incl[l] > k
            u32 lo = 0, hi = kWave - 1;
            while (lo < hi) {
              const u32 mid = (lo + hi) >> 1;
              if (s_incl[wid][mid] > k) hi = mid;
              else lo = mid + 1;
            }
            ls[u] = lo;
            ws[u] = colidx[s_start[wid][lo] + k];
          }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          if (ls[u] != kInf) {
            const u32 w = ws[u];
            const u32 r = hash_probe(table, mask, w);
            if (r) {
              const u32 y2 = s_y[wid][ls[u]];
              count_hit<PV>(r, w, x, y2, max(x, y2), c, tri);
            }
          }
        }
      }
      wave_lds_sync();
    }
  }
  block_flush_counts(c, 1, ctr, s_red);
}

// ---- block class: one workgroup per (x, chunk, partner segment) ------------------------
template <bool PV>
__global__ void __launch_bounds__(kIsectThreads) k_isect_block(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx,
    const uint8_t* __restrict__ vinfo, const u32* __restrict__ hoff, const u32* __restrict__ hadj,
    const Item* __restrict__ items, u32 nitems, IsectParams prm, Plan* __restrict__ plan,
    u64* __restrict__ ctr, u64* __restrict__ tri) {
  __shared__ u32 s_table[kBlockSlots];
  __shared__ u32 s_incl[kIsectThreads];
  __shared__ u32 s_start[kIsectThreads];
  __shared__ u32 s_y[kIsectThreads];
  __shared__ u32 s_tmp[kIsectThreads / kWave];
  __shared__ u64 s_red[5 * (kIsectThreads / kWave)];
  __shared__ u32 s_item;
  Counts c{0, 0, 0, 0, 0};
  while (true) {
    if (threadIdx.x == 0) s_item = atomicAdd(&plan->next_item, 1u);
    __syncthreads();
    const u32 it = s_item;
    if (it >= nitems) break;
    const Item item = items[it];
    const u32 x = item.x;
    const u32 bx = rowptr[x], dx = rowptr[x + 1] - bx;
    const u32 px = vinfo[x] & 0x80u;
    const u32 c0 = item.chunk * prm.chunk;
    const u32 clen = min(prm.chunk, dx - c0);
    const bool chunked = dx > prm.chunk;
    const u32 mask = table_mask(clen, kBlockSlots);
    c.staged += threadIdx.x == 0 ? clen : 0;
    for (u32 i = threadIdx.x; i <= mask; i += blockDim.x) s_table[i] = kInf;
    __syncthreads();
    for (u32 i = threadIdx.x; i < clen; i += blockDim.x) {
      const u32 w = colidx[bx + c0 + i];
      const u32 same = ((vinfo[w] & 0x80u) == px) ? 1u : 0u;
      hash_insert(s_table, mask, w | (same << 31));
    }
    const u32 wlo = colidx[bx + c0], whi = colidx[bx + c0 + clen - 1];
    const u32 hs = hoff[x] + item.seg * prm.seg;
    const u32 pn = min(prm.seg, hoff[x + 1] - hs);
    u32 y = 0, sy = 0, dy = 0;
    if (threadIdx.x < pn) {
      y = hadj[hs + threadIdx.x];
      sy = rowptr[y];
      u32 ey = rowptr[y + 1];
      if (chunked) {
        sy = lower_bound_g(colidx, sy, ey, wlo);
        ey = lower_bound_g(colidx, sy, ey, whi + 1u);
      }
      dy = ey - sy;
    }
    c.probes += dy;
    u32 total;
    const u32 incl = block_incl_scan(dy, s_tmp, &total);
    s_incl[threadIdx.x] = incl;
    s_start[threadIdx.x] = sy - (incl - dy);
    s_y[threadIdx.x] = y;
    __syncthreads();
    for (u32 k0 = 0; k0 < total; k0 += kIsectThreads * kUnroll) {
      u32 ws[kUnroll], ls[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const u32 k = k0 + u * kIsectThreads + threadIdx.x;
        ls[u] = kInf;
        if (k < total) {
          u32 lo = 0, hi = pn - 1;
          while (lo < hi) {
            const u32 mid = (lo + hi) >> 1;
            if (s_incl[mid] > k) hi = mid;
            else lo = mid + 1;
          }
          ls[u] = lo;
          ws[u] = colidx[s_start[lo] + k];
        }
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        if (ls[u] != kInf) {
          const u32 w = ws[u];
          const u32 r = hash_probe(s_table, mask, w);
          if (r) {
            const u32 y2 = s_y[ls[u]];
            count_hit<PV>(r, w, x, y2, max(x, y2), c, tri);
          }
        }
      }
    }
    __syncthreads();
  }
  block_flush_counts(c, 2, ctr, s_red);
}

__global__ void k_finalize(const u64* __restrict__ ctr, u64* __restrict__ out) {
  const u32 k = threadIdx.x;
  if (k < (u32)kNumCtr) {
    u64 s = 0;
    for (int i = 0; i < kCounterSlots; ++i) s += ctr[i * kNumCtr + k];
    out[k] = s;
  }
}

static u32 resident_blocks(u32 per_cu) { return (u32)num_cus() * per_cu; }

void launch_isect_lane(const u32* rowptr, const u32* colidx, const uint8_t* vinfo,
                       const u32* hoff, const u32* hadj, const u32* htile_row, u32 n, u32 nS,
                       IsectParams p, u64* ctr, u64* tri, hipStream_t s) {
  (void)n;
  if (nS == 0) return;
  const u32 g = min(cdiv(nS, kTile), resident_blocks(8));
  if (tri)
    hipLaunchKernelGGL(k_isect_lane<true>, dim3(g), dim3(kTileThreads), 0, s, rowptr, colidx,
                       vinfo, hoff, hadj, htile_row, nS, p.lane_max, ctr, tri);
  else
    hipLaunchKernelGGL(k_isect_lane<false>, dim3(g), dim3(kTileThreads), 0, s, rowptr, colidx,
                       vinfo, hoff, hadj, htile_row, nS, p.lane_max, ctr, tri);
}

void launch_isect_wave(const u32* rowptr, const u32* colidx, const uint8_t* vinfo,
                       const u32* hoff, const u32* hadj, const u32* wave_x, u32 nwx,
                       Plan* plan, u64* ctr, u64* tri, hipStream_t s) {
  if (nwx == 0) return;
  const u32 g = min(cdiv(nwx, kIsectThreads / kWave), resident_blocks(8));
  if (tri)
    hipLaunchKernelGGL(k_isect_wave<true>, dim3(g), dim3(kIsectThreads), 0, s, rowptr, colidx,
                       vinfo, hoff, hadj, wave_x, nwx, plan, ctr, tri);
  else
    hipLaunchKernelGGL(k_isect_wave<false>, dim3(g), dim3(kIsectThreads), 0, s, rowptr, colidx,
                       vinfo, hoff, hadj, wave_x, nwx, plan, ctr, tri);
}

void launch_isect_block(const u32* rowptr, const u32* colidx, const uint8_t* vinfo,
                        const u32* hoff, const u32* hadj, const Item* items, u32 nitems,
                        IsectParams p, Plan* plan, u64* ctr, u64* tri, hipStream_t s) {
  if (nitems == 0) return;
  const u32 g = min(nitems, resident_blocks(4));
  if (tri)
    hipLaunchKernelGGL(k_isect_block<true>, dim3(g), dim3(kIsectThreads), 0, s, rowptr, colidx,
                       vinfo, hoff, hadj, items, nitems, p, plan, ctr, tri);
  else
    hipLaunchKernelGGL(k_isect_block<false>, dim3(g), dim3(kIsectThreads), 0, s, rowptr, colidx,
                       vinfo, hoff, hadj, items, nitems, p, plan, ctr, tri);
}

void launch_finalize(const u64* ctr, u64* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, ctr, out);
}

}  // namespace tc

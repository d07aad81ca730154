// Cover-edge extraction (mark and compact) and intersection planning.
//
// Theorem Gen-CES (Section 4.1): the horizontal edges of a BFS — endpoints on the same
// level — cover every triangle.  Each horizontal edge {u, v} is stored once, under the
// endpoint x with the larger (degree class, ID) key; the other endpoint y goes into
// x's partner list H+(x).  That orientation makes the list staged in LDS the longer one
// and the streamed list the shorter one.  The ID order u < v of the paper's edge loop is
// applied later, in the apex rule, where it is needed.
//
// H+(x) is written in place of N(x)'s own range: hadj[rowptr[x] .. rowptr[x] + hcnt[x])
// (a partner list is never longer than the neighbour list), so one pass suffices.  The
// pass runs over CSR tiles: a wavefront ballot marks the horizontal, oriented entries, a
// block-wide prefix count ranks them, and one atomic per (tile, row) on hcnt[x] reserves
// that row's output range.
#include "tc_device.h"
#include "tc_launch.h"

namespace tc {

static inline u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }

constexpr u32 kPer = kTile / kTileThreads;  // entries per thread and tile

__device__ __forceinline__ bool cover_pred(const uint8_t* __restrict__ vinfo, u32 x, u32 y) {
  const u32 vx = vinfo[x], vy = vinfo[y];
  return ((vx ^ vy) & 0x80u) == 0 && key_less(vy & 127u, y, vx & 127u, x);
}

// Mark entries of tile ti and build s_excl[i] = number of marked entries before e0 + i
// (s_excl[kTile] = tile total).  rows[] / ys[] receive each thread's entries.
__device__ __forceinline__ void mark_tile(const TileInfo& ti, const u32* s_rp,
                                          const u32* __restrict__ rowptr,
                                          const u32* __restrict__ colidx,
                                          const uint8_t* __restrict__ vinfo, u32* s_excl,
                                          u32* s_tmp, u32 rows[kPer], u32 ys[kPer],
                                          bool preds[kPer]) {
  u32 run = 0;
#pragma unroll
  for (u32 r = 0; r < kPer; ++r) {
    const u32 e = ti.e0 + r * kTileThreads + threadIdx.x;
    bool p = false;
    u32 x = 0, y = 0;
    if (e < ti.e1) {
      x = tile_row_of(ti, s_rp, rowptr, e);
      y = colidx[e];
      p = cover_pred(vinfo, x, y);
    }
    rows[r] = x;
    ys[r] = y;
    preds[r] = p;
    // wave ballot + mbcnt for the in-wave rank, then a cross-wave prefix
    const u64 mask = __ballot(p);
    const u32 wid = threadIdx.x / kWave;
    if (lane_id() == 0) s_tmp[wid] = (u32)__popcll(mask);
    __syncthreads();
    u32 before = 0, tot = 0;
    for (u32 w = 0; w < kTileThreads / kWave; ++w) {
      const u32 c = s_tmp[w];
      if (w < wid) before += c;
      tot += c;
    }
    s_excl[r * kTileThreads + threadIdx.x] = run + before + mask_rank(mask);
    run += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) s_excl[kTile] = run;
  __syncthreads();
}

// Marked entries of row x inside the tile: [excl(start), excl(end)).
__device__ __forceinline__ void row_span(const TileInfo& ti, const u32* __restrict__ rowptr,
                                         const u32* s_rp, u32 x, u32* a, u32* b) {
  u32 lo, hi;
  if (ti.staged) {
    lo = s_rp[x - ti.r0];
    hi = s_rp[x - ti.r0 + 1];
  } else {
    lo = rowptr[x];
    hi = rowptr[x + 1];
  }
  *a = max(lo, ti.e0) - ti.e0;
  *b = min(hi, ti.e1) - ti.e0;
}

__global__ void __launch_bounds__(kTileThreads) k_extract_write(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx,
    const u32* __restrict__ tile_row, const uint8_t* __restrict__ vinfo, u32 m,
    u32* __restrict__ hcnt, u32* __restrict__ hadj) {
  __shared__ u32 s_rp[kTileRowCap];
  __shared__ u32 s_excl[kTile + 1];
  __shared__ u32 s_base[kTileRowCap];
  __shared__ u32 s_tmp[kTileThreads / kWave];
  const u32 ntiles = (m + kTile - 1) / kTile;
  for (u32 t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const TileInfo ti = tile_begin(rowptr, tile_row, t, m, s_rp);
    u32 rows[kPer], ys[kPer];
    bool preds[kPer];
    mark_tile(ti, s_rp, rowptr, colidx, vinfo, s_excl, s_tmp, rows, ys, preds);
    if (s_excl[kTile] > 0) {
      if (ti.staged) {
        // one reservation per row segment of this tile
        for (u32 x = ti.r0 + threadIdx.x; x <= ti.r1; x += blockDim.x) {
          u32 a, b;
          row_span(ti, rowptr, s_rp, x, &a, &b);
          u32 base = 0;
          if (a < b) {
            const u32 c = s_excl[b] - s_excl[a];
            if (c) base = s_rp[x - ti.r0] + atomicAdd(&hcnt[x], c) - s_excl[a];
          }
          s_base[x - ti.r0] = base;
        }
        __syncthreads();
#pragma unroll
        for (u32 r = 0; r < kPer; ++r) {
          if (preds[r]) {
            const u32 i = r * kTileThreads + threadIdx.x;
            hadj[s_base[rows[r] - ti.r0] + s_excl[i]] = ys[r];
          }
        }
      } else {
#pragma unroll
        for (u32 r = 0; r < kPer; ++r)
          if (preds[r]) hadj[rowptr[rows[r]] + atomicAdd(&hcnt[rows[r]], 1u)] = ys[r];
      }
    }
    __syncthreads();
  }
}

void launch_extract(const u32* rowptr, const u32* colidx, const u32* tile_row,
                    const uint8_t* vinfo, u32 n, u32 m, u32* hcnt, u32* hadj, hipStream_t s) {
  (void)n;
  if (m == 0) return;
  const u32 g = min(cdiv(m, kTile), (u32)num_cus() * 8);
  hipLaunchKernelGGL(k_extract_write, dim3(g), dim3(kTileThreads), 0, s, rowptr, colidx,
                     tile_row, vinfo, m, hcnt, hadj);
}

// ---- planning: split the staged endpoints x into the three intersection classes ----
// Each workgroup classifies kPlanPer * 256 consecutive vertices per pass and reserves
// its slots of the three lists with one global atomic each (a per-wavefront atomic on
// one shared counter serialises at the L2 for millions of vertices).  The total number
// of cover edges is summed on the way.
constexpr u32 kPlanPer = 8;

__global__ void __launch_bounds__(256) k_plan(const u32* __restrict__ rowptr,
                                              const u32* __restrict__ hcnt, u32 n, IsectParams p,
                                              u32* __restrict__ lane_x, u32* __restrict__ wave_x,
                                              u32* __restrict__ block_x,
                                              u32* __restrict__ block_items,
                                              Plan* __restrict__ plan) {
  __shared__ u32 s_tmp[3][256 / kWave];
  __shared__ u32 s_base[3];
  __shared__ u32 s_cov[256 / kWave];
  u32* const counters[3] = {&plan->num_lane_x, &plan->num_wave_x, &plan->num_block_x};
  const u32 span = kPlanPer * blockDim.x;
  u32 cover = 0;
  for (u32 base = blockIdx.x * span; base < n; base += gridDim.x * span) {
    u32 cls = 0;  // 2 bits per vertex: 0 no partners, 1 lane, 2 wavefront, 3 workgroup class
    u32 cnt[3] = {0, 0, 0};
#pragma unroll
    for (u32 k = 0; k < kPlanPer; ++k) {
      const u32 x = base + k * blockDim.x + threadIdx.x;
      u32 np = 0, d = 0;
      if (x < n) {
        np = hcnt[x];
        d = rowptr[x + 1] - rowptr[x];
      }
      const u32 c = np == 0 ? 0u : d <= p.lane_max ? 1u : d <= p.wave_max ? 2u : 3u;
      cover += np;
      cls |= c << (2 * k);
      cnt[0] += c == 1u;
      cnt[1] += c == 2u;
      cnt[2] += c == 3u;
    }
    u32 pos[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      u32 tot;
      const u32 incl = block_incl_scan(cnt[l], s_tmp[l], &tot);
      if (threadIdx.x == 0) s_base[l] = tot ? atomicAdd(counters[l], tot) : 0u;
      pos[l] = incl - cnt[l];
    }
    __syncthreads();
#pragma unroll
    for (int l = 0; l < 3; ++l) pos[l] += s_base[l];
#pragma unroll
    for (u32 k = 0; k < kPlanPer; ++k) {
      const u32 x = base + k * blockDim.x + threadIdx.x;
      const u32 c = (cls >> (2 * k)) & 3u;
      if (c == 1u) lane_x[pos[0]++] = x;
      if (c == 2u) wave_x[pos[1]++] = x;
      if (c == 3u) {
        block_x[pos[2]] = x;
        block_items[pos[2]] = (hcnt[x] + p.seg - 1) / p.seg;
        ++pos[2];
      }
    }
    __syncthreads();  // s_base is rewritten by the next pass
  }
  cover = wave_sum_u32(cover);
  if (lane_id() == 0) s_cov[threadIdx.x / kWave] = cover;
  __syncthreads();
  if (threadIdx.x == 0) {
    u32 t = 0;
    for (u32 w = 0; w < blockDim.x / kWave; ++w) t += s_cov[w];
    if (t) atomicAdd(&plan->num_cover, t);
  }
}

void launch_plan(const u32* rowptr, const u32* hcnt, u32 n, IsectParams p, u32* lane_x,
                 u32* wave_x, u32* block_x, u32* block_items, Plan* plan, hipStream_t s) {
  if (n == 0) return;
  const u32 g = min(cdiv(n, 256 * kPlanPer), (u32)num_cus() * 4);
  hipLaunchKernelGGL(k_plan, dim3(g), dim3(256), 0, s, rowptr, hcnt, n, p, lane_x, wave_x,
                     block_x, block_items, plan);
}

__global__ void k_fill_items(const u32* __restrict__ rowptr, const u32* __restrict__ hcnt,
                             const u32* __restrict__ block_x, const u32* __restrict__ item_off,
                             u32 nbx, IsectParams p, Item* __restrict__ items) {
  for (u32 j = blockIdx.x * blockDim.x + threadIdx.x; j < nbx; j += gridDim.x * blockDim.x) {
    const u32 x = block_x[j];
    const u32 np = hcnt[x];
    const u32 nsg = (np + p.seg - 1) / p.seg;
    u32 o = item_off[j];
    for (u32 sg = 0; sg < nsg; ++sg) items[o++] = Item{x, sg};
  }
}

void launch_fill_items(const u32* rowptr, const u32* hcnt, const u32* block_x,
                       const u32* item_off, u32 nbx, IsectParams p, Item* items,
                       hipStream_t s) {
  if (nbx == 0) return;
  const u32 g = min(cdiv(nbx, 256), (u32)num_cus() * 8);
  hipLaunchKernelGGL(k_fill_items, dim3(g), dim3(256), 0, s, rowptr, hcnt, block_x, item_off,
                     nbx, p, items);
}

}  // namespace tc

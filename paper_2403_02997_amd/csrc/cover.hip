// Cover-edge extraction (mark and compact) and intersection planning.
//
// Theorem Gen-CES (Section 4.1): the horizontal edges of a BFS — endpoints on the same
// level — cover every triangle.  Each horizontal edge {u, v} is stored once, under the
// endpoint x with the larger (degree class, ID) key; the other endpoint y goes into
// x's partner list H+(x).  That orientation makes the list staged in LDS the longer one
// and the streamed list the shorter one.  The ID order u < v of the paper's edge loop is
// applied later, in the apex rule, where it is needed.
//
// One row-centric pass per vertex v writes
//   colidx2[rowptr[v] .. split[v])       the neighbours on v's level, ascending,
//   colidx2[split[v] .. rowptr[v + 1])   the neighbours on the other levels, ascending,
//   hadj[rowptr[v] .. rowptr[v] + hcnt[v]) the partner list H+(v) (in place of N(v)'s
//                                          range: a partner list is never longer).
// Rows of at most 32 entries are handled by one lane, rows of at most 4096 by one
// wavefront (ballot ranks keep both parts in order), longer ones by a whole workgroup.  The level split
// lets the counting skip the same-level neighbours that cannot be a counted apex.
#include "tc_isect.h"

namespace tc {

static inline u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }

// Register-resident row splits.  Every entry of a row (or of a 1024-entry chunk) is
// loaded before the first vinfo gather is issued, so a row costs one load round trip
// and one gather round trip instead of one of each per few entries; the same-level and
// partner flags are kept as bit masks, so writing the row needs no second gather.

// A row of at most kSplitLane entries, by one lane.  more[b] (wavefront-uniform) says
// whether any lane's row is longer than 8 b entries; blocks of 8 past every lane's row
// are skipped.
__device__ __forceinline__ void split_lane_row_reg(const u32* __restrict__ colidx,
                                                   const uint8_t* __restrict__ vinfo, u32 v,
                                                   u32 vx, u32 lo, u32 d, const bool* more,
                                                   u32* __restrict__ colidx2,
                                                   u32* __restrict__ hadj, u32* ns_out,
                                                   u32* nh_out) {
  constexpr u32 B = 8, NB = kSplitLane / B;
  static_assert(kSplitLane <= 32, "flags are one 32-bit mask per lane");
  u32 w[kSplitLane];
#pragma unroll
  for (u32 b = 0; b < NB; ++b) {
    if (more[b]) {
#pragma unroll
      for (u32 i = 0; i < B; ++i) {
        const u32 j = b * B + i;
        w[j] = j < d ? colidx[lo + j] : v;
      }
    }
  }
  u32 sm = 0, pm = 0;
#pragma unroll
  for (u32 b = 0; b < NB; ++b) {
    if (more[b]) {
#pragma unroll
      for (u32 i = 0; i < B; ++i) {
        const u32 j = b * B + i;
        const u32 vw = vinfo[w[j]];
        const bool same = j < d && ((vw ^ vx) & 0x80u) == 0;
        const bool part = same && key_less(vw & 127u, w[j], vx & 127u, v);
        sm |= (same ? 1u : 0u) << j;
        pm |= (part ? 1u : 0u) << j;
      }
    }
  }
  const u32 ns = (u32)__popc(sm);
#pragma unroll
  for (u32 b = 0; b < NB; ++b) {
    if (more[b]) {
#pragma unroll
      for (u32 i = 0; i < B; ++i) {
        const u32 j = b * B + i;
        if (j < d) {
          const u32 below = (1u << j) - 1u;
          const u32 rs = (u32)__popc(sm & below);
          if ((sm >> j) & 1u) colidx2[lo + rs] = w[j];
          else colidx2[lo + ns + (j - rs)] = w[j];
          if ((pm >> j) & 1u) hadj[lo + (u32)__popc(pm & below)] = w[j];
        }
      }
    }
  }
  *ns_out = ns;
  *nh_out = (u32)__popc(pm);
}

// Entries c0 .. c0 + 64 kSplitRegU of the row of v at `lo` (d entries), by one wavefront,
// lane l holding entries c0 + 64 u + l.  MODE 0 counts the same-level entries (into cs)
// and the partners (into ch); MODE 1 writes them, the other-level part starting at
// ns_total; MODE 2 is a whole row in one chunk: it counts, then writes.
constexpr u32 kSplitRegU = 16;
constexpr u32 kSplitReg = kSplitRegU * kWave;  // rows up to this length in one chunk

template <int MODE>
__device__ __forceinline__ void split_chunk_reg(const u32* __restrict__ colidx,
                                                const uint8_t* __restrict__ vinfo, u32 v,
                                                u32 vx, u32 lo, u32 c0, u32 d, u32 ns_total,
                                                u32* __restrict__ colidx2, u32* __restrict__ hadj,
                                                u32& cs, u32& co, u32& ch) {
  constexpr u32 U = kSplitRegU;
  const u32 lane = lane_id();
  const u32 nu = min((d - c0 + kWave - 1) / kWave, U);  // wavefront-uniform
  u32 w[U];
#pragma unroll
  for (u32 u = 0; u < U; ++u) {
    if (u < nu) {
      const u32 j = c0 + u * kWave + lane;
      w[u] = j < d ? colidx[lo + j] : v;
    }
  }
  u32 sm = 0, pm = 0;
#pragma unroll
  for (u32 u = 0; u < U; ++u) {
    if (u < nu) {
      const u32 j = c0 + u * kWave + lane;
      const u32 vw = vinfo[w[u]];
      const bool same = j < d && ((vw ^ vx) & 0x80u) == 0;
      const bool part = same && key_less(vw & 127u, w[u], vx & 127u, v);
      sm |= (same ? 1u : 0u) << u;
      pm |= (part ? 1u : 0u) << u;
    }
  }
  if (MODE == 0) {
#pragma unroll
    for (u32 u = 0; u < U; ++u) {
      if (u < nu) {
        cs += (u32)__popcll(__ballot((sm >> u) & 1u));
        ch += (u32)__popcll(__ballot((pm >> u) & 1u));
      }
    }
    return;
  }
  u32 nsb = ns_total;
  if (MODE == 2) {
    nsb = 0;
#pragma unroll
    for (u32 u = 0; u < U; ++u)
      if (u < nu) nsb += (u32)__popcll(__ballot((sm >> u) & 1u));
  }
#pragma unroll
  for (u32 u = 0; u < U; ++u) {
    if (u < nu) {
      const u32 j = c0 + u * kWave + lane;
      const bool in = j < d;
      const bool same = (sm >> u) & 1u, part = (pm >> u) & 1u;
      const u64 ms = __ballot(same), mo = __ballot(in && !same), mh = __ballot(part);
      if (same) colidx2[lo + cs + mask_rank(ms)] = w[u];
      else if (in) colidx2[lo + nsb + co + mask_rank(mo)] = w[u];
      if (part) hadj[lo + ch + mask_rank(mh)] = w[u];
      cs += (u32)__popcll(ms);
      co += (u32)__popcll(mo);
      ch += (u32)__popcll(mh);
    }
  }
}

__global__ void __launch_bounds__(256) k_split_rows(const u32* __restrict__ rowptr,
                                                   const u32* __restrict__ colidx,
                                                   const uint8_t* __restrict__ vinfo, u32 n,
                                                   u32* __restrict__ colidx2,
                                                   u32* __restrict__ split, u32* __restrict__ hcnt,
                                                   u32* __restrict__ hadj,
                                                   u32* __restrict__ long_rows,
                                                   u32* __restrict__ num_long) {
  const u32 lane = lane_id();
  const u32 nr = (n + kWave - 1) / kWave * kWave;  // whole wavefronts iterate together
  for (u32 v = blockIdx.x * blockDim.x + threadIdx.x; v < nr; v += gridDim.x * blockDim.x) {
    u32 lo = 0, d = 0, vx = 0;
    if (v < n) {
      lo = rowptr[v];
      d = rowptr[v + 1] - lo;
      vx = vinfo[v];
    }
    const bool short_row = v < n && d <= kSplitLane;
    const bool mid = d > kSplitLane && d <= kSplitWave;
    const bool lng = d > kSplitWave;
    bool more[kSplitLane / 8];
#pragma unroll
    for (u32 b = 0; b < kSplitLane / 8; ++b) more[b] = __ballot(short_row && d > b * 8) != 0;
    if (short_row) {
      u32 ns, nh;
      split_lane_row_reg(colidx, vinfo, v, vx, lo, d, more, colidx2, hadj, &ns, &nh);
      split[v] = lo + ns;
      hcnt[v] = nh;
    }
    // long rows go to the workgroup kernel
    const u32 pos = wave_append(num_long, lng);
    if (lng) long_rows[pos] = v;
    // medium rows: one wavefront each, kSplitReg entries per chunk
    u64 mm = __ballot(mid);
    while (mm) {
      const int b = __ffsll((unsigned long long)mm) - 1;
      mm &= mm - 1;
      const u32 bv = __shfl(v, b, kWave), blo = __shfl(lo, b, kWave);
      const u32 bd = __shfl(d, b, kWave), bvx = __shfl(vx, b, kWave);
      u32 cs = 0, co = 0, ch = 0;
      if (bd <= kSplitReg) {
        split_chunk_reg<2>(colidx, vinfo, bv, bvx, blo, 0, bd, 0, colidx2, hadj, cs, co, ch);
      } else {
        u32 ns = 0, nh = 0, unused = 0;
        for (u32 c0 = 0; c0 < bd; c0 += kSplitReg)
          split_chunk_reg<0>(colidx, vinfo, bv, bvx, blo, c0, bd, 0, colidx2, hadj, ns, unused,
                             nh);
        for (u32 c0 = 0; c0 < bd; c0 += kSplitReg)
          split_chunk_reg<1>(colidx, vinfo, bv, bvx, blo, c0, bd, ns, colidx2, hadj, cs, co, ch);
      }
      if ((int)lane == b) {
        split[bv] = blo + cs;
        hcnt[bv] = ch;
      }
    }
  }
}

// Long rows: one 1024-thread workgroup per row; each wavefront takes a contiguous
// segment, and a workgroup scan of the segments' counts gives every wavefront its output
// offsets, so both parts stay in ascending order.
constexpr u32 kLongThreads = 1024;
constexpr u32 kLongWaves = kLongThreads / kWave;

__global__ void __launch_bounds__(kLongThreads) k_split_long(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx,
    const uint8_t* __restrict__ vinfo, const u32* __restrict__ long_rows,
    const u32* __restrict__ num_long, u32* __restrict__ next_long, u32* __restrict__ colidx2,
    u32* __restrict__ split, u32* __restrict__ hcnt, u32* __restrict__ hadj) {
  __shared__ u32 s_cnt[2][kLongWaves];
  __shared__ u32 s_row;
  const u32 wid = threadIdx.x / kWave, lane = lane_id();
  const u32 nl = *num_long;
  while (true) {
    if (threadIdx.x == 0) {
      const u32 i = atomicAdd(next_long, 1u);
      s_row = i < nl ? long_rows[i] : kInf;
    }
    __syncthreads();
    const u32 v = s_row;
    if (v == kInf) break;
    const u32 lo = rowptr[v], d = rowptr[v + 1] - lo, vx = vinfo[v];
    const u32 step = kWave * kSplitUnroll;
    const u32 seg = (d + kLongWaves * step - 1) / (kLongWaves * step) * step;
    const u32 j0 = min(wid * seg, d), j1 = min(j0 + seg, d);
    u32 ns = 0, no = 0, nh = 0;
    for (u32 j = j0; j < j1; j += step)
      split_steps<true>(colidx, vinfo, v, vx, lo, j, j1, 0, 0, 0, colidx2, hadj, ns, no, nh);
    if (lane == 0) {
      s_cnt[0][wid] = ns;
      s_cnt[1][wid] = nh;
    }
    __syncthreads();
    u32 bs = 0, bh = 0, ts = 0, th = 0;
    for (u32 w = 0; w < kLongWaves; ++w) {
      if (w < wid) {
        bs += s_cnt[0][w];
        bh += s_cnt[1][w];
      }
      ts += s_cnt[0][w];
      th += s_cnt[1][w];
    }
    u32 cs = 0, co = 0, ch = 0;
    for (u32 j = j0; j < j1; j += step)
      split_steps<false>(colidx, vinfo, v, vx, lo, j, j1, bs, ts + (j0 - bs), bh, colidx2, hadj,
                         cs, co, ch);
    if (threadIdx.x == 0) {
      split[v] = lo + ts;
      hcnt[v] = th;
    }
    __syncthreads();  // s_cnt and s_row are rewritten for the next row
  }
}

void launch_split_rows(const u32* rowptr, const u32* colidx, const uint8_t* vinfo, u32 n,
                       u32* colidx2, u32* split, u32* hcnt, u32* hadj, u32* long_rows,
                       u32* counters, hipStream_t s) {
  if (n == 0) return;
  const u32 g = min(cdiv(n, 256), (u32)num_cus() * 8);
  hipLaunchKernelGGL(k_split_rows, dim3(g), dim3(256), 0, s, rowptr, colidx, vinfo, n, colidx2,
                     split, hcnt, hadj, long_rows, counters);
  hipLaunchKernelGGL(k_split_long, dim3(num_cus()), dim3(kLongThreads), 0, s, rowptr, colidx,
                     vinfo, long_rows, counters, counters + 1, colidx2, split, hcnt, hadj);
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

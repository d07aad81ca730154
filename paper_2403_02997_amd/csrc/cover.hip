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
//   sabove[v]                            the first entry of the first part above v,
//   hcnt[v]                              |H+(v)|,
// and the partner records of H+(w) for its same-level neighbours w that stage v, at
// hrec[rowptr[w] .. rowptr[w] + hcnt[w]) (in place of N(w)'s range: a partner list is
// never longer).  Rows of at most 32 entries are handled by one lane, rows of at most
// 4096 by one wavefront (ballot ranks keep both parts in order), longer ones by a whole
// workgroup.  The level split and the records let the counting skip the same-level
// neighbours that cannot be a counted apex.
//
// Hub partners: when w is a hub (degree class >= the hub threshold), the edge {v, w} is
// counted by the hub pass instead: v's split still advances w's cursor (the planner's
// check) but writes bit hubidx[w] of H(v) in place of the record, and appends v's work
// items (N'(v) in kHubChunk pieces) once per row.  A hub row flags its hcnt with kHubFlag
// so that the planner gives it no intersection work.
#include "tc_isect.h"

namespace tc {

static inline u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }

// Register-resident row splits.  Every entry of a row (or of a 1024-entry chunk) is
// loaded before the first vinfo gather is issued, so a row costs one load round trip
// and one gather round trip instead of one of each per few entries; the same-level,
// partner and below-v flags are kept as bit masks, so writing the row needs no second
// gather.
//
// Besides the level-split row, the split of row v writes sabove[v] (the first
// same-level neighbour above v) and, for every same-level neighbour w that stages v
// (key(w) > key(v): v is in H+(w)), v's partner record under w: the first entry of v's
// same-level part above max(v, w) (w's rank + 1 when w > v, else v's own rank), the
// start of v's other-level part and the end of v's row.  Records are appended to w's
// slots at rowptr[w] through the cursor hcur[w] (initialised to rowptr[w]); a symmetric
// graph fills exactly hcnt[w] of them, which the planner checks.

struct SplitOut {
  u32* colidx2;
  u32* hcur;
  uint4* hrec;
  u32 m;  // records are written only below m (a guard for graphs that break the contract)
  HubView hub;
};

// Degree class from which a vertex is a hub (255: none).
__device__ __forceinline__ u32 hub_limit(const HubView& hv) {
  const u32 lim = *hv.lim;
  return lim ? lim : 255u;
}

// H(v) is gathered in LDS (kHubWords words per row being split): a lane's own slot for
// lane rows, the slot of the row's lane for wavefront rows, one per workgroup for long
// rows.  hub_or sets hub k's bit; hub_store writes the words to hy[v].
__device__ __forceinline__ void hub_or(u32* s_hy, u32 k) {
  atomicOr(&s_hy[k >> 5], 1u << (k & 31u));
}

__device__ __forceinline__ void hub_store(const HubView& hv, const u32* s_hy, u32 v) {
  uint4* d = reinterpret_cast<uint4*>(hv.hy + (size_t)v * kHubWords);
#pragma unroll
  for (u32 q = 0; q < kHubWords / 4; ++q)
    d[q] = make_uint4(s_hy[4 * q], s_hy[4 * q + 1], s_hy[4 * q + 2], s_hy[4 * q + 3]);
}

// Hub work items of row v: N'(v) = its entries from sabove[v] on (len of them), in
// pieces of kHubChunk, appended from *num_items on (one lane).
__device__ __forceinline__ void hub_items(const HubView& hv, u32 v, u32 len) {
  const u32 nch = (len + kHubChunk - 1) / kHubChunk;
  if (nch == 0) return;
  const u32 pos = atomicAdd(hv.num_items, nch);
  for (u32 i = 0; i < nch; ++i)
    if (pos + i < hv.cap) hv.items[pos + i] = make_uint2(v, i * kHubChunk);
}

// A row of at most kSplitLane entries, by one lane.  more[b] (wavefront-uniform) says
// whether any lane's row is longer than 8 b entries; blocks of 8 past every lane's row
// are skipped.
__device__ __forceinline__ void split_lane_row_reg(const u32* __restrict__ colidx,
                                                   const uint8_t* __restrict__ vinfo, u32 v,
                                                   u32 vx, u32 lo, u32 d, const bool* more,
                                                   const SplitOut& o, u32 hl, u32* s_hy,
                                                   u32* ns_out, u32* nh_out, u32* sr_out) {
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
  // same level, partner, below v, record for w, w is a hub
  u32 sm = 0, pm = 0, lm = 0, rm = 0, hm = 0;
#pragma unroll
  for (u32 b = 0; b < NB; ++b) {
    if (more[b]) {
#pragma unroll
      for (u32 i = 0; i < B; ++i) {
        const u32 j = b * B + i;
        const u32 vw = vinfo[w[j]];
        const bool same = j < d && ((vw ^ vx) & 0x80u) == 0;
        const bool part = same && key_less(vw & 127u, w[j], vx & 127u, v);
        const bool rec = same && !part && w[j] != v;
        sm |= (same ? 1u : 0u) << j;
        pm |= (part ? 1u : 0u) << j;
        lm |= (same && w[j] < v ? 1u : 0u) << j;
        rm |= (rec ? 1u : 0u) << j;
        hm |= (rec && (vw & 127u) >= hl ? 1u : 0u) << j;
      }
    }
  }
  const u32 ns = (u32)__popc(sm), sr = (u32)__popc(lm);
#pragma unroll
  for (u32 b = 0; b < NB; ++b) {
    if (more[b]) {
#pragma unroll
      for (u32 i = 0; i < B; ++i) {
        const u32 j = b * B + i;
        if (j < d) {
          const u32 rs = (u32)__popc(sm & ((1u << j) - 1u));
          if ((sm >> j) & 1u) o.colidx2[lo + rs] = w[j];
          else o.colidx2[lo + ns + (j - rs)] = w[j];
        }
      }
    }
  }
  // records, 8 entries at a time: the cursor atomics of a block are all in flight
  // before the first record is stored
#pragma unroll
  for (u32 b = 0; b < NB; ++b) {
    if (more[b] && __ballot((rm >> (b * B)) & 0xFFu) != 0) {
      u32 idx[B];
#pragma unroll
      for (u32 i = 0; i < B; ++i) {
        const u32 j = b * B + i;
        idx[i] = (rm >> j) & 1u ? atomicAdd(&o.hcur[w[j]], 1u) : o.m;
      }
#pragma unroll
      for (u32 i = 0; i < B; ++i) {
        const u32 j = b * B + i;
        if (idx[i] < o.m && !((hm >> j) & 1u)) {
          const u32 rs = (u32)__popc(sm & ((1u << j) - 1u));
          o.hrec[idx[i]] = make_uint4(w[j] > v ? lo + rs + 1 : lo + sr, lo + ns, lo + d, v);
        }
      }
    }
  }
  // hub partners: H(v) in this lane's LDS slot, and v's hub work items
  if (__ballot(hm != 0)) {
    if (hm) {
#pragma unroll
      for (u32 q = 0; q < kHubWords; ++q) s_hy[q] = 0;
    }
#pragma unroll
    for (u32 b = 0; b < NB; ++b) {
      if (more[b] && __ballot((hm >> (b * B)) & 0xFFu) != 0) {
        u32 hk[B];
#pragma unroll
        for (u32 i = 0; i < B; ++i) {
          const u32 j = b * B + i;
          hk[i] = (hm >> j) & 1u ? (u32)o.hub.hubidx[w[j]] : 0u;
        }
#pragma unroll
        for (u32 i = 0; i < B; ++i)
          if ((hm >> (b * B + i)) & 1u) hub_or(s_hy, hk[i]);
      }
    }
    if (hm) {
      hub_store(o.hub, s_hy, v);
      hub_items(o.hub, v, d - sr);
    }
  }
  *ns_out = ns;
  *nh_out = (u32)__popc(pm);
  *sr_out = sr;
}

// Entries c0 .. min(c0 + kSplitReg, cend) of the row of v (colidx[lo .. lo + d)), one
// wavefront, lane l holding entries c0 + 64 u + l (kSplitReg = 16 entries per lane).

struct ChunkRegs {
  u32 w[kSplitRegU];
  u32 sm, pm, lm, rm, hm, nu;  // flag bits per u: same level, partner of v, same level
                               // below v, record of v for w, w is a hub
};

__device__ __forceinline__ void chunk_load(const u32* __restrict__ colidx,
                                           const uint8_t* __restrict__ vinfo, u32 v, u32 vx,
                                           u32 lo, u32 c0, u32 cend, u32 hl, ChunkRegs& r) {
  constexpr u32 U = kSplitRegU;
  const u32 lane = lane_id();
  r.nu = min((cend - c0 + kWave - 1) / kWave, U);  // wavefront-uniform
#pragma unroll
  for (u32 u = 0; u < U; ++u) {
    if (u < r.nu) {
      const u32 j = c0 + u * kWave + lane;
      r.w[u] = j < cend ? colidx[lo + j] : v;
    }
  }
  r.sm = r.pm = r.lm = r.rm = r.hm = 0;
#pragma unroll
  for (u32 u = 0; u < U; ++u) {
    if (u < r.nu) {
      const u32 j = c0 + u * kWave + lane;
      const u32 vw = vinfo[r.w[u]];
      const bool same = j < cend && ((vw ^ vx) & 0x80u) == 0;
      const bool part = same && key_less(vw & 127u, r.w[u], vx & 127u, v);
      const bool rec = same && !part && r.w[u] != v;
      r.sm |= (same ? 1u : 0u) << u;
      r.pm |= (part ? 1u : 0u) << u;
      r.lm |= (same && r.w[u] < v ? 1u : 0u) << u;
      r.rm |= (rec ? 1u : 0u) << u;
      r.hm |= (rec && (vw & 127u) >= hl ? 1u : 0u) << u;
    }
  }
}

// Adds the chunk's same-level entries, partners and same-level entries below v.
__device__ __forceinline__ void chunk_count(const ChunkRegs& r, u32& ns, u32& nh, u32& sr) {
#pragma unroll
  for (u32 u = 0; u < kSplitRegU; ++u) {
    if (u < r.nu) {
      ns += (u32)__popcll(__ballot((r.sm >> u) & 1u));
      nh += (u32)__popcll(__ballot((r.pm >> u) & 1u));
      sr += (u32)__popcll(__ballot((r.lm >> u) & 1u));
    }
  }
}

// Writes the chunk: its same-level entries from same_base + cs of v's same part, its
// other-level ones from other_base + co of the row; ns / sr are the row's totals.
__device__ __forceinline__ void chunk_write(const ChunkRegs& r, u32 v, u32 lo, u32 d, u32 c0,
                                            u32 cend, u32 same_base, u32 other_base, u32 ns,
                                            u32 sr, const SplitOut& o, u32& cs, u32& co,
                                            u32* s_hy, u32& nhub) {
  const u32 lane = lane_id();
  // the cursor atomics of the whole chunk are in flight before the first store
  u32 idx[kSplitRegU];
#pragma unroll
  for (u32 u = 0; u < kSplitRegU; ++u)
    if (u < r.nu) idx[u] = (r.rm >> u) & 1u ? atomicAdd(&o.hcur[r.w[u]], 1u) : o.m;
#pragma unroll
  for (u32 u = 0; u < kSplitRegU; ++u) {
    if (u < r.nu) {
      const u32 j = c0 + u * kWave + lane;
      const bool in = j < cend;
      const bool same = (r.sm >> u) & 1u;
      const u64 ms = __ballot(same), mo = __ballot(in && !same);
      const u32 ps = same_base + cs + mask_rank(ms);  // position in v's same part
      if (same) o.colidx2[lo + ps] = r.w[u];
      else if (in) o.colidx2[lo + other_base + co + mask_rank(mo)] = r.w[u];
      if (idx[u] < o.m && !((r.hm >> u) & 1u))
        o.hrec[idx[u]] = make_uint4(r.w[u] > v ? lo + ps + 1 : lo + sr, lo + ns, lo + d, v);
      cs += (u32)__popcll(ms);
      co += (u32)__popcll(mo);
    }
  }
  if (__ballot(r.hm != 0)) {
    nhub += (u32)__popc(r.hm);
#pragma unroll
    for (u32 u = 0; u < kSplitRegU; ++u)
      if (u < r.nu && ((r.hm >> u) & 1u)) hub_or(s_hy, o.hub.hubidx[r.w[u]]);
  }
}

// Four wavefronts per SIMD (at most 128 registers): the split is bound by the latency
// of its gathers and scattered record writes, and the compiler's free choice (about
// 144 registers, three wavefronts) measured slower.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) k_split_rows(const u32* __restrict__ rowptr,
                                                   const u32* __restrict__ colidx,
                                                   const uint8_t* __restrict__ vinfo, u32 n,
                                                   SplitOut o, u32* __restrict__ split,
                                                   u32* __restrict__ sabove,
                                                   u32* __restrict__ hcnt,
                                                   u32* __restrict__ long_rows,
                                                   u32* __restrict__ num_long) {
  __shared__ u32 s_hy[256 * kHubWords];  // H(v) of the row of each lane
  const u32 lane = lane_id();
  const u32 hl = hub_limit(o.hub);
  u32* const my_hy = s_hy + threadIdx.x * kHubWords;
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
      u32 ns, nh, sr;
      split_lane_row_reg(colidx, vinfo, v, vx, lo, d, more, o, hl, my_hy, &ns, &nh, &sr);
      split[v] = lo + ns;
      sabove[v] = lo + sr;
      hcnt[v] = nh | ((vx & 127u) >= hl ? kHubFlag : 0u);
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
      u32 ns = 0, nh = 0, sr = 0, cs = 0, co = 0, nhub = 0;
      ChunkRegs r;
      // the slot of lane b (which split no lane row in this pass) gathers H(bv)
      u32* const row_hy = s_hy + (threadIdx.x - lane + (u32)b) * kHubWords;
      if (lane < kHubWords) row_hy[lane] = 0;
      if (bd <= kSplitReg) {
        chunk_load(colidx, vinfo, bv, bvx, blo, 0, bd, hl, r);
        chunk_count(r, ns, nh, sr);
        chunk_write(r, bv, blo, bd, 0, bd, 0, ns, ns, sr, o, cs, co, row_hy, nhub);
      } else {
        for (u32 c0 = 0; c0 < bd; c0 += kSplitReg) {
          chunk_load(colidx, vinfo, bv, bvx, blo, c0, bd, hl, r);
          chunk_count(r, ns, nh, sr);
        }
        for (u32 c0 = 0; c0 < bd; c0 += kSplitReg) {
          chunk_load(colidx, vinfo, bv, bvx, blo, c0, bd, hl, r);
          chunk_write(r, bv, blo, bd, c0, bd, 0, ns, ns, sr, o, cs, co, row_hy, nhub);
        }
      }
      if (__ballot(nhub != 0) && (int)lane == b) {
        hub_store(o.hub, row_hy, bv);  // the wavefront's LDS operations complete in order
        hub_items(o.hub, bv, bd - sr);
      }
      if ((int)lane == b) {
        split[bv] = blo + ns;
        sabove[bv] = blo + sr;
        hcnt[bv] = nh | ((bvx & 127u) >= hl ? kHubFlag : 0u);
      }
    }
  }
}

// Long rows: one 1024-thread workgroup per row; each wavefront takes a contiguous
// segment, and a workgroup scan of the segments' counts gives every wavefront its output
// offsets, so both parts stay in ascending order.  A segment of at most kSplitReg entries
// stays in registers across the scan.
constexpr u32 kLongThreads = 1024;
constexpr u32 kLongWaves = kLongThreads / kWave;

__global__ void __launch_bounds__(kLongThreads) k_split_long(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx,
    const uint8_t* __restrict__ vinfo, const u32* __restrict__ long_rows,
    const u32* __restrict__ num_long, u32* __restrict__ next_long, SplitOut o,
    u32* __restrict__ split, u32* __restrict__ sabove, u32* __restrict__ hcnt) {
  __shared__ u32 s_cnt[3][kLongWaves];
  __shared__ u32 s_row;
  __shared__ u32 s_hy[kHubWords];
  __shared__ u32 s_any;
  const u32 wid = threadIdx.x / kWave, lane = lane_id();
  const u32 nl = *num_long;
  const u32 hl = hub_limit(o.hub);
  while (true) {
    if (threadIdx.x == 0) {
      const u32 i = atomicAdd(next_long, 1u);
      s_row = i < nl ? long_rows[i] : kInf;
      s_any = 0;
    }
    if (threadIdx.x < kHubWords) s_hy[threadIdx.x] = 0;
    __syncthreads();
    const u32 v = s_row;
    if (v == kInf) break;
    const u32 lo = rowptr[v], d = rowptr[v + 1] - lo, vx = vinfo[v];
    const u32 seg = (d + kLongWaves * kWave - 1) / (kLongWaves * kWave) * kWave;
    const u32 j0 = min(wid * seg, d), j1 = min(j0 + seg, d);
    const bool one = seg <= kSplitReg;  // workgroup-uniform
    u32 ns = 0, nh = 0, sr = 0;
    ChunkRegs r;
    for (u32 c0 = j0; c0 < j1; c0 += kSplitReg) {
      chunk_load(colidx, vinfo, v, vx, lo, c0, j1, hl, r);
      chunk_count(r, ns, nh, sr);
    }
    if (lane == 0) {
      s_cnt[0][wid] = ns;
      s_cnt[1][wid] = nh;
      s_cnt[2][wid] = sr;
    }
    __syncthreads();
    u32 bs = 0, ts = 0, th = 0, tsr = 0;
    for (u32 w = 0; w < kLongWaves; ++w) {
      if (w < wid) bs += s_cnt[0][w];
      ts += s_cnt[0][w];
      th += s_cnt[1][w];
      tsr += s_cnt[2][w];
    }
    u32 cs = 0, co = 0, nhub = 0;
    for (u32 c0 = j0; c0 < j1; c0 += kSplitReg) {
      if (!one) chunk_load(colidx, vinfo, v, vx, lo, c0, j1, hl, r);
      chunk_write(r, v, lo, d, c0, j1, bs, ts + (j0 - bs), ts, tsr, o, cs, co, s_hy, nhub);
    }
    nhub = wave_sum_u32(nhub);
    if (lane == 0 && nhub) s_any = 1u;
    __syncthreads();  // s_hy is complete
    if (threadIdx.x == 0) {
      split[v] = lo + ts;
      sabove[v] = lo + tsr;
      hcnt[v] = th | ((vx & 127u) >= hl ? kHubFlag : 0u);
      if (s_any) {
        hub_store(o.hub, s_hy, v);
        hub_items(o.hub, v, d - tsr);
      }
    }
    __syncthreads();  // s_cnt, s_hy and s_row are rewritten for the next row
  }
}

void launch_split_rows(const u32* rowptr, const u32* colidx, const uint8_t* vinfo, u32 n, u32 m,
                       u32* colidx2, u32* split, u32* sabove, u32* hcnt, u32* hcur, uint4* hrec,
                       u32* long_rows, u32* counters, const HubView& hv, hipStream_t s) {
  if (n == 0) return;
  const SplitOut o{colidx2, hcur, hrec, m, hv};
  const u32 g = min(cdiv(n, 256), (u32)num_cus() * 8);
  hipLaunchKernelGGL(k_split_rows, dim3(g), dim3(256), 0, s, rowptr, colidx, vinfo, n, o, split,
                     sabove, hcnt, long_rows, counters);
  hipLaunchKernelGGL(k_split_long, dim3(num_cus()), dim3(kLongThreads), 0, s, rowptr, colidx,
                     vinfo, long_rows, counters, counters + 1, o, split, sabove, hcnt);
}

// ---- planning: split the staged endpoints x into the three intersection classes ----
// Each workgroup classifies kPlanPer * 256 consecutive vertices per pass and reserves
// its slots of the three lists with one global atomic each (a per-wavefront atomic on
// one shared counter serialises at the L2 for millions of vertices).  The total number
// of cover edges is summed on the way.
constexpr u32 kPlanPer = 8;

__global__ void __launch_bounds__(256) k_plan(const u32* __restrict__ rowptr,
                                              const u32* __restrict__ hcnt,
                                              const u32* __restrict__ hcur, u32 n, IsectParams p,
                                              u32* __restrict__ lane_x, u32* __restrict__ wave_x,
                                              u32* __restrict__ block_x,
                                              u32* __restrict__ block_items,
                                              Plan* __restrict__ plan) {
  __shared__ u32 s_tmp[3][256 / kWave];
  __shared__ u32 s_base[3];
  __shared__ u32 s_cov[256 / kWave];
  u32* const counters[3] = {&plan->num_lane_x, &plan->num_wave_x, &plan->num_block_x};
  const u32 span = kPlanPer * blockDim.x;
  u32 cover = 0, bad = 0;
  for (u32 base = blockIdx.x * span; base < n; base += gridDim.x * span) {
    u32 cls = 0;  // 2 bits per vertex: 0 no partners, 1 lane, 2 wavefront, 3 workgroup class
    u32 cnt[3] = {0, 0, 0};
#pragma unroll
    for (u32 k = 0; k < kPlanPer; ++k) {
      const u32 x = base + k * blockDim.x + threadIdx.x;
      u32 np = 0, d = 0;
      bool hub = false;  // a hub's cover edges go to the hub pass
      if (x < n) {
        const u32 lo = rowptr[x];
        const u32 hc = hcnt[x];
        np = hc & ~kHubFlag;
        hub = (hc & kHubFlag) != 0;
        d = rowptr[x + 1] - lo;
        bad += hcur[x] != lo + np ? 1u : 0u;
      }
      const u32 c = np == 0 || hub ? 0u : d <= p.lane_max ? 1u : d <= p.wave_max ? 2u : 3u;
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
  if (bad) atomicAdd(&plan->bad_records, bad);
  cover = wave_sum_u32(cover);
  if (lane_id() == 0) s_cov[threadIdx.x / kWave] = cover;
  __syncthreads();
  if (threadIdx.x == 0) {
    u32 t = 0;
    for (u32 w = 0; w < blockDim.x / kWave; ++w) t += s_cov[w];
    if (t) atomicAdd(&plan->num_cover, t);
  }
}

void launch_plan(const u32* rowptr, const u32* hcnt, const u32* hcur, u32 n, IsectParams p,
                 u32* lane_x, u32* wave_x, u32* block_x, u32* block_items, Plan* plan,
                 hipStream_t s) {
  if (n == 0) return;
  const u32 g = min(cdiv(n, 256 * kPlanPer), (u32)num_cus() * 4);
  hipLaunchKernelGGL(k_plan, dim3(g), dim3(256), 0, s, rowptr, hcnt, hcur, n, p, lane_x,
                     wave_x, block_x, block_items, plan);
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

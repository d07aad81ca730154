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
//           chunk goes into a 128 KB LDS hash set and each wavefront streams one
//           partner list at a time with 16-byte loads.
// The counting call runs the pruned forms of the wave and block classes: from the
// partner records and the level-split rows, x stages only its entries from sabove[x] on
// and each partner streams only the range of its record, so every common entry is a
// counted apex and the LDS sets hold IDs without level flags.  The full forms (c1, c2,
// t2 and per-vertex counts) stage all of N(x) and stream whole rows of colidx.
#include "tc_isect.h"

namespace tc {

static inline u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }

// Partner IDs of the full forms: the .w fields of the partner records.
__device__ __forceinline__ const u32* record_ids(const uint4* hrec) {
  return reinterpret_cast<const u32*>(hrec) + 3;
}

// ---- lane class: one thread per staged vertex ---------------------------------------------
template <bool PV>
__global__ void __launch_bounds__(kTileThreads) k_isect_lane(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx,
    const uint8_t* __restrict__ vinfo, const u32* __restrict__ hcnt,
    const uint4* __restrict__ hrec, const u32* __restrict__ lane_x, u32 nlx,
    u64* __restrict__ ctr, u64* __restrict__ tri) {
  __shared__ u64 s_red[5 * (kTileThreads / kWave)];
  Counts c{0, 0, 0, 0, 0};
  const u32 stride = gridDim.x * blockDim.x;
  for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t < nlx; t += stride)
    lane_vertex<PV, 4>(rowptr, 0u, colidx, vinfo, hcnt, record_ids(hrec), lane_x[t], c, tri);
  block_flush_counts(c, 0, ctr, s_red);
}

// ---- wave class: one wavefront per staged vertex x ---------------------------------------
// REC: the pruned form over the level-split rows (colidx = colidx2, tail4 = its padded
// last quad); otherwise the full form over colidx.  ST (with REC): same-level hits are
// tallied as t2 and other-level ones as c1 (the two terms of the split).
template <bool PV, bool VEC, bool REC, bool ST = false>
__global__ void __launch_bounds__(kIsectThreads) k_isect_wave(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx, u32 m,
    const u32* __restrict__ tail4, const uint8_t* __restrict__ vinfo,
    const u32* __restrict__ hcnt, const uint4* __restrict__ hrec,
    const u32* __restrict__ sabove, const u32* __restrict__ wave_x, u32 nwx,
    Plan* __restrict__ plan, u64* __restrict__ ctr, u64* __restrict__ tri) {
  constexpr int kW = kIsectThreads / kWave;
  __shared__ __align__(16) u32 s_table[kW][kWaveSlots];
  __shared__ uint4 s_pinfo[kW][kWave];  // {quad base, lo, hi, y} of each compacted partner
  __shared__ u32 s_end[kW][kWave];
  __shared__ u32 s_mark[kW][kWave];
  __shared__ u64 s_red[5 * kW];
  const u32 wid = threadIdx.x / kWave, lane = lane_id();
  Counts c{0, 0, 0, 0, 0};
  if constexpr (REC && !ST) {
    // Pruned count: 64 vertices claimed per counter atomic, their row data loaded in one
    // step; those of up to kSubMax entries are counted four at a time, one per 16-lane
    // group (subwave_vertex), the others one at a time by the whole wavefront.
    while (true) {
      u32 c0 = 0;
      if (lane == 0) c0 = atomicAdd(&plan->next_wave, (u32)kWave);
      const u32 base = __shfl(c0, 0, kWave);
      if (base >= nwx) break;  // wave-uniform
      const u32 i = base + lane;
      const bool live = i < nwx;
      u32 x = 0;
      WaveMeta mt{0, 0, 0, 0};
      if (live) {
        x = wave_x[i];
        mt = wave_meta(rowptr, sabove, hcnt, x);
      }
      const bool sub = live && mt.ex - mt.bx <= kSubMax;
      u64 todo = __ballot(sub);
      u32* gtab = s_table[wid] + (lane / kSubLanes) * kSubSlots;
      while (todo) {
        int src = -1;  // the g-th lowest remaining lane for group g
#pragma unroll
        for (u32 g = 0; g < kSubGroups; ++g) {
          const int b = todo ? __ffsll((unsigned long long)todo) - 1 : -1;
          if (b >= 0) todo &= todo - 1;
          if (g == lane / kSubLanes) src = b;
        }
        const int s0 = src < 0 ? 0 : src;
        WaveMeta gm{(u32)__shfl(mt.bx, s0, kWave), (u32)__shfl(mt.ex, s0, kWave),
                    (u32)__shfl(mt.sb, s0, kWave), (u32)__shfl(mt.np, s0, kWave)};
        // every lane shuffles (the source lane may sit in a group without a vertex), then
        // a group without one drops the value
        const u32 xs = (u32)__shfl(x, s0, kWave);
        const u32 gx = src < 0 ? 0u : xs;
        if (src < 0) gm = WaveMeta{0, 0, 0, 0};
        Tally tl{0, 0, 0, 0};
        subwave_vertex<kPartRec, PV>(colidx, m, 0u, nullptr, hrec, nullptr, gm, gtab, tl, c, gx,
                                     tri);
        tl.fold(c);
      }
      todo = __ballot(live && !sub);
      while (todo) {
        const int b = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const WaveMeta mb{(u32)__shfl(mt.bx, b, kWave), (u32)__shfl(mt.ex, b, kWave),
                          (u32)__shfl(mt.sb, b, kWave), (u32)__shfl(mt.np, b, kWave)};
        Tally tl{0, 0, 0, 0};
        wave_vertex<PV, VEC, REC, 4, ST>(rowptr, 0u, colidx, m, tail4, vinfo, hcnt,
                                         record_ids(hrec), hrec, nullptr, (u32)__shfl(x, b, kWave),
                                         mb, s_table[wid], s_pinfo[wid], s_end[wid], s_mark[wid],
                                         tl, c, tri);
        tl.fold(c);
      }
    }
  } else {
    // Vertices are claimed kWaveClaim at a time (one counter atomic per vertex would
    // serialise hundreds of thousands of same-address atomics at the L2), with all their
    // IDs loaded at once; the next vertex's row data is loaded while the current one runs.
    u32 base = 0, cnt = 0, xs = 0, j = 0;
    auto claim = [&]() {
      u32 c0 = 0;
      if (lane == 0) c0 = atomicAdd(&plan->next_wave, kWaveClaim);
      base = __shfl(c0, 0, kWave);
      cnt = base < nwx ? min(kWaveClaim, nwx - base) : 0u;
      xs = lane < cnt ? wave_x[base + lane] : 0u;
      j = 0;
    };
    claim();
    if (cnt > 0) {
      u32 x = __shfl(xs, 0, kWave);
      j = 1;
      WaveMeta mt{};
      if (REC) mt = wave_meta(rowptr, sabove, hcnt, x);
      while (true) {
        if (j == cnt) claim();
        const bool more = cnt > 0;
        u32 x1 = 0;
        WaveMeta mt1{};
        if (more) {
          x1 = __shfl(xs, j, kWave);
          ++j;
          if (REC) mt1 = wave_meta(rowptr, sabove, hcnt, x1);
        }
        Tally tl{0, 0, 0, 0};
        wave_vertex<PV, VEC, REC, 4, ST>(rowptr, 0u, colidx, m, tail4, vinfo, hcnt, record_ids(hrec),
                                     hrec, nullptr, x, mt, s_table[wid], s_pinfo[wid], s_end[wid],
                                     s_mark[wid], tl, c, tri);
        tl.fold(c);
        if (!more) break;
        x = x1;
        mt = mt1;
      }
    }
  }
  block_flush_counts(c, 1, ctr, s_red);
}

// ---- block class: one 1024-thread workgroup per (x, segment of partners) ----------------
template <bool PV, bool VEC, bool PRUNED, bool ST = false>
__global__ void __launch_bounds__(kBigThreads) k_isect_block(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx, u32 m,
    const u32* __restrict__ tail4, const u32* __restrict__ colidx2,
    const u32* __restrict__ split, const u32* __restrict__ sabove,
    const u32* __restrict__ tail4b, const uint8_t* __restrict__ vinfo,
    const u32* __restrict__ hcnt, const uint4* __restrict__ hrec, const Item* __restrict__ items,
    u32 nitems, IsectParams prm, Plan* __restrict__ plan, u64* __restrict__ ctr,
    u64* __restrict__ tri) {
  __shared__ __align__(16) u32 s_table[kBigSlots];
  __shared__ u32 s_qincl[kBigSeg];
  __shared__ uint4 s_pinfo[kBigSeg];  // {quad base, lo, hi, y} of each partner
  __shared__ u32 s_tmp[kBigWaves];
  __shared__ u64 s_red[5 * kBigWaves];
  __shared__ u32 s_item;
  __shared__ u32 s_ycnt[PV ? kBigSeg : 1];
  const BlockShared sh{s_table, s_qincl, s_pinfo, s_tmp, s_ycnt};
  const u32 tid = threadIdx.x;
  Counts c{0, 0, 0, 0, 0};
  Tally tl{0, 0, 0, 0};
  while (true) {
    if (tid == 0) s_item = atomicAdd(&plan->next_item, 1u);
    __syncthreads();
    const u32 it = s_item;
    if (it >= nitems) break;
    const Item item = items[it];
    if constexpr (PRUNED)
      block_item_rec<VEC, true, ST, kPartRec, kQuadUnroll, PV>(
          rowptr, 0u, colidx2, m, tail4b, split, sabove, hcnt, hrec, nullptr, nullptr, item.x,
          item.seg, prm, sh, tl, c, tri);
    else
      block_item<VEC, 4>(rowptr, 0u, colidx, m, tail4, vinfo, hcnt, record_ids(hrec), item.x,
                         item.seg, prm, sh, tl, c);
    tl.fold(c);
  }
  block_flush_counts(c, 2, ctr, s_red);
}

// Copy of colidx's last partial 16-byte quad (elements m & ~3 .. m-1), padded with kInf.
__global__ void k_tail4(const u32* __restrict__ colidx, u32 m, u32* __restrict__ tail4) {
  const u32 i = threadIdx.x;
  if (i < 4) {
    const u32 idx = (m & ~3u) + i;
    tail4[i] = idx < m ? colidx[idx] : kInf;
  }
}

void launch_tail4(const u32* colidx, u32 m, u32* tail4, hipStream_t s) {
  hipLaunchKernelGGL(k_tail4, dim3(1), dim3(64), 0, s, colidx, m, tail4);
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
                       const SplitView& sv, const u32* lane_x, u32 nlx, u64* ctr, u64* tri,
                       hipStream_t s) {
  if (nlx == 0) return;
  const u32 g = min(cdiv(nlx, kTileThreads), resident_blocks(8));
  if (tri)
    hipLaunchKernelGGL(k_isect_lane<true>, dim3(g), dim3(kTileThreads), 0, s, rowptr, colidx,
                       vinfo, sv.hcnt, sv.hrec, lane_x, nlx, ctr, tri);
  else
    hipLaunchKernelGGL(k_isect_lane<false>, dim3(g), dim3(kTileThreads), 0, s, rowptr, colidx,
                       vinfo, sv.hcnt, sv.hrec, lane_x, nlx, ctr, tri);
}

void launch_isect_wave(const u32* rowptr, const u32* colidx, u32 m, const u32* tail4,
                       const uint8_t* vinfo, const SplitView& sv, const u32* wave_x, u32 nwx,
                       Plan* plan, u64* ctr, u64* tri, bool pruned, bool split_stats,
                       hipStream_t s) {
  if (nwx == 0) return;
  const u32 g = min(cdiv(nwx, kIsectThreads / kWave), resident_blocks(8));
  const bool rec = pruned;
  const u32* src = rec ? sv.colidx2 : colidx;  // the streamed and staged rows
  const u32* tail = rec ? sv.tail4b : tail4;
  const bool vec = ((uintptr_t)src & 15u) == 0;
#define TC_LAUNCH_WAVE(PV, VEC, REC, ST)                                                       \
  hipLaunchKernelGGL((k_isect_wave<PV, VEC, REC, ST>), dim3(g), dim3(kIsectThreads), 0, s,      \
                     rowptr, src, m, tail, vinfo, sv.hcnt, sv.hrec, sv.sabove, wave_x, nwx,     \
                     plan, ctr, tri)
  if (tri) {  // per-vertex counts: the pruned form
    if (vec) TC_LAUNCH_WAVE(true, true, true, false);
    else TC_LAUNCH_WAVE(true, false, true, false);
  } else if (rec && split_stats) {
    if (vec) TC_LAUNCH_WAVE(false, true, true, true);
    else TC_LAUNCH_WAVE(false, false, true, true);
  } else if (rec) {
    if (vec) TC_LAUNCH_WAVE(false, true, true, false);
    else TC_LAUNCH_WAVE(false, false, true, false);
  } else {
    if (vec) TC_LAUNCH_WAVE(false, true, false, false);
    else TC_LAUNCH_WAVE(false, false, false, false);
  }
#undef TC_LAUNCH_WAVE
}

void launch_isect_block(const u32* rowptr, const u32* colidx, u32 m, const u32* tail4,
                        const uint8_t* vinfo, const SplitView& sv, const Item* items,
                        u32 nitems, IsectParams p, Plan* plan, u64* ctr, u64* tri, bool pruned,
                        bool split_stats, hipStream_t s) {
  if (nitems == 0) return;
  const u32 g = min(nitems, resident_blocks(1));
  const bool rec = pruned;
  const bool vec = ((uintptr_t)(rec ? sv.colidx2 : colidx) & 15u) == 0;
#define TC_LAUNCH_BLOCK(PV, VEC, PR, ST)                                                       \
  hipLaunchKernelGGL((k_isect_block<PV, VEC, PR, ST>), dim3(g), dim3(kBigThreads), 0, s,        \
                     rowptr, colidx, m, tail4, sv.colidx2, sv.split, sv.sabove, sv.tail4b,      \
                     vinfo, sv.hcnt, sv.hrec, items, nitems, p, plan, ctr, tri)
  if (tri) {  // per-vertex counts: the pruned form
    if (vec) TC_LAUNCH_BLOCK(true, true, true, false);
    else TC_LAUNCH_BLOCK(true, false, true, false);
  } else if (rec && split_stats) {
    if (vec) TC_LAUNCH_BLOCK(false, true, true, true);
    else TC_LAUNCH_BLOCK(false, false, true, true);
  } else if (rec) {
    if (vec) TC_LAUNCH_BLOCK(false, true, true, false);
    else TC_LAUNCH_BLOCK(false, false, true, false);
  } else {
    if (vec) TC_LAUNCH_BLOCK(false, true, false, false);
    else TC_LAUNCH_BLOCK(false, false, false, false);
  }
#undef TC_LAUNCH_BLOCK
}

void launch_finalize(const u64* ctr, u64* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, ctr, out);
}

}  // namespace tc

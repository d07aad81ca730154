// Hub pass: the cover edges staged under the highest-degree vertices, counted one
// partner at a time.
//
// For a cover edge {x, y} staged under x, the apex test of CETC-Seq (Section 4.2) counts
// the w in N(x) ∩ N(y) with L(w) != L(x) or w > max(x, y).  With S(x) = x's other-level
// neighbours and its same-level neighbours above x, and N'(y) the same for y, that count
// is |S(x) ∩ N'(y)|: a w of N'(y) on x's level and at or below x is in neither part of
// S(x).  For the hubs h_0 .. h_{K-1} (K <= 256) the pass stores, per vertex w, the bit
// mask M(w) of the hubs whose S holds w, and per partner y the mask H(y) of the hubs
// that stage y.  Then
//     sum over hubs x staging y of |S(x) ∩ N'(y)|  =  sum over w in N'(y) of |M(w) & H(y)|,
// one streamed N'(y) and one mask lookup per entry instead of one intersection per hub
// edge.  In R-MAT graphs the hubs share most of their partners, so the pass reads each
// partner list once where the per-edge intersections read it once per hub.
//
// Steps: k_hub_select picks the hub classes from the degree-class histogram and numbers
// the hubs; the split (cover.hip) writes H(y) and the work items; k_hub_cuts and
// k_hub_mask transpose the hubs' S lists into the vertex-major masks M, one ID window
// per workgroup in LDS; k_hub_count streams the items.
#include "tc_device.h"
#include "tc_launch.h"

namespace tc {

static inline u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }

// ---- hub selection -----------------------------------------------------------------
// The hubs are the vertices of degree class >= c*, the smallest class >= min_class whose
// vertices and those of all higher classes number at most max_hubs (none if there are
// no such vertices).  Every workgroup derives c* from the histogram; hubs take indices in
// the order their workgroups reach the counter.
__global__ void __launch_bounds__(256) k_hub_select(const uint8_t* __restrict__ vinfo, u32 n,
                                                    const u32* __restrict__ hist, HubParams hp,
                                                    uint8_t* __restrict__ hubidx,
                                                    u32* __restrict__ hublist,
                                                    Plan* __restrict__ plan) {
  __shared__ u32 s_h[128];
  __shared__ u32 s_lim;
  const u32 t = threadIdx.x;
  if (t < 128) s_h[t] = hist[t];
  if (t == 0) s_lim = 128;
  __syncthreads();
  if (t < 128 && t >= max(hp.min_class, 1u)) {
    u32 suf = 0;
    for (u32 c = t; c < 128; ++c) suf += s_h[c];
    if (suf > 0 && suf <= hp.max_hubs) atomicMin(&s_lim, t);
  }
  __syncthreads();
  const u32 lim = s_lim;  // 128: no hubs
  if (blockIdx.x == 0 && t == 0) plan->hub_lim = lim < 128 ? lim : 0u;
  if (lim >= 128) return;
  const u32 nr = (n + kWave - 1) / kWave * kWave;
  for (u32 v = blockIdx.x * blockDim.x + t; v < nr; v += gridDim.x * blockDim.x) {
    const bool hub = v < n && (vinfo[v] & 127u) >= lim;
    const u32 k = wave_append(&plan->num_hubs, hub);
    if (hub) {
      hubidx[v] = (uint8_t)k;  // k < max_hubs <= 256
      hublist[k] = v;
    }
  }
}

void launch_hub_select(const uint8_t* vinfo, u32 n, const u32* class_hist, HubParams hp,
                       uint8_t* hubidx, u32* hublist, Plan* plan, hipStream_t s) {
  if (n == 0 || hp.max_hubs == 0) return;
  const u32 g = min(cdiv(n, 256), (u32)num_cus() * 4);
  hipLaunchKernelGGL(k_hub_select, dim3(g), dim3(256), 0, s, vinfo, n, class_hist, hp, hubidx,
                     hublist, plan);
}

// ---- masks M(w) ---------------------------------------------------------------------
// Hub k's S list is two sorted runs of colidx2: run 2k = its same-level part above h_k
// (sabove .. split), run 2k + 1 = its other-level part (split .. row end).  The masks are
// built one window of kHubLdsWords / NW IDs at a time in LDS; cut[r * (nwin + 1) + b] is the
// first position of run r whose ID is >= b * window (the run's end if none).
constexpr u32 kHubLdsWords = 16384;  // 64 KB of LDS per window
constexpr u32 kHubThreads = 256;

u32 hub_mask_words(u32 nhubs) { return nhubs <= 128 ? 4u : 8u; }
static u32 hub_window(u32 nw) { return kHubLdsWords / nw; }
static u32 hub_windows(u32 n, u32 nw) { return cdiv(n, hub_window(nw)); }

size_t hub_cut_words(u32 nhubs, u32 n) {
  const u32 nw = hub_mask_words(nhubs);
  return (size_t)2 * nhubs * (hub_windows(n, nw) + 1);
}

__device__ __forceinline__ void hub_run(const u32* __restrict__ rowptr,
                                        const u32* __restrict__ split,
                                        const u32* __restrict__ sabove,
                                        const u32* __restrict__ hublist, u32 r, u32& lo,
                                        u32& hi) {
  const u32 h = hublist[r >> 1];
  lo = (r & 1u) ? split[h] : sabove[h];
  hi = (r & 1u) ? rowptr[h + 1] : split[h];
}

__global__ void __launch_bounds__(256) k_hub_cuts(const u32* __restrict__ rowptr,
                                                  const u32* __restrict__ colidx2,
                                                  const u32* __restrict__ split,
                                                  const u32* __restrict__ sabove,
                                                  const u32* __restrict__ hublist, u32 nruns,
                                                  u32 nwin, u32 win, u32* __restrict__ cuts) {
  const u32 total = nruns * (nwin + 1);
  for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const u32 r = i / (nwin + 1), b = i - r * (nwin + 1);
    u32 lo, hi;
    hub_run(rowptr, split, sabove, hublist, r, lo, hi);
    cuts[i] = lower_bound_g(colidx2, lo, hi, b * win);  // b * win < 2^31 (n < 2^30)
  }
}

// One workgroup per window: every hub's entries in the window set its bit in LDS, then
// the window's masks are written out whole (no clearing pass, no global atomics).
template <u32 NW>
__global__ void __launch_bounds__(kHubThreads) k_hub_mask(const u32* __restrict__ colidx2,
                                                          const u32* __restrict__ cuts,
                                                          u32 nhubs, u32 n, u32 nwin,
                                                          u32* __restrict__ hubmask) {
  constexpr u32 W = kHubLdsWords / NW;
  __shared__ uint4 s_tab4[kHubLdsWords / 4];
  __shared__ u32 s_incl[kMaxHubs];      // inclusive prefix of the hubs' entry counts
  __shared__ u32 s_s0[kMaxHubs], s_s1[kMaxHubs], s_l0[kMaxHubs];
  __shared__ u32 s_tmp[kHubThreads / kWave];
  u32* s_tab = reinterpret_cast<u32*>(s_tab4);
  const u32 t = threadIdx.x;
  for (u32 b = blockIdx.x; b < nwin; b += gridDim.x) {
    const u32 wb = b * W;
    for (u32 i = t; i < kHubLdsWords / 4; i += kHubThreads) s_tab4[i] = make_uint4(0, 0, 0, 0);
    u32 len = 0;
    if (t < nhubs) {
      const u32* c0 = cuts + (size_t)(2 * t) * (nwin + 1) + b;
      const u32* c1 = c0 + (nwin + 1);
      const u32 s0 = c0[0], l0 = c0[1] - s0, s1 = c1[0], l1 = c1[1] - s1;
      s_s0[t] = s0;
      s_s1[t] = s1;
      s_l0[t] = l0;
      len = l0 + l1;
    }
    u32 tot;
    const u32 incl = block_incl_scan(len, s_tmp, &tot);  // ends with a barrier
    if (t < nhubs) s_incl[t] = incl;
    __syncthreads();
    for (u32 e = t; e < tot; e += kHubThreads) {
      // hub k of entry e: the smallest k with s_incl[k] > e
      u32 lo = 0, hi = nhubs - 1;
      while (lo < hi) {
        const u32 mid = (lo + hi) >> 1;
        if (s_incl[mid] > e) hi = mid;
        else lo = mid + 1;
      }
      const u32 k = lo;
      const u32 first = k ? s_incl[k - 1] : 0u;
      const u32 j = e - first;
      const u32 l0 = s_l0[k];
      const u32 pos = j < l0 ? s_s0[k] + j : s_s1[k] + (j - l0);
      const u32 w = colidx2[pos];  // wb <= w < wb + W by the cuts
      atomicOr(&s_tab[(w - wb) * NW + (k >> 5)], 1u << (k & 31u));
    }
    __syncthreads();
    const u32 nid = min(W, n - wb);
    uint4* dst = reinterpret_cast<uint4*>(hubmask + (size_t)wb * NW);
    for (u32 i = t; i < nid * NW / 4; i += kHubThreads) dst[i] = s_tab4[i];
    __syncthreads();  // the table is cleared for the next window
  }
}

// ---- counting -------------------------------------------------------------------------
// One wavefront per work item (y, offset): up to kHubChunk entries of N'(y), each
// looked up in M and masked with H(y).  The entries of a lane are all loaded before the
// mask lookups, and the lookups of a lane are all in flight before the first count.
// ST: the apexes w before split[y] (on y's level, hence on the hub's) are tallied in the
// t2 counter, the others in c1 (the two terms of the split).
constexpr u32 kHubU = kHubChunk / kWave;  // entries per lane and item

// One 32-bit word c of a 16-byte mask word.
__device__ __forceinline__ u32 word_of(const uint4& v, u32 c) {
  return c == 0 ? v.x : c == 1 ? v.y : c == 2 ? v.z : v.w;
}

// PV: per-vertex counts.  Each unit of popcount(M(w) & H(y)) is the triangle {h, y, w} of
// one hub h: t(w) gets the popcount of its entry, t(y) the item's sum, and t(h) for every
// hub bit of H(y) the number of the item's entries whose mask holds it (ballot counts,
// gathered per workgroup in LDS and added once per hub at the end; hublist maps the bit
// to the hub's ID).
template <u32 NW, bool ST, bool PV = false>
__global__ void __launch_bounds__(256) k_hub_count(const u32* __restrict__ rowptr,
                                                   const u32* __restrict__ colidx2,
                                                   const u32* __restrict__ sabove,
                                                   const u32* __restrict__ split,
                                                   const u32* __restrict__ hy,
                                                   const u32* __restrict__ hubmask,
                                                   const uint2* __restrict__ items, u32 nitems,
                                                   u64* __restrict__ ctr,
                                                   const u32* __restrict__ hublist, u32 nhubs,
                                                   u64* __restrict__ tri) {
  static_assert(!(PV && ST), "per-vertex counts tally no split");
  constexpr u32 NQ = NW / 4;  // 16-byte words per mask
  __shared__ u64 s_red[2 * 256 / kWave];
  __shared__ unsigned long long s_hub[PV ? kMaxHubs : 1];
  if (PV) {
    for (u32 k = threadIdx.x; k < kMaxHubs; k += blockDim.x) s_hub[k] = 0;
    __syncthreads();
  }
  const u32 lane = lane_id();
  const u32 wid = threadIdx.x / kWave;
  const u32 gw = blockIdx.x * (blockDim.x / kWave) + wid;
  const u32 nwv = gridDim.x * (blockDim.x / kWave);
  const uint4* __restrict__ m4 = reinterpret_cast<const uint4*>(hubmask);
  u64 acc = 0, acc_same = 0;
  for (u32 i = gw; i < nitems; i += nwv) {
    const uint2 it = items[i];
    const u32 y = it.x;
    const u32 b = sabove[y] + it.y;               // < rowptr[y + 1] (items cover N'(y))
    const u32 e = b + min(kHubChunk, rowptr[y + 1] - b);
    const u32 ys = ST ? split[y] : 0u;            // start of y's other-level part
    uint4 hq[NQ];
    const uint4* hy4 = reinterpret_cast<const uint4*>(hy + (size_t)y * kHubWords);
#pragma unroll
    for (u32 q = 0; q < NQ; ++q) hq[q] = hy4[q];
    u32 w[kHubU];
#pragma unroll
    for (u32 u = 0; u < kHubU; ++u) {
      const u32 j = b + u * kWave + lane;
      w[u] = j < e ? colidx2[j] : kInf;
    }
    u32 part = 0, part_same = 0;
    constexpr u32 G = 8;  // lookups in flight per lane
#pragma unroll
    for (u32 u0 = 0; u0 < kHubU; u0 += G) {
      if (__ballot(w[u0] != kInf) == 0) break;  // past the end for every lane
      uint4 mv[G][NQ];
#pragma unroll
      for (u32 u = 0; u < G; ++u)
#pragma unroll
        for (u32 q = 0; q < NQ; ++q)
          mv[u][q] = w[u0 + u] != kInf ? m4[(size_t)w[u0 + u] * NQ + q] : make_uint4(0, 0, 0, 0);
#pragma unroll
      for (u32 u = 0; u < G; ++u) {
        u32 h = 0;
#pragma unroll
        for (u32 q = 0; q < NQ; ++q)
          h += __popc(mv[u][q].x & hq[q].x) + __popc(mv[u][q].y & hq[q].y) +
               __popc(mv[u][q].z & hq[q].z) + __popc(mv[u][q].w & hq[q].w);
        if (ST && b + (u0 + u) * kWave + lane < ys) part_same += h;
        else part += h;
        if (PV) tri_add(tri, w[u0 + u], h);  // h is 0 past the end (zero masks)
      }
      if (PV) {
#pragma unroll
        for (u32 q = 0; q < NQ; ++q) {
#pragma unroll
          for (u32 cw = 0; cw < 4; ++cw) {
            u32 hw = (u32)__builtin_amdgcn_readfirstlane((int)word_of(hq[q], cw));  // uniform
            while (hw) {
              const u32 bit = __ffs(hw) - 1;
              hw &= hw - 1;
              u32 cnt = 0;
#pragma unroll
              for (u32 u = 0; u < G; ++u)
                cnt += (u32)__popcll(__ballot((word_of(mv[u][q], cw) >> bit) & 1u));
              if (lane == 0 && cnt) atomicAdd(&s_hub[(4 * q + cw) * 32 + bit], (unsigned long long)cnt);
            }
          }
        }
      }
    }
    acc += part;
    acc_same += part_same;
    if (PV) {
      const u64 sy = wave_sum_u64(part);
      if (lane == 0) tri_add(tri, y, sy);
    }
  }
  acc = wave_sum_u64(acc);
  if (ST) acc_same = wave_sum_u64(acc_same);
  if (lane == 0) {
    s_red[wid] = acc;
    if (ST) s_red[blockDim.x / kWave + wid] = acc_same;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 sum = 0, sum_same = 0;
    for (u32 k = 0; k < blockDim.x / kWave; ++k) {
      sum += s_red[k];
      if (ST) sum_same += s_red[blockDim.x / kWave + k];
    }
    u64* slot = &ctr[(blockIdx.x % kCounterSlots) * kNumCtr];
    if (sum) atomicAdd((unsigned long long*)&slot[0], (unsigned long long)sum);
    if (sum_same) atomicAdd((unsigned long long*)&slot[2], (unsigned long long)sum_same);
  }
  if (PV) {
    // every wavefront's hub counts are in after the barrier above
    for (u32 k = threadIdx.x; k < nhubs; k += blockDim.x) tri_add(tri, hublist[k], s_hub[k]);
  }
}

void launch_hub_masks(const u32* rowptr, const u32* colidx2, const u32* split,
                      const u32* sabove, const u32* hublist, u32 nhubs, u32 n, u32* cuts,
                      u32* hubmask, hipStream_t s) {
  if (nhubs == 0 || n == 0) return;
  const u32 nw = hub_mask_words(nhubs);
  const u32 win = hub_window(nw), nwin = hub_windows(n, nw);
  const u32 ncut = 2 * nhubs * (nwin + 1);
  hipLaunchKernelGGL(k_hub_cuts, dim3(min(cdiv(ncut, 256), (u32)num_cus() * 8)), dim3(256), 0,
                     s, rowptr, colidx2, split, sabove, hublist, 2 * nhubs, nwin, win, cuts);
  const u32 gm = min(nwin, (u32)num_cus() * 4);
  if (nw == 4)
    hipLaunchKernelGGL(k_hub_mask<4>, dim3(gm), dim3(kHubThreads), 0, s, colidx2, cuts, nhubs, n,
                       nwin, hubmask);
  else
    hipLaunchKernelGGL(k_hub_mask<8>, dim3(gm), dim3(kHubThreads), 0, s, colidx2, cuts, nhubs, n,
                       nwin, hubmask);
}

void launch_hub_count(const u32* rowptr, const u32* colidx2, const u32* sabove,
                      const u32* split, u32 nhubs, const u32* hy, const u32* hubmask,
                      const uint2* items, u32 nitems, u64* ctr, bool split_stats,
                      const u32* hublist, u64* tri, hipStream_t s) {
  if (nhubs == 0 || nitems == 0) return;
  const u32 gc = min(cdiv(nitems, 256 / kWave), (u32)num_cus() * 8);
#define TC_LAUNCH_HUB(NW, ST, PV)                                                              \
  hipLaunchKernelGGL((k_hub_count<NW, ST, PV>), dim3(gc), dim3(256), 0, s, rowptr, colidx2,     \
                     sabove, split, hy, hubmask, items, nitems, ctr, hublist, nhubs, tri)
  if (hub_mask_words(nhubs) == 4) {
    if (tri) TC_LAUNCH_HUB(4, false, true);
    else if (split_stats) TC_LAUNCH_HUB(4, true, false);
    else TC_LAUNCH_HUB(4, false, false);
  } else {
    if (tri) TC_LAUNCH_HUB(8, false, true);
    else if (split_stats) TC_LAUNCH_HUB(8, true, false);
    else TC_LAUNCH_HUB(8, false, false);
  }
#undef TC_LAUNCH_HUB
}

}  // namespace tc

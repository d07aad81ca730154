// Batched counting: many independent graphs in one persistent launch.
//
// A planner orders the graphs by stored entries, largest power-of-two class first.  Then
// one persistent grid of 1024-thread workgroups (one per compute unit) pops graphs from
// that order; the workgroup that takes a graph runs the whole method on it without
// leaving the kernel and without waiting for any other workgroup:
//
//   1. component roots: union-find with smallest-ID roots (the root each restart of
//      the paper's CETC-Seq BFS loop starts from);
//   2. level BFS from all roots, one frontier level per workgroup barrier;
//   3. per-vertex info byte (level parity, degree class);
//   4. level split of every row and the partner lists H+(x) (Theorem Gen-CES), with the
//      same row routines as the single-graph path (rows longer than kSplitWave by the
//      whole workgroup);
//   5. intersections with the apex rule of CETC-Seq (Section 4.2), with the same
//      per-vertex routines as the single-graph kernels: lane merges for d(x) <= lane_max,
//      one wavefront per staged vertex for d(x) <= wave_max (the 128 KB table split into
//      16 wavefront tables), and the pruned workgroup passes for longer lists;
//   6. counts[g] = c1 + t2.
//
// Per-vertex scratch (parent, level, queue, info, partner counts, row records) lives in
// the workspace at the graph's row offset, per-entry scratch (level-split rows, partner
// lists) at its column offset, so graphs never share memory and the call allocates
// nothing.
#include "tc_isect.h"

namespace tc {

constexpr int kBT = kBigThreads;   // threads per workgroup
constexpr int kBW = kBT / kWave;   // wavefronts per workgroup
constexpr u32 kBuckets = 40;       // planner cost classes

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
    ctl->pad[0] = 0;
    ctl->pad[1] = 0;
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
// i < count.  Each wavefront takes 64 list entries and walks the concatenation of their
// adjacency lists, 64 lanes wide and kTravU positions per lane in flight: the owner of
// position k is the first lane whose inclusive degree prefix exceeds k (a binary search
// over the lanes' prefixes with cross-lane reads), so short lists cost no extra round
// trips and long ones are read coalesced.  f is reached by all lanes of a wavefront
// together (for wave_append).
constexpr u32 kTravU = 4;

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
    const u32 incl = wave_incl_scan(d);
    const u32 total = __shfl(incl, kWave - 1, kWave);
    const u32 base = lo - (incl - d);  // entry of position k of this lane's list: base + k
    for (u32 k0 = 0; k0 < total; k0 += kWave * kTravU) {
      u32 vv[kTravU], uu[kTravU];
      bool act[kTravU];
#pragma unroll
      for (u32 t = 0; t < kTravU; ++t) {
        const u32 k = k0 + t * kWave + lane;
        act[t] = k < total;
        // first lane j with incl_j > k (lanes past the total search harmlessly)
        u32 a = 0, b = kWave - 1;
#pragma unroll
        for (int st = 0; st < 6; ++st) {
          const u32 mid = (a + b) >> 1;
          const u32 im = (u32)__shfl(incl, (int)mid, kWave);
          if (im > k) b = mid;
          else a = mid + 1;
        }
        uu[t] = (u32)__shfl(u, (int)a, kWave);
        const u32 eb = (u32)__shfl(base, (int)a, kWave);
        vv[t] = act[t] ? ci[eb + k] : 0u;
      }
#pragma unroll
      for (u32 t = 0; t < kTravU; ++t) f(uu[t], vv[t], act[t]);
    }
  }
}

// Vertices of a graph whose BFS keeps its visited bitmap in the workgroup's LDS table.
constexpr u32 kLdsBfsMax = (u32)kBigSlots * 32u;

// Sampled links of every vertex with its neighbours number `first` and `first + 1` in
// ascending order (cc_min_link), then a full compression.  All threads call it.
__device__ __forceinline__ void batch_sample_links(const u32* __restrict__ rp,
                                                   const u32* __restrict__ ci, u32 n,
                                                   u32* parent, u32 first) {
  for (u32 v = threadIdx.x; v < n; v += kBT) {
    const u32 lo = rp[v], d = rp[v + 1] - lo;
    if (d > first) {
      const u32 a = ci[lo + first];
      if (first > 0 || a > v) cc_min_link(parent, v, a);
    }
    if (d > first + 1) cc_min_link(parent, v, ci[lo + first + 1]);
  }
  __syncthreads();
  for (u32 v = threadIdx.x; v < n; v += kBT) parent[v] = cc_find(parent, v);
  __syncthreads();
}

// The most frequent root among up to kBatchModeSamples spread-out vertices that have
// neighbours (the dominant set of the sampled union-find); *thin is set when it holds
// fewer than 90 % of them.  All threads call it and get the same result; s_root holds
// kBT words, s_best kBW words, s_live kBW words.
constexpr u32 kBatchModeSamples = 512;

__device__ __forceinline__ u32 batch_dominant_root(const u32* __restrict__ rp, u32 n,
                                                   u32* parent, u32* s_root, u64* s_best,
                                                   u32* s_live, bool* thin) {
  const u32 i = threadIdx.x, lane = lane_id(), wid = threadIdx.x / kWave;
  const u32 ns = min(n, kBatchModeSamples);
  u32 r = kInf;
  bool live = false;
  if (i < ns) {
    const u32 v = n <= kBatchModeSamples ? i : (u32)(((u64)i * 2654435761ull + 12345u) % n);
    live = rp[v + 1] > rp[v];
    r = live ? cc_find(parent, v) : kInf;
    s_root[i] = r;
  }
  __syncthreads();
  u32 cnt = 0;
  if (live)
    for (u32 j = 0; j < ns; ++j) cnt += s_root[j] == r;
  // largest (count, root) pair; ties go to the larger root, any choice is correct
  u64 key = live ? ((u64)cnt << 32) | r : 0ull;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const u64 o = __shfl_xor(key, off, kWave);
    key = o > key ? o : key;
  }
  const u32 nlive = (u32)__popcll(__ballot(live));
  if (lane == 0) {
    s_best[wid] = key;
    s_live[wid] = nlive;
  }
  __syncthreads();
  u64 b = 0;
  u32 tl = 0;
  for (u32 w = 0; w < (u32)kBW; ++w) {
    b = s_best[w] > b ? s_best[w] : b;
    tl += s_live[w];
  }
  __syncthreads();  // s_root, s_best and s_live are free again
  *thin = (u32)(b >> 32) * 10u < tl * 9u;
  return tl ? (u32)b : kInf;
}

struct BatchArrays {
  const u32* rowptr_cat;
  const u32* colidx_cat;
  u32 m_total;        // entries of colidx_cat
  const u32* tail4;   // padded last quad of colidx_cat
  const int64_t* row_off;
  const int64_t* col_off;
  u32* parent_all;
  u32* level_all;
  u32* queue_all;
  uint8_t* vinfo_all;
  u32* hcnt_all;
  uint4* vrec_all;    // per row: {row start, sabove, split, row end}, local to the graph
  u32* colidx2_all;   // m_total + 4 entries (the padding keeps quad loads in bounds)
  u32* hadj_all;
};

// The wavefront's rows with `sel` (lane's own row v at local offset lo, d entries, info
// vx), 64 / GL at a time, one per group of GL lanes (split_group_row); writes their row
// records and partner counts.
template <u32 GL, u32 U>
__device__ __forceinline__ void batch_split_groups(const BatchArrays& A, const uint8_t* vinfo,
                                                   u32 v, u32 lo, u32 d, u32 vx, u32 cb,
                                                   bool sel, uint4* vrec, u32* hcnt) {
  constexpr u32 NG = kWave / GL;
  const u32 lane = lane_id();
  u64 mg = __ballot(sel);
  while (mg) {
    int src = -1;  // the g-th lowest remaining lane for group g
#pragma unroll
    for (u32 gi = 0; gi < NG; ++gi) {
      const int bl = mg ? __ffsll((unsigned long long)mg) - 1 : -1;
      if (bl >= 0) mg &= mg - 1;
      if (gi == lane / GL) src = bl;
    }
    // every lane takes part in the shuffles (a source lane outside them reads as 0)
    const int s0 = src < 0 ? 0 : src;
    const u32 gv = __shfl(v, s0, kWave), glo = __shfl(lo, s0, kWave);
    const u32 gd0 = __shfl(d, s0, kWave), gvx = __shfl(vx, s0, kWave);
    const u32 gd = src < 0 ? 0u : gd0;
    u32 ns, nh, sr;
    split_group_row<GL, U>(A.colidx_cat, vinfo, gv, gvx, cb + glo, gd, A.colidx2_all, A.hadj_all,
                           &ns, &nh, &sr);
    if (src >= 0 && (lane & (GL - 1u)) == 0) {
      vrec[gv] = make_uint4(glo, glo + sr, glo + ns, glo + gd);
      hcnt[gv] = nh;
    }
  }
}

template <bool VEC>
__global__ void __launch_bounds__(kBT) k_batch_main(BatchArrays A, u32 G,
                                                   const u32* __restrict__ order,
                                                   BatchCtl* __restrict__ ctl, IsectParams prm,
                                                   u64* __restrict__ counts) {
  __shared__ __align__(16) u32 s_table[kBigSlots];  // one workgroup table or 16 wave tables
  __shared__ u32 s_qincl[kBigSeg];                    // also the wavefronts' partner ends
  __shared__ uint4 s_pinfo[kBigSeg];                  // also the wavefronts' partner info
  __shared__ u32 s_mark[kBigSeg];                     // wavefront marks / block-class list
  __shared__ u32 s_tmp[kBW];
  __shared__ u64 s_red[3 * kBW];
  __shared__ u32 s_g, s_qtail, s_cnt, s_next;
  const BlockShared sh{s_table, s_qincl, s_pinfo, s_tmp};
  const u32 lane = lane_id(), wid = threadIdx.x / kWave;

  while (true) {
    if (threadIdx.x == 0) {
      const u32 idx = atomicAdd(&ctl->next, 1u);
      s_g = idx < G ? order[idx] : kInf;
      s_qtail = 0;
      s_cnt = 0;
      s_next = 0;
    }
    __syncthreads();
    const u32 g = s_g;
    if (g == kInf) break;
    const int64_t rb = A.row_off[g];
    const u32 n = (u32)(A.row_off[g + 1] - rb - 1);
    const u32 cb = (u32)A.col_off[g];
    const u32 m = (u32)(A.col_off[g + 1] - A.col_off[g]);
    if (n == 0 || m == 0) {
      if (threadIdx.x == 0) counts[g] = 0;
      __syncthreads();
      continue;
    }
    const u32* rp = A.rowptr_cat + rb;
    const u32* ci = A.colidx_cat + cb;  // local view for the traversals
    u32* parent = A.parent_all + rb;
    u32* level = A.level_all + rb;
    u32* queue = A.queue_all + rb;
    uint8_t* vinfo = A.vinfo_all + rb;
    u32* hcnt = A.hcnt_all + rb;
    uint4* vrec = A.vrec_all + rb;

    // ---- 1. component roots: sampled union-find, smallest-ID roots ----
    for (u32 v = threadIdx.x; v < n; v += kBT) {
      const u32 lo = rp[v], hi = rp[v + 1];
      parent[v] = lo < hi ? min(v, ci[lo]) : v;
    }
    __syncthreads();
    for (u32 v = threadIdx.x; v < n; v += kBT) parent[v] = cc_find(parent, v);
    __syncthreads();
    batch_sample_links(rp, ci, n, parent, 0);
    bool thin = false;
    u32 dom = batch_dominant_root(rp, n, parent, s_mark, s_red, s_tmp, &thin);
    if (thin) {  // many sampled links lost to races: a second round before the full pass
      batch_sample_links(rp, ci, n, parent, 2);
      dom = batch_dominant_root(rp, n, parent, s_mark, s_red, s_tmp, &thin);
    }
    // every vertex outside the dominant set joins all its neighbours
    {
      const u32 nr = (n + kWave - 1) / kWave * kWave;
      for (u32 v = threadIdx.x; v < nr; v += kBT) {
        const bool out = v < n && load_coherent(&parent[v]) != dom && rp[v + 1] > rp[v];
        const u32 pos = wave_append(&s_cnt, out);
        if (out) queue[pos] = v;
      }
    }
    __syncthreads();
    block_for_each_entry(rp, ci, s_cnt, queue, [&](u32 u, u32 v, bool act) {
      if (act) cc_union(parent, u, v);
    });
    __syncthreads();
    for (u32 v = threadIdx.x; v < n; v += kBT) parent[v] = cc_find(parent, v);
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();

    // ---- 2. level BFS from every root ----
    // Graphs of up to kLdsBfsMax vertices keep a visited bitmap in LDS (the intersection
    // table is free until step 5): a neighbour is claimed by one LDS atomicOr instead of
    // a global compare-and-swap on its level.
    const bool lds_bfs = n <= kLdsBfsMax;
    u32* s_vis = s_table;
    if (lds_bfs)
      for (u32 i = threadIdx.x; i < (n + 31) / 32; i += kBT) s_vis[i] = 0;
    __syncthreads();
    {
      const u32 nr = (n + kWave - 1) / kWave * kWave;
      for (u32 v = threadIdx.x; v < nr; v += kBT) {
        bool push = false;
        if (v < n) {
          const bool root = parent[v] == v;
          level[v] = root ? 0u : kInf;
          push = root && rp[v + 1] > rp[v];
          if (root && lds_bfs) atomicOr(&s_vis[v >> 5], 1u << (v & 31u));
        }
        const u32 pos = wave_append(&s_qtail, push);
        if (push) queue[pos] = v;
      }
    }
    __syncthreads();
    // Direction-optimising levels (Beamer et al., SC 2012) when the frontier bitmap fits
    // beside the visited one: a level whose frontier holds more than 1/14 of the entries
    // still unexplored runs bottom-up (every unvisited vertex looks for a frontier
    // neighbour and stops at the first), and the search returns to top-down once the
    // frontier holds fewer than n / 24 vertices.
    const u32 nw = (n + 31) / 32;
    const bool bu_ok = lds_bfs && 2 * nw <= (u32)kBigSlots;
    u32* s_fr = s_table + nw;
    u32 mu = m;  // entries of the vertices that have not been in a frontier yet
    bool bu = false;
    u32 qs = 0, k = 0;
    while (true) {
      const u32 qe = s_qtail;
      if (qs == qe) break;
      if (threadIdx.x == 0) s_cnt = 0;
      __syncthreads();
      const u32 next = k + 1;
      if (bu_ok) {  // the frontier's entries
        u32 mf = 0;
        for (u32 i = threadIdx.x; i < qe - qs; i += kBT) {
          const u32 u = queue[qs + i];
          mf += rp[u + 1] - rp[u];
        }
        mf = wave_sum_u32(mf);
        if (lane == 0 && mf) atomicAdd(&s_cnt, mf);
        __syncthreads();
        const u32 mfs = s_cnt;
        mu -= min(mu, mfs);
        bu = bu ? qe - qs >= n / 24 : mfs > mu / 14;
      }
      if (bu) {
        for (u32 i = threadIdx.x; i < nw; i += kBT) s_fr[i] = 0;
        __syncthreads();
        for (u32 i = threadIdx.x; i < qe - qs; i += kBT) {
          const u32 u = queue[qs + i];
          atomicOr(&s_fr[u >> 5], 1u << (u & 31u));
        }
        __syncthreads();
        const u32 nr = (n + kWave - 1) / kWave * kWave;
        for (u32 v = threadIdx.x; v < nr; v += kBT) {
          bool claimed = false;
          if (v < n && ((s_vis[v >> 5] >> (v & 31u)) & 1u) == 0) {
            const u32 lo = rp[v], hi = rp[v + 1];
            for (u32 j = lo; j < hi && !claimed; j += 4) {
              u32 w[4];
#pragma unroll
              for (u32 t = 0; t < 4; ++t) w[t] = j + t < hi ? ci[j + t] : 0u;
#pragma unroll
              for (u32 t = 0; t < 4; ++t)
                claimed |= j + t < hi && ((s_fr[w[t] >> 5] >> (w[t] & 31u)) & 1u) != 0;
            }
          }
          if (claimed) {
            level[v] = next;
            atomicOr(&s_vis[v >> 5], 1u << (v & 31u));
          }
          const u32 pos = wave_append(&s_qtail, claimed);
          if (claimed) queue[pos] = v;
        }
      } else if (lds_bfs) {
        block_for_each_entry(rp, ci, qe - qs, queue + qs, [&](u32 u, u32 v, bool act) {
          (void)u;
          bool claimed = false;
          if (act) {
            const u32 bit = 1u << (v & 31u);
            claimed = (s_vis[v >> 5] & bit) == 0 && (atomicOr(&s_vis[v >> 5], bit) & bit) == 0;
          }
          if (claimed) level[v] = next;
          const u32 pos = wave_append(&s_qtail, claimed);
          if (claimed) queue[pos] = v;
        });
      } else {
        block_for_each_entry(rp, ci, qe - qs, queue + qs, [&](u32 u, u32 v, bool act) {
          (void)u;
          bool claimed = false;
          if (act && load_coherent(&level[v]) == kInf)
            claimed = atomicCAS(&level[v], kInf, next) == kInf;
          const u32 pos = wave_append(&s_qtail, claimed);
          if (claimed) queue[pos] = v;
        });
      }
      __syncthreads();
      qs = qe;
      ++k;
    }
    if (threadIdx.x == 0) s_cnt = 0;  // the split's long-row count starts from zero
    __syncthreads();

    // ---- 3. per-vertex info ----
    for (u32 v = threadIdx.x; v < n; v += kBT)
      vinfo[v] = (uint8_t)(((level[v] & 1u) << 7) | degree_class(rp[v + 1] - rp[v]));
    __syncthreads();

    // ---- 4. level split and partner lists (vrec[] local, arrays at cb) ----
    // vrec[v] = {row start, sabove, split, row end}: sabove is the first entry of v's
    // same-level part above v, split the first of its other-level part
    {
      const u32 nr = (n + kWave - 1) / kWave * kWave;
      for (u32 v = threadIdx.x; v < nr; v += kBT) {
        u32 lo = 0, d = 0, vx = 0;
        if (v < n) {
          lo = rp[v];
          d = rp[v + 1] - lo;
          vx = vinfo[v];
        }
        const bool short_row = v < n && d <= kSplitLane;
        bool more[kSplitLane / 8];
#pragma unroll
        for (u32 b = 0; b < kSplitLane / 8; ++b) more[b] = __ballot(short_row && d > b * 8) != 0;
        if (short_row) {
          u32 ns, nh, sr;
          split_short_row(A.colidx_cat, vinfo, v, vx, cb + lo, d, more, A.colidx2_all,
                          A.hadj_all, &ns, &nh, &sr);
          vrec[v] = make_uint4(lo, lo + sr, lo + ns, lo + d);
          hcnt[v] = nh;
        }
        const bool lng = d > kSplitWave;
        const u32 pos = wave_append(&s_cnt, lng);
        if (lng) queue[pos] = v;  // the BFS queue is free again
        // rows of kSplitLane < d <= kSplitGroup: four at a time, one per 16-lane group
        // (rows of up to 256 entries two at a time in 32-lane halves measured slower)
        batch_split_groups<16, kSplitGroup / 16>(A, vinfo, v, lo, d, vx, cb,
                                                 d > kSplitLane && d <= kSplitGroup, vrec,
                                                 hcnt);
        u64 mm = __ballot(d > kSplitGroup && d <= kSplitWave);
        while (mm) {
          const int b = __ffsll((unsigned long long)mm) - 1;
          mm &= mm - 1;
          const u32 bv = __shfl(v, b, kWave), blo = __shfl(lo, b, kWave);
          const u32 bd = __shfl(d, b, kWave), bvx = __shfl(vx, b, kWave);
          u32 ns = 0, nh = 0, sr = 0;
          if (bd <= kSplitReg) {
            split_wave_row(A.colidx_cat, vinfo, bv, bvx, cb + blo, bd, A.colidx2_all, A.hadj_all,
                           &ns, &nh, &sr);
          } else {
            u32 no = 0;
            for (u32 j0 = 0; j0 < bd; j0 += kWave * kSplitUnroll)
              split_steps<true>(A.colidx_cat, vinfo, bv, bvx, cb + blo, j0, bd, 0, 0, 0,
                                A.colidx2_all, A.hadj_all, ns, no, nh, sr);
            u32 cs = 0, co = 0, ch = 0, cl = 0;
            for (u32 j0 = 0; j0 < bd; j0 += kWave * kSplitUnroll)
              split_steps<false>(A.colidx_cat, vinfo, bv, bvx, cb + blo, j0, bd, 0, ns, 0,
                                 A.colidx2_all, A.hadj_all, cs, co, ch, cl);
          }
          if ((int)lane == b) {
            vrec[bv] = make_uint4(blo, blo + sr, blo + ns, blo + bd);
            hcnt[bv] = nh;
          }
        }
      }
      __syncthreads();
      // long rows: each wavefront takes a contiguous segment of the row
      const u32 nl = s_cnt;
      for (u32 li = 0; li < nl; ++li) {
        const u32 v = queue[li];
        const u32 lo = rp[v], d = rp[v + 1] - lo, vx = vinfo[v];
        const u32 step = kWave * kSplitUnroll;
        const u32 segw = (d + kBW * step - 1) / (kBW * step) * step;
        const u32 j0 = min(wid * segw, d), j1 = min(j0 + segw, d);
        u32 ns = 0, no = 0, nh = 0, sr = 0;
        for (u32 j = j0; j < j1; j += step)
          split_steps<true>(A.colidx_cat, vinfo, v, vx, cb + lo, j, j1, 0, 0, 0, A.colidx2_all,
                            A.hadj_all, ns, no, nh, sr);
        if (lane == 0) {
          s_mark[wid] = ns;
          s_mark[kBW + wid] = nh;
          s_mark[2 * kBW + wid] = sr;
        }
        __syncthreads();
        u32 bs = 0, bh = 0, ts = 0, th = 0, tsr = 0;
        for (u32 w = 0; w < (u32)kBW; ++w) {
          if (w < wid) {
            bs += s_mark[w];
            bh += s_mark[kBW + w];
          }
          ts += s_mark[w];
          th += s_mark[kBW + w];
          tsr += s_mark[2 * kBW + w];
        }
        u32 cs = 0, co = 0, ch = 0, cl = 0;
        for (u32 j = j0; j < j1; j += step)
          split_steps<false>(A.colidx_cat, vinfo, v, vx, cb + lo, j, j1, bs, ts + (j0 - bs), bh,
                             A.colidx2_all, A.hadj_all, cs, co, ch, cl);
        if (threadIdx.x == 0) {
          vrec[v] = make_uint4(lo, lo + tsr, lo + ts, lo + d);
          hcnt[v] = th;
        }
        __syncthreads();
      }
    }
    __syncthreads();

    // ---- 5a. lane class ----
    Counts c{0, 0, 0, 0, 0};
    for (u32 v = threadIdx.x; v < n; v += kBT)
      if (hcnt[v] > 0 && rp[v + 1] - rp[v] <= prm.lane_max)
        lane_vertex<false>(rp, cb, A.colidx_cat, vinfo, hcnt, A.hadj_all, v, c, nullptr);

    // ---- 5b. wavefront class, pruned: 16 wavefront tables in the workgroup table ----
    // A wavefront claims 64 vertices at once and reads their row bounds, partner counts
    // and sabove points in one load per lane.  Vertices of up to kSubMax entries are then
    // taken four at a time, one per group of 16 lanes (subwave_vertex, each group with a
    // quarter of the wavefront's table); longer ones one at a time with the whole
    // wavefront (wave_vertex).  Each x stages its level-split row from sabove[x] on (its
    // other-level neighbours and same-level ones above x) as plain keys; each partner y
    // streams its split row from sabove[y] on, and every hit is a counted apex.
    {
      const u32 sub_max = min(kSubMax, prm.wave_max);
      while (true) {
        u32 c0 = 0;
        if (lane == 0) c0 = atomicAdd(&s_next, (u32)kWave);
        const u32 base = __shfl(c0, 0, kWave);
        if (base >= n) break;  // wave-uniform
        const u32 x = base + lane;
        WaveMeta mt{0, 0, 0, 0};
        bool sub = false, whole = false;
        if (x < n) {
          const uint4 r = vrec[x];
          const u32 np = hcnt[x];
          const u32 d = r.w - r.x;
          const bool cls = np > 0 && d > prm.lane_max && d <= prm.wave_max;
          sub = cls && d <= sub_max;
          whole = cls && !sub;
          if (cls) mt = WaveMeta{cb + r.x, cb + r.w, cb + r.y, np};
        }
        u64 todo = __ballot(sub);
        u32* gtab = s_table + wid * kWaveSlots + (lane / kSubLanes) * kSubSlots;
        while (todo) {
          // up to four vertices, the g-th lowest remaining lane for group g
          int src = -1;
#pragma unroll
          for (u32 g = 0; g < kSubGroups; ++g) {
            const int b = todo ? __ffsll((unsigned long long)todo) - 1 : -1;
            if (b >= 0) todo &= todo - 1;
            if (g == lane / kSubLanes) src = b;
          }
          const int s0 = src < 0 ? 0 : src;
          WaveMeta gm{(u32)__shfl(mt.bx, s0, kWave), (u32)__shfl(mt.ex, s0, kWave),
                      (u32)__shfl(mt.sb, s0, kWave), (u32)__shfl(mt.np, s0, kWave)};
          if (src < 0) gm = WaveMeta{0, 0, 0, 0};
          Tally tl{0, 0, 0, 0};
          subwave_vertex<kPartAbove>(A.colidx2_all, A.m_total, cb, A.hadj_all, nullptr, vrec,
                                     gm, gtab, tl, c);
          tl.fold(c);
        }
        todo = __ballot(whole);
        while (todo) {
          const int b = __ffsll((unsigned long long)todo) - 1;
          todo &= todo - 1;
          const WaveMeta mb{(u32)__shfl(mt.bx, b, kWave), (u32)__shfl(mt.ex, b, kWave),
                            (u32)__shfl(mt.sb, b, kWave), (u32)__shfl(mt.np, b, kWave)};
          Tally tl{0, 0, 0, 0};
          wave_vertex<false, true, false, 1, false, false, true>(
              rp, cb, A.colidx2_all, A.m_total, A.tail4, vinfo, hcnt, A.hadj_all, nullptr,
              vrec, (u32)__shfl(x, b, kWave), mb, s_table + wid * kWaveSlots,
              s_pinfo + wid * kWave, s_qincl + wid * kWave, s_mark + wid * kWave, tl, c, nullptr);
          tl.fold(c);
        }
      }
    }
    __syncthreads();

    // ---- 5c. workgroup class, pruned, over batches of up to 1024 staged vertices ----
    // x's row from sabove[x] on staged as plain keys, each partner y's row streamed from
    // sabove[y] on (block_item_rec with kPartAbove)
    {
      Tally tl{0, 0, 0, 0};
      for (u32 base = 0; base < n; base += kBT) {
        const u32 v = base + threadIdx.x;
        const bool isx = v < n && hcnt[v] > 0 && rp[v + 1] - rp[v] > prm.wave_max;
        u32 tot;
        const u32 incl = block_incl_scan(isx ? 1u : 0u, s_tmp, &tot);
        if (isx) s_mark[incl - 1] = v;
        __syncthreads();
        for (u32 i = 0; i < tot; ++i) {
          const u32 x = s_mark[i];
          const u32 nseg = (hcnt[x] + prm.seg - 1) / prm.seg;
          for (u32 sg = 0; sg < nseg; ++sg)
            // colidx2 carries 4 padding entries, so its quad loads never need a tail copy
            // (two windows per wavefront keep the whole kernel within its registers)
            block_item_rec<VEC, true, false, kPartAbove, 4>(
                rp, cb, A.colidx2_all, A.m_total, A.tail4, nullptr, nullptr, hcnt, nullptr,
                A.hadj_all, vrec, x, sg, prm, sh, tl, c);
        }
        __syncthreads();  // s_mark is rewritten by the next batch
      }
      tl.fold(c);
    }

    // ---- 6. per-graph total ----
    const u64 c1 = wave_sum_u64(c.c1), t2 = wave_sum_u64(c.t2);
    if (lane == 0) {
      s_red[2 * wid] = c1;
      s_red[2 * wid + 1] = t2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      u64 a = 0, b = 0;
      for (int w = 0; w < kBW; ++w) {
        a += s_red[2 * w];
        b += s_red[2 * w + 1];
      }
      counts[g] = a + b;
    }
    __syncthreads();
  }
}

// ---- workspace ------------------------------------------------------------------------
struct BatchLayout {
  size_t ctl, order, parent, level, queue, vinfo, hcnt, vrec, colidx2, hadj, tail, bytes;
};

static size_t up256(size_t v) { return (v + 255) / 256 * 256; }

static BatchLayout batch_layout(u32 G, u64 rows, u64 cols) {
  BatchLayout L;
  size_t o = 0;
  L.ctl = o; o += up256(batch_ctl_bytes());
  L.order = o; o += up256((size_t)G * 4);
  L.parent = o; o += up256(rows * 4);
  L.level = o; o += up256(rows * 4);
  L.queue = o; o += up256(rows * 4);
  L.vinfo = o; o += up256(rows);
  L.hcnt = o; o += up256(rows * 4);
  L.vrec = o; o += up256(rows * 16);
  L.colidx2 = o; o += up256((cols + 4) * 4);
  L.hadj = o; o += up256(cols * 4);
  L.tail = o; o += 256;
  L.bytes = o + 256;  // alignment slack of the caller's pointer
  return L;
}

size_t batch_workspace_bytes(u32 G, u64 total_rows, u64 total_cols) {
  return batch_layout(G, total_rows, total_cols).bytes;
}

void launch_batch(const u32* rowptr_cat, const u32* colidx_cat, const int64_t* row_off,
                  const int64_t* col_off, u32 G, u64 total_rows, u64 total_cols, void* ws,
                  IsectParams p, u64* counts, hipStream_t s) {
  const BatchLayout L = batch_layout(G, total_rows, total_cols);
  char* base = (char*)(((uintptr_t)ws + 255) / 256 * 256);
  BatchCtl* ctl = (BatchCtl*)(base + L.ctl);
  u32* order = (u32*)(base + L.order);
  u32* tail4 = (u32*)(base + L.tail);
  BatchArrays A;
  A.rowptr_cat = rowptr_cat;
  A.colidx_cat = colidx_cat;
  A.m_total = (u32)total_cols;
  A.tail4 = tail4;
  A.row_off = row_off;
  A.col_off = col_off;
  A.parent_all = (u32*)(base + L.parent);
  A.level_all = (u32*)(base + L.level);
  A.queue_all = (u32*)(base + L.queue);
  A.vinfo_all = (uint8_t*)(base + L.vinfo);
  A.hcnt_all = (u32*)(base + L.hcnt);
  A.vrec_all = (uint4*)(base + L.vrec);
  A.colidx2_all = (u32*)(base + L.colidx2);
  A.hadj_all = (u32*)(base + L.hadj);
  hipLaunchKernelGGL(k_batch_prepare, dim3(1), dim3(256), 0, s, col_off, G, ctl, order);
  if (total_cols > 0) launch_tail4(colidx_cat, (u32)total_cols, tail4, s);
  const u32 grid = (u32)min((int)G, num_cus());
  if ((((uintptr_t)colidx_cat) & 15u) == 0)
    hipLaunchKernelGGL(k_batch_main<true>, dim3(grid), dim3(kBT), 0, s, A, G, order, ctl, p,
                       counts);
  else
    hipLaunchKernelGGL(k_batch_main<false>, dim3(grid), dim3(kBT), 0, s, A, G, order, ctl, p,
                       counts);
}

}  // namespace tc

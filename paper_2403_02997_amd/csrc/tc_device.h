// Device-side building blocks shared by the gfx950 kernels of the cover-edge
// triangle-counting path: 64-lane wavefront primitives, the CSR tile-to-row lookup,
// the per-vertex info byte, the LDS open-addressing hash set, and counter slots.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

typedef uint32_t u32;
typedef uint64_t u64;

constexpr int kWave = 64;          // CDNA wavefront width
constexpr u32 kInf = 0xFFFFFFFFu;  // unvisited level / empty hash slot
constexpr int kCounterSlots = 256; // spread of the u64 result counters (contention)

// ---- CSR tiles ------------------------------------------------------------------
// Edge-parallel kernels split the m stored entries into tiles of kTile entries.
// tile_row[t] is the row holding entry t * kTile (tile_row[ntiles] = row of entry m-1),
// so the rows overlapping tile t are tile_row[t] .. tile_row[t+1].
constexpr int kTile = 1024;
constexpr int kTileThreads = 256;
constexpr int kTileRowCap = 2048;  // rows of one tile staged in LDS

// ---- wavefront primitives ----------------------------------------------------------
__device__ __forceinline__ u32 lane_id() { return __lane_id(); }

// Number of set bits of `mask` in lanes below this one (mbcnt).
__device__ __forceinline__ u32 mask_rank(u64 mask) {
  return __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, 0u));
}

__device__ __forceinline__ u64 wave_sum_u64(u64 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ u32 wave_sum_u32(u32 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Inclusive prefix sum across the 64 lanes of a wavefront.
__device__ __forceinline__ u32 wave_incl_scan(u32 v) {
  const u32 lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    u32 t = __shfl_up(v, off, kWave);
    if (lane >= (u32)off) v += t;
  }
  return v;
}

// Wave-aggregated append: every lane with `pred` gets a distinct slot of `*counter`.
// Must be reached by all active lanes of the wavefront together.
__device__ __forceinline__ u32 wave_append(u32* counter, bool pred) {
  const u64 mask = __ballot(pred);
  u32 base = 0;
  if (mask) {
    const int leader = __ffsll((unsigned long long)mask) - 1;
    if ((int)lane_id() == leader) base = atomicAdd(counter, (u32)__popcll(mask));
    base = __shfl(base, leader, kWave);
  }
  return base + mask_rank(mask);
}

// Relaxed agent-scope load: bypasses the non-coherent per-CU cache so that values
// written by other workgroups during the same launch are observed.
__device__ __forceinline__ u32 load_coherent(const u32* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- block-level inclusive scan (blockDim.x = kTileThreads) --------------------------
// `s_tmp` holds at least kTileThreads / kWave entries.  Returns the inclusive prefix of
// v over thread order; *total receives the block sum.
__device__ __forceinline__ u32 block_incl_scan(u32 v, u32* s_tmp, u32* total) {
  const u32 lane = lane_id(), wid = threadIdx.x / kWave;
  const u32 nw = blockDim.x / kWave;
  u32 x = wave_incl_scan(v);
  if (lane == kWave - 1) s_tmp[wid] = x;
  __syncthreads();
  u32 add = 0, tot = 0;
  for (u32 w = 0; w < nw; ++w) {
    const u32 s = s_tmp[w];
    if (w < wid) add += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return x + add;
}

// ---- per-vertex info byte ----------------------------------------------------------
// bit 7: parity of the BFS level (L mod 2); bits 0..6: degree class, a monotone
// quantised log2 of the degree (4 steps per octave).  Two adjacent vertices are on the
// same level iff their parities agree, because a BFS edge joins levels that differ by
// at most one.  Cover edges are oriented towards the endpoint with the larger
// (degree class, vertex ID) key, whose neighbour list is the one staged in LDS.
__device__ __forceinline__ u32 degree_class(u32 d) {
  if (d == 0) return 0;
  const u32 lg = 31u - (u32)__clz(d);
  const u32 frac = lg >= 2 ? (d >> (lg - 2)) & 3u : ((d << (2 - lg)) & 3u);
  const u32 c = 1u + 4u * lg + frac;
  return c > 127u ? 127u : c;
}

__device__ __forceinline__ bool key_less(u32 cls_a, u32 a, u32 cls_b, u32 b) {
  return cls_a < cls_b || (cls_a == cls_b && a < b);
}

// ---- tile lookup -------------------------------------------------------------------
// Stage rowptr[r0 .. r1+1] of tile t in LDS.  Returns false (and stages nothing) when
// the tile spans more than kTileRowCap rows (long runs of empty rows); callers then
// fall back to a binary search in global memory.
struct TileInfo {
  u32 e0, e1;   // entries [e0, e1)
  u32 r0, r1;   // rows r0 .. r1 overlap the tile
  bool staged;
};

__device__ __forceinline__ TileInfo tile_begin(const u32* __restrict__ rowptr,
                                               const u32* __restrict__ tile_row, u32 t,
                                               u32 m, u32* s_rp) {
  TileInfo ti;
  ti.e0 = t * (u32)kTile;
  ti.e1 = min(ti.e0 + (u32)kTile, m);
  ti.r0 = tile_row[t];
  ti.r1 = tile_row[t + 1];
  const u32 nr = ti.r1 - ti.r0 + 2;  // rowptr entries r0 .. r1 + 1
  ti.staged = nr <= (u32)kTileRowCap;
  if (ti.staged)
    for (u32 i = threadIdx.x; i < nr; i += blockDim.x) s_rp[i] = rowptr[ti.r0 + i];
  __syncthreads();
  return ti;
}

// Row of entry e (ti.e0 <= e < ti.e1): the largest r in [r0, r1] with rowptr[r] <= e.
__device__ __forceinline__ u32 tile_row_of(const TileInfo& ti, const u32* s_rp,
                                           const u32* __restrict__ rowptr, u32 e) {
  u32 lo = 0, hi = ti.r1 - ti.r0;  // answer index in [lo, hi]
  if (ti.staged) {
    while (lo < hi) {
      const u32 mid = (lo + hi + 1) >> 1;
      if (s_rp[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
  } else {
    while (lo < hi) {
      const u32 mid = (lo + hi + 1) >> 1;
      if (rowptr[ti.r0 + mid] <= e) lo = mid;
      else hi = mid - 1;
    }
  }
  return ti.r0 + lo;
}

// Orders LDS accesses of one wavefront (writes by some lanes, reads by others).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- LDS hash set of a neighbour list -----------------------------------------------
// Bucketed open addressing: a table of `slots` u32 (a power of two) is read as buckets of
// four slots, one 16-byte LDS load per bucket.  A vertex w of the staged list is stored
// as the key (w << 1) | same, with `same` set when w is on the owner's BFS level
// (w < 2^30 - 1, so keys stay below 2^31 and never equal the empty marker).  Inserts fill
// a bucket's slots in order; an insert that finds its bucket full sets the overflow flag
// (bit 31) of the bucket's last slot and moves on to the next bucket.  A probe therefore
// ends at the first bucket that holds w or carries no flag, and the rare flagged bucket
// is the only case in which a wavefront has to wait for some of its lanes.
constexpr u32 kFlag = 0x80000000u;

// Bucket mask for `keys` keys at load factor <= 1/8 where cap_slots allows: at least 16
// buckets (64 slots), at most cap_slots / 4.  The chunk sizes keep the load factor of
// the workgroup table at 1/8 and of the wavefront tables at 1/4 or less.
__device__ __forceinline__ u32 bucket_mask(u32 keys, u32 cap_slots) {
  u32 want = keys * 8;
  if (want < 64) want = 64;
  u32 p = 1u << (32 - __clz(want - 1));
  if (p > cap_slots) p = cap_slots;
  return p / 4 - 1;
}

// Shift-xor mix (one shift and one fused xor-and per key); the low bits index the
// buckets, and bits 13 and up are folded onto them.
__device__ __forceinline__ u32 hash_mix(u32 w) { return w ^ (w >> 13); }

// Inserts key (derived from w: (w << 1) | level flag, or w itself in membership sets)
// into the bucket chain of w.
__device__ __forceinline__ void hash_insert_key(u32* table, u32 bmask, u32 w, u32 key) {
  u32 b = hash_mix(w) & bmask;
  while (true) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (atomicCAS(&table[4 * b + j], kInf, key) == kInf) return;
    atomicOr(&table[4 * b + 3], kFlag);  // the bucket is full: probes must go on
    b = (b + 1) & bmask;
  }
}

__device__ __forceinline__ void hash_insert(u32* table, u32 bmask, u32 w, u32 same) {
  hash_insert_key(table, bmask, w, (w << 1) | same);
}

// Bucket v against k2 = w << 1: 1 when w is present on another level, 2 on the owner's
// level, 3 when absent here but the bucket is flagged (the probe continues in the next
// bucket), 0 when absent.  A slot matches iff key ^ k2 is 0 or 1, and that value is the
// level flag; only the last slot can carry the overflow flag, and an empty slot (all
// ones) never matches.
__device__ __forceinline__ u32 bucket_check(uint4 v, u32 k2) {
  const u32 mn = min(min(v.x ^ k2, v.y ^ k2), min(v.z ^ k2, (v.w & ~kFlag) ^ k2));
  const bool flagged = v.w - kFlag < kInf - kFlag;  // kFlag <= v.w < kInf
  return mn <= 1u ? 1u + mn : (flagged ? 3u : 0u);
}

// Membership form of bucket_check for sets built without level flags (every key is
// w << 1): 1 when present, 3 when absent but flagged, 0 when absent.  An empty slot
// (all ones, or all ones but the flag bit in the last slot) is odd and never matches.
__device__ __forceinline__ u32 bucket_has(uint4 v, u32 k2) {
  const bool hit = v.x == k2 || v.y == k2 || v.z == k2 || (v.w & ~kFlag) == k2;
  const bool flagged = v.w - kFlag < kInf - kFlag;  // kFlag <= v.w < kInf
  return hit ? 1u : (flagged ? 3u : 0u);
}

template <bool MEMBER>
__device__ __forceinline__ u32 bucket_result(uint4 v, u32 k2) {
  return MEMBER ? bucket_has(v, k2) : bucket_check(v, k2);
}

__device__ __forceinline__ u32 hash_probe(const u32* table, u32 bmask, u32 w) {
  const uint4* t4 = reinterpret_cast<const uint4*>(table);
  const u32 k2 = w << 1;
  u32 b = hash_mix(w) & bmask;
  while (true) {
    const u32 r = bucket_check(t4[b], k2);
    if (r != 3u) return r;
    b = (b + 1) & bmask;
  }
}

// Probes of N independent keys; res[i] = 0 where !ok[i].  The first bucket of every key
// is read (always in bounds) before any is examined.  Keys whose bucket was full continue
// in one wave-uniform loop that resolves one pending key per lane and pass, so the rare
// overflow costs one bucket check per pass rather than one per key position.  MEMBER
// selects the membership check (sets without level flags; results 0 or 1).
template <int N, bool MEMBER = false>
__device__ __forceinline__ void hash_probe_n(const u32* table, u32 bmask, const u32 (&w)[N],
                                             const bool (&ok)[N], u32 (&res)[N]) {
  const uint4* t4 = reinterpret_cast<const uint4*>(table);
  uint4 v[N];
  u32 b[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    b[i] = hash_mix(w[i]) & bmask;
    v[i] = t4[b[i]];
  }
  // branch-free first checks; the overflow path below is entered only when some lane
  // of the wavefront met a full bucket
  bool any = false;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    res[i] = bucket_result<MEMBER>(v[i], w[i] << 1) & (0u - (u32)ok[i]);
    any |= res[i] == 3u;
  }
  if (!__ballot(any)) return;
  u32 pend = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) pend |= (res[i] == 3u ? 1u : 0u) << i;
  while (__ballot(pend != 0)) {
    if (pend) {
      const u32 i = __ffs(pend) - 1;
      u32 wi = w[0], bi = b[0];
#pragma unroll
      for (int j = 1; j < N; ++j) {
        wi = (u32)j == i ? w[j] : wi;
        bi = (u32)j == i ? b[j] : bi;
      }
      bi = (bi + 1) & bmask;
      const u32 r = bucket_result<MEMBER>(t4[bi], wi << 1);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if ((u32)j == i) {
          b[j] = bi;
          res[j] = r;
        }
      }
      if (r != 3u) pend &= pend - 1;
    }
  }
}

// Membership probes of N independent keys against a set of plain IDs (built with
// hash_insert_key(.., w, w)); adds to hits the number of this lane's keys with ok[i]
// that are present.  Keys whose first bucket was full and flagged continue bucket by
// bucket in a rare wavefront-uniform loop.  An empty slot (all ones, or all ones but
// the flag bit) never equals an ID below 2^30.
__device__ __forceinline__ bool bucket_holds(uint4 v, u32 w) {
  return v.x == w || v.y == w || v.z == w || (v.w & ~kFlag) == w;
}
__device__ __forceinline__ bool bucket_flagged(uint4 v) { return v.w - kFlag < kInf - kFlag; }

// SPLIT: present keys with sm[i] set go to hits_same instead of hits (the split
// statistics of the pruned count tell same-level apexes from other-level ones by the
// streamed element's position).
template <int N, bool SPLIT>
__device__ __forceinline__ void hash_count_split_n(const u32* table, u32 bmask,
                                                   const u32 (&w)[N], const bool (&ok)[N],
                                                   const bool (&sm)[N], u32& hits,
                                                   u32& hits_same) {
  const uint4* t4 = reinterpret_cast<const uint4*>(table);
  uint4 v[N];
  u32 b[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    b[i] = hash_mix(w[i]) & bmask;
    v[i] = t4[b[i]];
  }
  bool more = false;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const bool hold = bucket_holds(v[i], w[i]);
    if (SPLIT) {
      hits += ok[i] && hold && !sm[i] ? 1u : 0u;
      hits_same += ok[i] && hold && sm[i] ? 1u : 0u;
    } else {
      hits += ok[i] && hold ? 1u : 0u;
    }
    more |= ok[i] && !hold && bucket_flagged(v[i]);
  }
  if (!__ballot(more)) return;
  u32 pend = 0;
#pragma unroll
  for (int i = 0; i < N; ++i)
    pend |= (ok[i] && !bucket_holds(v[i], w[i]) && bucket_flagged(v[i]) ? 1u : 0u) << i;
  while (__ballot(pend != 0)) {
    if (pend) {
      const u32 i = __ffs(pend) - 1;
      u32 wi = w[0], bi = b[0];
      bool si = sm[0];
#pragma unroll
      for (int j = 1; j < N; ++j) {
        wi = (u32)j == i ? w[j] : wi;
        bi = (u32)j == i ? b[j] : bi;
        si = (u32)j == i ? sm[j] : si;
      }
      bi = (bi + 1) & bmask;
      const uint4 vv = t4[bi];
      const bool hit = bucket_holds(vv, wi);
#pragma unroll
      for (int j = 0; j < N; ++j)
        if ((u32)j == i) b[j] = bi;
      if (SPLIT && si) hits_same += hit ? 1u : 0u;
      else hits += hit ? 1u : 0u;
      if (hit || !bucket_flagged(vv)) pend &= pend - 1;
    }
  }
}

// Slot (4 b + j) of the plain key w in bucket b, or kInf.
__device__ __forceinline__ u32 bucket_slot(uint4 v, u32 w, u32 b) {
  return v.x == w ? 4 * b
                  : v.y == w ? 4 * b + 1
                             : v.z == w ? 4 * b + 2 : (v.w & ~kFlag) == w ? 4 * b + 3 : kInf;
}

// Membership probes of N keys in a set built by hash_insert_key with key = w, giving the
// slot that holds each (kInf where absent or !ok[i]): per-vertex attribution counts the
// hits of each staged key.  First buckets are read for all keys before any is examined;
// keys whose bucket was full continue in one wave-uniform loop, as in hash_count_split_n.
template <int N>
__device__ __forceinline__ void hash_slots_n(const u32* table, u32 bmask, const u32 (&w)[N],
                                             const bool (&ok)[N], u32 (&slot)[N]) {
  const uint4* t4 = reinterpret_cast<const uint4*>(table);
  uint4 v[N];
  u32 b[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    b[i] = hash_mix(w[i]) & bmask;
    v[i] = t4[b[i]];
  }
  u32 pend = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    slot[i] = ok[i] ? bucket_slot(v[i], w[i], b[i]) : kInf;
    pend |= (ok[i] && slot[i] == kInf && bucket_flagged(v[i]) ? 1u : 0u) << i;
  }
  while (__ballot(pend != 0)) {
    if (pend) {
      const u32 i = __ffs(pend) - 1;
      u32 wi = w[0], bi = b[0];
#pragma unroll
      for (int j = 1; j < N; ++j) {
        wi = (u32)j == i ? w[j] : wi;
        bi = (u32)j == i ? b[j] : bi;
      }
      bi = (bi + 1) & bmask;
      const uint4 vv = t4[bi];
      const u32 sl = bucket_slot(vv, wi, bi);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if ((u32)j == i) {
          b[j] = bi;
          slot[j] = sl;
        }
      }
      if (sl != kInf || !bucket_flagged(vv)) pend &= pend - 1;
    }
  }
}

template <int N>
__device__ __forceinline__ void hash_count_n(const u32* table, u32 bmask, const u32 (&w)[N],
                                             const bool (&ok)[N], u32& hits) {
  bool sm[N];
#pragma unroll
  for (int i = 0; i < N; ++i) sm[i] = false;
  u32 unused = 0;
  hash_count_split_n<N, false>(table, bmask, w, ok, sm, hits, unused);
}

struct Counts;

// Per-thread tallies of one work item in 32-bit registers, folded into Counts after it.
// For a probe result r in {0, 1, 2}: s accumulates r (= c1 + 2 c2), c2 the same-level
// hits r >> 1, t2 the same-level hits above both endpoints.
struct Tally {
  u32 s, c2, t2, probes;
  __device__ __forceinline__ void add(u32 r, u32 w, u32 vmax) {
    const u32 q = r >> 1;
    s += r;
    c2 += q;
    t2 += w > vmax ? q : 0u;
  }
  __device__ __forceinline__ void fold(Counts& c);
};

// ---- union-find with smallest-ID roots ---------------------------------------------
// parent[x] <= x always holds: links go from the larger root to the smaller one, so the
// final root of a component is its smallest vertex ID.  Finds use path halving (both
// ideas as in ECL-CC, Jaiganesh & Burtscher, HPDC 2018).
__device__ __forceinline__ u32 cc_find(u32* parent, u32 x) {
  while (true) {
    const u32 p = load_coherent(&parent[x]);
    if (p == x) return x;
    const u32 gp = load_coherent(&parent[p]);
    if (gp == p) return p;
    parent[x] = gp;  // path halving: gp is an ancestor of x, gp <= p <= x
    x = gp;
  }
}

__device__ __forceinline__ void cc_union(u32* parent, u32 a, u32 b) {
  while (true) {
    a = cc_find(parent, a);
    b = cc_find(parent, b);
    if (a == b) return;
    if (a < b) {
      const u32 t = a; a = b; b = t;
    }
    // a > b: hang root a below b
    const u32 old = atomicCAS(&parent[a], a, b);
    if (old == a) return;
    a = old;  // a was linked meanwhile; continue from its new parent
  }
}

// One sampled link (Afforest, Sutton, Ben-Nun & Barak, IPDPS 2018): lowers
// parent[r_hi] to r_lo for the current parents r of a and b with one atomicMin and no
// retry loop.  If r_hi had been linked meanwhile, its old link may be dropped, which only
// leaves two sets unmerged that are truly connected (a later pass over every edge of the
// vertices outside the dominant set makes the links left out); every parent stays
// within its component and parent[x] <= x holds throughout.
__device__ __forceinline__ void cc_min_link(u32* parent, u32 a, u32 b) {
  const u32 ra = load_coherent(&parent[a]), rb = load_coherent(&parent[b]);
  if (ra == rb) return;
  const u32 hi = max(ra, rb), lo = min(ra, rb);
  if (load_coherent(&parent[hi]) > lo) atomicMin(&parent[hi], lo);
}

// ---- result counters ----------------------------------------------------------------
// ctr[slot * kNumCtr + i]: i = 0 c1, 1 c2, 2 t2 (same-level apex with w > max(u, v)),
// 3 + cls: elements streamed from partner lists, 6 + cls: elements of N(x) staged or
// merged, for cls = 0 lane, 1 wavefront, 2 workgroup class.
constexpr int kNumCtr = 10;

struct Counts {
  u64 c1, c2, t2, probes, staged;
};

__device__ __forceinline__ void Tally::fold(Counts& c) {
  c.c1 += s - 2 * c2;
  c.c2 += c2;
  c.t2 += t2;
  c.probes += probes;
  s = c2 = t2 = probes = 0;
}

// Tally one common neighbour w of the cover edge {x, y}: r = 1 when w is on another
// level than x (c1), r = 2 on the same level (c2; counted into T only when w is larger
// than both endpoints).  Returns whether the triangle {x, y, w} is counted.
__device__ __forceinline__ bool count_hit(u32 r, u32 w, u32 vmax, Counts& c) {
  if (r == 1) {
    c.c1 += 1;
    return true;
  }
  if (r == 2) {
    c.c2 += 1;
    if (w > vmax) {
      c.t2 += 1;
      return true;
    }
  }
  return false;
}

// Adds v to the per-vertex count tri[u] (skipped when v is 0).
__device__ __forceinline__ void tri_add(u64* tri, u32 u, u64 v) {
  if (v) atomicAdd((unsigned long long*)&tri[u], (unsigned long long)v);
}

// First index in [lo, hi) of the sorted array a with a[i] >= v.
__device__ __forceinline__ u32 lower_bound_g(const u32* __restrict__ a, u32 lo, u32 hi, u32 v) {
  while (lo < hi) {
    // lo and hi are absolute entry positions (up to 2^32 - 2^20): lo + hi would wrap
    const u32 mid = lo + ((hi - lo) >> 1);
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Block-wide reduction of the counters followed by one atomic per counter into the
// slot chosen by the block index.  `s_red` holds 5 * (blockDim.x / kWave) u64.
__device__ __forceinline__ void block_flush_counts(Counts c, int cls, u64* __restrict__ ctr,
                                                   u64* s_red) {
  u64 v[5] = {c.c1, c.c2, c.t2, c.probes, c.staged};
  const u32 wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    v[i] = wave_sum_u64(v[i]);
    if (lane_id() == 0) s_red[wid * 5 + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    u64 s = 0;
    for (u32 w = 0; w < nw; ++w) s += s_red[w * 5 + threadIdx.x];
    const int idx = threadIdx.x < 3 ? (int)threadIdx.x : (threadIdx.x == 3 ? 3 + cls : 6 + cls);
    if (s) atomicAdd((unsigned long long*)&ctr[(blockIdx.x % kCounterSlots) * kNumCtr + idx],
                     (unsigned long long)s);
  }
}

}  // namespace tc

// Per-vertex and per-item intersection routines shared by the single-graph kernels and
// the batched per-graph kernel, and the row-split step of cover-edge extraction.
//
// Indexing: vertex IDs and rowptr / split values are local to a graph; neighbour
// arrays (colidx, colidx2, hadj) are indexed absolutely, at cb + a local offset, where
// cb is the graph's first stored entry (0 for a single graph).  Quads of 16 bytes are
// aligned to the start of the neighbour array, so per-graph offsets need no alignment.
// Partner IDs are read as hadj[i * HS]: HS = 1 for a plain partner list, 4 for the
// .w field of the single-graph partner records (PartnerRec).
//
// A partner record (uint4) of cover edge {x, y}, stored under x, holds absolute offsets
// into the level-split rows: .x = the first same-level neighbour of y above max(x, y),
// .y = the start of y's other-level neighbours, .z = the end of y's row, .w = y.  The
// apex rule counts exactly the common neighbours of x and y in y's entries .x .. .z
// that are other-level or above x, which are the entries of x's row from sabove[x] on
// (its same-level neighbours above x, then its other-level ones): every hit of the two
// ranges is one counted apex, so the pruned passes need membership only.
#pragma once

#include "tc_device.h"
#include "tc_launch.h"

namespace tc {

constexpr int kWaveSlots = 2048;   // LDS hash slots per wavefront (d(x) <= 512)
constexpr int kIsectThreads = 256;
constexpr int kUnroll = 4;         // independent list loads in flight per lane
static_assert(kUnroll == 4, "the wavefront routine packs one mark byte per window in a word");
constexpr u32 kWaveClaim = 16;     // wavefront-class vertices claimed per counter atomic
constexpr int kBigThreads = 1024;
constexpr int kBigWaves = kBigThreads / kWave;
constexpr int kBigSlots = 32768;   // 128 KB of LDS
constexpr int kBigSeg = 1024;      // partners per work item (one per thread for set-up)
constexpr int kQuadUnroll = 4;     // windows per wavefront loaded before probing
static_assert(kBigSlots == kBigWaves * kWaveSlots, "the wavefront tables share the big table");

// ---- lane class: one thread merges N(x) with each partner's list ---------------------
template <bool PV, int HS = 1>
__device__ __forceinline__ void lane_vertex(const u32* __restrict__ rowptr, u32 cb,
                                            const u32* __restrict__ colidx,
                                            const uint8_t* __restrict__ vinfo,
                                            const u32* __restrict__ hcnt,
                                            const u32* __restrict__ hadj, u32 x, Counts& c,
                                            u64* __restrict__ tri) {
  const u32 bx = cb + rowptr[x], ex = cb + rowptr[x + 1], np = hcnt[x];
  const u32 px = vinfo[x] & 0x80u;
  u64 xh = 0;  // PV: counted triangles of x, added once at the end
  for (u32 q = 0; q < np; ++q) {
    const u32 y = hadj[(size_t)(bx + q) * HS];
    u32 yh = 0;  // PV: counted triangles of this cover edge, added to t(y) once
    u32 i = bx, j = cb + rowptr[y];
    const u32 je = cb + rowptr[y + 1];
    c.probes += je - j;
    c.staged += ex - i;
    const u32 vmax = max(x, y);
    if (i < ex && j < je) {
      u32 a = colidx[i], b = colidx[j];
      while (true) {
        if (a < b) {
          if (++i == ex) break;
          a = colidx[i];
        } else if (a > b) {
          if (++j == je) break;
          b = colidx[j];
        } else {
          const u32 r = 1u + (((vinfo[a] & 0x80u) == px) ? 1u : 0u);
          if (count_hit(r, a, vmax, c) && PV) {
            tri_add(tri, a, 1);
            ++yh;
          }
          if (++i == ex || ++j == je) break;
          a = colidx[i];
          b = colidx[j];
        }
      }
    }
    if (PV) {
      tri_add(tri, y, yh);
      xh += yh;
    }
  }
  if (PV) tri_add(tri, x, xh);
}

// ---- wave class: one wavefront per staged vertex x -----------------------------------
// Row data of a staged vertex, loaded ahead of its turn by the pruned kernel.
struct WaveMeta {
  u32 bx, ex, sb, np;  // row start and end, first staged entry, partner count
};

__device__ __forceinline__ WaveMeta wave_meta(const u32* __restrict__ rowptr,
                                              const u32* __restrict__ sabove,
                                              const u32* __restrict__ hcnt, u32 x) {
  return WaveMeta{rowptr[x], rowptr[x + 1], sabove[x], hcnt[x]};
}

// N(x) goes to the wavefront's LDS hash set (kWaveSlots slots).  The partners' lists are
// taken 64 at a time, padded out to whole 16-byte quads (VEC) and concatenated; each lane
// then loads one quad per window, so a lane has 4 * kUnroll list elements in flight.
// The partner of a quad comes from the partners' quad ends: those inside the current
// windows mark their positions in LDS, and a ballot plus a population count gives every
// lane its partner.  pinfo / pend / mark are the wavefront's 64-entry LDS arrays.
// REC = false: the full form (N(x) with level flags against each partner's whole row of
// colidx; c1, c2, t2).  REC = true: the pruned form over the level-split rows (colidx
// is then colidx2): x's entries from sabove[x] on against each partner record's range,
// membership only; every hit goes to s.  With REC the row data comes in mt (loaded
// ahead by the caller) and the first 64 partner records are loaded before the staged
// set is built, so their latency overlaps the inserts.  ST (with REC): hits in a
// record's same-level range (.x .. .y) go to tl.t2, those in its other-level range
// (.y .. .z) to tl.s, so the two terms of the split (Alg. CETC-Seq-S) come out apart.
// SR: the full form over the level-split rows (colidx is then colidx2, with 4 readable
// entries past m): mt holds x's row, its split point (mt.sb, the start of its
// other-level part) and its partner count, so an entry's level flag is its position in
// the row (no level gathers); the first 64 partners and their row bounds are loaded
// before the staged set is built.
// SA: the pruned count over the level-split rows with a plain partner list: mt as with
// SR but mt.sb = sabove[x], x's entries from there on staged as plain keys, each partner
// y's row streamed from vrec[y].y = sabove[y] to vrec[y].w (graph-local, like rowptr),
// membership only (the hits are those of the records' ranges, see kPartAbove).
template <bool PV, bool VEC, bool REC = false, int HS = 1, bool ST = false, bool SR = false,
          bool SA = false>
__device__ __forceinline__ void wave_vertex(
    const u32* __restrict__ rowptr, u32 cb, const u32* __restrict__ colidx, u32 m,
    const u32* __restrict__ tail4, const uint8_t* __restrict__ vinfo,
    const u32* __restrict__ hcnt, const u32* __restrict__ hadj,
    const uint4* __restrict__ hrec, const uint4* __restrict__ vrec, u32 x, WaveMeta mt,
    u32* table, uint4* pinfo, u32* pend, u32* mark, Tally& tl, Counts& c,
    u64* __restrict__ tri) {
  static_assert(!PV || (REC && !ST), "per-vertex counts: the pruned form without split tallies");
  static_assert(!ST || REC, "split statistics come from the partner records");
  static_assert(!(SR && (REC || PV || HS != 1)), "split rows: full form over plain partner lists");
  static_assert(!(SA && (REC || SR || PV || HS != 1)), "sabove ranges: plain partner lists");
  constexpr bool MT = REC || SR || SA;  // row data from mt
  constexpr bool KEYS = REC || SA;      // pruned: plain staged keys, membership count
  constexpr bool PL = SR || SA;         // plain partner list, first 64 partners ahead
  constexpr u32 NE = VEC ? 4 : 1;       // elements per quad
  const u32 lane = lane_id();
  const u64 le = lane == kWave - 1 ? ~0ull : (2ull << lane) - 1;
  const u32 bx = MT ? mt.bx : cb + rowptr[x], ex = MT ? mt.ex : cb + rowptr[x + 1];
  const u32 sb = KEYS ? mt.sb : bx;  // first staged entry
  const u32 sp = SR ? mt.sb : 0u;    // SR: first other-level entry of x's row
  const u32 dx = ex - sb;
  const u32 hs = bx, np = MT ? mt.np : hcnt[x];  // H+(x) sits in place of N(x)
  const u32 px = MT ? 0u : vinfo[x] & 0x80u;
  uint4 r0 = make_uint4(0, 0, 0, 0);  // REC: the first batch of partner records
  if (REC && lane < np) r0 = hrec[hs + lane];
  u32 y0 = 0, lo0 = 0, hi0 = 0;       // PL: the first batch of partners and their rows
  if (PL && lane < np) {
    y0 = hadj[hs + lane];
    if (SA) {
      const uint4 r = vrec[y0];
      lo0 = cb + r.y;
      hi0 = cb + r.w;
    } else {
      lo0 = cb + rowptr[y0];
      hi0 = cb + rowptr[y0 + 1];
    }
  }
  // PV: the set fills the lower half of the wavefront's table and the upper half counts
  // the hits of each slot's key, added to t(w) once at the end
  constexpr u32 kCnt = kWaveSlots / 2;
  const u32 mask = bucket_mask(dx, PV ? kCnt : (u32)kWaveSlots);
  c.staged += lane == 0 ? dx : 0;
  u32 xh = 0;  // PV: this lane's counted triangles of x, summed over the wavefront at the end
  // pruned forms: the staged keys (at most kWaveSlots / 4, i.e. 8 per lane) are all
  // loaded before the table is cleared and filled
  constexpr u32 SK = KEYS ? kWaveSlots / 4 / kWave : 1;
  u32 sk[SK];
  if (KEYS) {
#pragma unroll
    for (u32 t = 0; t < SK; ++t) {
      const u32 i = lane + t * kWave;
      sk[t] = i < dx ? colidx[sb + i] : 0u;
    }
  }
  for (u32 i = lane; i < (mask + 1) * 4; i += kWave) {
    table[i] = kInf;
    if (PV) table[kCnt + i] = 0;
  }
  wave_lds_sync();
  if (KEYS) {
#pragma unroll
    for (u32 t = 0; t < SK; ++t)
      if (lane + t * kWave < dx) hash_insert_key(table, mask, sk[t], sk[t]);
  }
  for (u32 i = lane; !KEYS && i < dx; i += kWave) {
    const u32 w = colidx[sb + i];
    if (SR) {
      hash_insert(table, mask, w, sb + i < sp ? 1u : 0u);
    } else {
      const u32 same = ((vinfo[w] & 0x80u) == px) ? 1u : 0u;
      hash_insert(table, mask, w, same);
    }
  }
  wave_lds_sync();
  for (u32 pb = 0; pb < np; pb += kWave) {
    const u32 p = pb + lane;
    u32 y = 0, lo = 0, hi = 0;
    if (p < np) {
      if (REC) {
        const uint4 r = pb == 0 ? r0 : hrec[hs + p];
        y = ST ? r.y : r.w;  // the pruned form reads y for per-vertex counts only; ST keeps the range split there
        lo = r.x;
        hi = r.z;
      } else if (PL && pb == 0) {
        y = y0;
        lo = lo0;
        hi = hi0;
      } else if (SA) {
        y = hadj[hs + p];
        const uint4 r = vrec[y];
        lo = cb + r.y;
        hi = cb + r.w;
      } else {
        y = hadj[(size_t)(hs + p) * HS];
        lo = cb + rowptr[y];
        hi = cb + rowptr[y + 1];
      }
    }
    tl.probes += hi - lo;
    const u32 qa = VEC ? (lo & ~3u) : lo;
    const u32 nq = lo < hi ? (VEC ? (hi - qa + 3u) >> 2 : hi - lo) : 0u;
    const u32 incl = wave_incl_scan(nq);
    const u32 total = __shfl(incl, kWave - 1, kWave);
    // partners with elements, compacted: their quad ends are strictly increasing
    const u64 ne = __ballot(nq > 0);
    const u32 npc = (u32)__popcll(ne);
    if (nq > 0) {
      const u32 r = mask_rank(ne);
      pinfo[r] = make_uint4((VEC ? qa >> 2 : qa) - (incl - nq), lo, hi, y);
      pend[r] = incl;
    }
    wave_lds_sync();
    const u32 my_end = lane < npc ? pend[lane] : kInf;  // quad end of partner `lane`
    for (u32 k0 = 0; k0 < total; k0 += kWave * kUnroll) {
      // Quad q belongs to partner #{r : end_r <= q}.  Partner ends strictly inside one of
      // the kUnroll windows of 64 quads from k0 mark their position (byte u of word j for
      // position 64 u + j); ends at a window start count in that window's base.
      mark[lane] = 0;
      wave_lds_sync();
      const u32 t = my_end - k0;
      if (my_end > k0 && t < kWave * kUnroll && (t & (kWave - 1)) != 0)
        reinterpret_cast<uint8_t*>(mark)[(t & (kWave - 1)) * 4 + t / kWave] = 1;
      wave_lds_sync();
      const u32 word = mark[lane];
      u32 e[kUnroll][NE];
      uint4 inf[kUnroll];
      u32 addr[kUnroll];
      bool live[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const u32 w0 = k0 + u * kWave;
        const u32 q = w0 + lane;
        const u64 mk = __ballot(((word >> (8 * u)) & 0xFFu) != 0);
        const u32 base = (u32)__popcll(__ballot(my_end <= w0));
        const u32 l = min(base + (u32)__popcll(mk & le), npc - 1);
        live[u] = q < total;
        inf[u] = pinfo[l];
        addr[u] = (inf[u].x + q) * NE;
        if (VEC) {
          // one unconditional 16-byte load: a quad that would run past the end of colidx
          // (or a dead lane) reads the padded copy of the last partial quad; REC and SR
          // rows (colidx2) have 4 readable entries past m, so a quad only clamps its address
          const u32* src = MT ? colidx + min(addr[u], (m - 1) & ~3u)
                              : (live[u] && addr[u] + 3 < m) ? colidx + addr[u] : tail4;
          const uint4 v = *reinterpret_cast<const uint4*>(src);
          e[u][0] = v.x;
          e[u][NE > 1 ? 1 : 0] = v.y;
          e[u][NE > 2 ? 2 : 0] = v.z;
          e[u][NE > 3 ? 3 : 0] = v.w;
        } else {
          e[u][0] = colidx[live[u] ? addr[u] : 0u];
        }
      }
      if constexpr (SA) __builtin_amdgcn_sched_barrier(0);  // as in subwave_vertex
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const u32 y2 = inf[u].w;
        const u32 vmax = max(x, y2);
        const u32 span = inf[u].z - inf[u].y;  // elements lo .. hi-1 are valid
        bool ok[NE];
#pragma unroll
        for (u32 i = 0; i < NE; ++i) ok[i] = live[u] && (addr[u] + i - inf[u].y) < span;
        if (REC && ST) {
          bool sm[NE];
#pragma unroll
          for (u32 i = 0; i < NE; ++i) sm[i] = addr[u] + i < inf[u].w;
          hash_count_split_n<NE, true>(table, mask, e[u], ok, sm, tl.s, tl.t2);
        } else if (KEYS && PV) {
          // every hit is a counted apex: count it under its slot, its partner and x
          u32 sl[NE], qh = 0;
          hash_slots_n<NE>(table, mask, e[u], ok, sl);
#pragma unroll
          for (u32 i = 0; i < NE; ++i) {
            if (sl[i] != kInf) {
              atomicAdd(&table[kCnt + sl[i]], 1u);
              ++qh;
            }
          }
          tri_add(tri, y2, qh);
          xh += qh;
          tl.s += qh;
        } else if (KEYS) {
          hash_count_n<NE>(table, mask, e[u], ok, tl.s);
        } else {
          u32 res[NE];
          hash_probe_n<NE>(table, mask, e[u], ok, res);
#pragma unroll
          for (u32 i = 0; i < NE; ++i) tl.add(res[i], e[u][i], vmax);
        }
      }
    }
    wave_lds_sync();
  }
  if (PV) {
    for (u32 i = lane; i < (mask + 1) * 4; i += kWave) {
      const u32 k = table[kCnt + i];
      if (k) tri_add(tri, table[i] & ~kFlag, k);
    }
    const u64 sx = wave_sum_u64(xh);
    if (lane == 0) tri_add(tri, x, sx);
    wave_lds_sync();  // the next vertex clears the table
  }
}

// ---- sub-wavefront class: four staged vertices per wavefront ---------------------------
// A staged vertex with a few dozen entries and a handful of partners fills a small part
// of a wavefront's 64 lanes and windows.  Here each group of 16 lanes takes its own x:
// its staged entries go to the group's 256-slot LDS hash set, its partners' ranges are
// streamed 16 partners at a time, 4 quads per lane in flight, and the owner of a quad is
// found by a binary search over the group's quad prefix sums (cross-lane reads, no LDS
// marks).  x's entries from mt.sb = sabove[x] on are staged as plain keys, and the
// staged keys and the first 16 partners' ranges are loaded before the table is built.
// Where the partners and their ranges come from (PM):
//   kPartRec   : partner records hrec (pruned count): x's entries from mt.sb = sabove[x]
//                on staged as plain keys, each record's range .x .. .z streamed,
//                membership only (every hit a counted apex, in tl.s);
//   kPartAbove : plain partner list hadj with the per-vertex row records vrec (pruned
//                count, batched): staged as kPartRec, each partner y's row streamed from
//                vrec[y].y = sabove[y], its first same-level entry above y, to its end
//                vrec[y].w, membership only.  For x > y the
//                range also holds y's same-level entries in (y, x], which the staged
//                keys (same-level ones above x only) never match, so the hits are the
//                same as with the range from above max(x, y).
// PV (kPartRec): per-vertex counts of the group's vertex x: t(x) summed over the group,
// t(y) added once per quad, t(w) counted per slot of the group's set in the unused upper
// half of the wavefront table and added once at the end.
// All 64 lanes call it together; a group without a vertex passes mt.np = 0 and an empty
// row.
constexpr u32 kSubLanes = 16;
constexpr u32 kSubGroups = kWave / kSubLanes;
constexpr u32 kSubMax = 64;     // d(x) of the sub-wavefront class at most
constexpr u32 kSubSlots = 256;  // LDS hash slots per group
constexpr u32 kSubU = 4;        // quads per lane in flight
constexpr u32 kSubCnt = kSubGroups * kSubSlots;  // PV: a group's slot counters sit this far on
static_assert(2 * kSubCnt <= kWaveSlots, "the groups' sets and counters share one wavefront table");

__device__ __forceinline__ u32 group_incl_scan(u32 v) {
  const u32 gl = lane_id() & (kSubLanes - 1);
#pragma unroll
  for (u32 off = 1; off < kSubLanes; off <<= 1) {
    const u32 t = __shfl_up(v, off, kSubLanes);
    if (gl >= off) v += t;
  }
  return v;
}

__device__ __forceinline__ u32 wave_max_u32(u32 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, (u32)__shfl_xor(v, off, kWave));
  return v;
}

enum PartnerMode { kPartRec = 1, kPartAbove = 2 };

// colidx2 has 4 readable entries past m; table is this group's kSubSlots slots; vrec
// (kPartAbove) is local to the graph like rowptr: {row start, sabove, split, row end}.
template <int PM, bool PV = false>
__device__ __forceinline__ void subwave_vertex(const u32* __restrict__ colidx2, u32 m, u32 cb,
                                               const u32* __restrict__ hadj,
                                               const uint4* __restrict__ hrec,
                                               const uint4* __restrict__ vrec,
                                               const WaveMeta& mt, u32* table, Tally& tl,
                                               Counts& c, u32 x = 0, u64* __restrict__ tri = nullptr) {
  static_assert(PM == kPartRec || PM == kPartAbove, "pruned forms only");
  static_assert(!PV || PM == kPartRec, "per-vertex counts come from the records");
  constexpr u32 SK = kSubMax / kSubLanes;  // staged keys per lane at most
  const u32 lane = lane_id(), gl = lane & (kSubLanes - 1), gb = lane & ~(kSubLanes - 1);
  const u32 bx = mt.bx, np = mt.np, sb = mt.sb;
  const u32 dx = mt.ex - sb;  // staged entries: x's row from sabove[x] on
  // the partner info of batch b (up to 16 partners, one per lane of the group)
  auto partner = [&](u32 b, u32& lo, u32& hi, u32& y) {
    const u32 p = b * kSubLanes + gl;
    lo = hi = y = 0;
    if (p < np) {
      if (PM == kPartRec) {
        const uint4 r = hrec[bx + p];  // the records sit in place of N(x)
        lo = r.x;
        hi = r.z;
        y = r.w;
      } else {
        const uint4 r = vrec[hadj[bx + p]];  // one 16-byte load: the row's sabove and end
        lo = cb + r.y;
        hi = cb + r.w;
      }
    }
  };
  // the staged keys and the first batch of partners are loaded before the table is
  // cleared and filled, so their round trips overlap
  u32 sk[SK];
#pragma unroll
  for (u32 t = 0; t < SK; ++t) {
    const u32 i = gl + t * kSubLanes;
    sk[t] = i < dx ? colidx2[sb + i] : 0u;
  }
  u32 lo0, hi0, y0;
  partner(0, lo0, hi0, y0);
  const u32 mask = bucket_mask(dx ? dx : 1u, kSubSlots);
  c.staged += gl == 0 ? dx : 0;
  u32 xh = 0;  // PV: this lane's counted triangles of x
  for (u32 i = gl; i < (mask + 1) * 4; i += kSubLanes) {
    table[i] = kInf;
    if (PV) table[kSubCnt + i] = 0;
  }
  wave_lds_sync();
#pragma unroll
  for (u32 t = 0; t < SK; ++t)
    if (gl + t * kSubLanes < dx) hash_insert_key(table, mask, sk[t], sk[t]);
  wave_lds_sync();
  const u32 nbat = wave_max_u32((np + kSubLanes - 1) / kSubLanes);
  for (u32 b = 0; b < nbat; ++b) {
    u32 lo = lo0, hi = hi0, y = y0;
    if (b > 0) partner(b, lo, hi, y);
    tl.probes += hi - lo;
    const u32 qa = lo & ~3u;
    const u32 nq = lo < hi ? (hi - qa + 3u) >> 2 : 0u;
    const u32 incl = group_incl_scan(nq);
    const u32 total = __shfl(incl, (int)(gb + kSubLanes - 1), kWave);
    const u32 qbase = (qa >> 2) - (incl - nq);  // quad q of the group's concatenation: qbase + q
    const u32 tmax = wave_max_u32(total);
    for (u32 k0 = 0; k0 < tmax; k0 += kSubLanes * kSubU) {
      u32 e[kSubU][4];
      u32 addr[kSubU], jlo[kSubU], jspan[kSubU], jy[kSubU];
      bool live[kSubU];
#pragma unroll
      for (u32 u = 0; u < kSubU; ++u) {
        const u32 q = k0 + u * kSubLanes + gl;
        live[u] = q < total;
        // owner: the first lane of the group whose inclusive quad count exceeds q
        u32 a = 0, z = kSubLanes - 1;
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const u32 mid = (a + z) >> 1;
          const u32 im = (u32)__shfl(incl, (int)(gb + mid), kWave);
          if (im > q) z = mid;
          else a = mid + 1;
        }
        const int j = (int)(gb + a);
        const u32 qb = (u32)__shfl(qbase, j, kWave);
        jlo[u] = (u32)__shfl(lo, j, kWave);
        jspan[u] = (u32)__shfl(hi, j, kWave) - jlo[u];
        jy[u] = PV ? (u32)__shfl(y, j, kWave) : 0u;
        addr[u] = (qb + q) * 4;
        const uint4 v = *reinterpret_cast<const uint4*>(colidx2 + min(addr[u], (m - 1) & ~3u));
        e[u][0] = v.x;
        e[u][1] = v.y;
        e[u][2] = v.z;
        e[u][3] = v.w;
      }
      // batched (kPartAbove): all kSubU loads in flight before the probes; in the fused
      // kernel's register budget the scheduler otherwise starts hashing the first
      // window's elements, which waits for its load, before it issues the next one (the
      // single-graph kernels are scheduled well and measured slower with the barrier)
      if constexpr (PM == kPartAbove) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (u32 u = 0; u < kSubU; ++u) {
        bool ok[4];
#pragma unroll
        for (u32 i = 0; i < 4; ++i) ok[i] = live[u] && (addr[u] + i - jlo[u]) < jspan[u];
        if (PV) {
          u32 sl[4], qh = 0;
          hash_slots_n<4>(table, mask, e[u], ok, sl);
#pragma unroll
          for (u32 i = 0; i < 4; ++i) {
            if (sl[i] != kInf) {
              atomicAdd(&table[kSubCnt + sl[i]], 1u);
              ++qh;
            }
          }
          tri_add(tri, jy[u], qh);
          xh += qh;
          tl.s += qh;
        } else {
          hash_count_n<4>(table, mask, e[u], ok, tl.s);
        }
      }
    }
  }
  wave_lds_sync();  // the table is reused by the next vertex of the group
  if (PV) {
    for (u32 i = gl; i < (mask + 1) * 4; i += kSubLanes) {
      const u32 k = table[kSubCnt + i];
      if (k) tri_add(tri, table[i] & ~kFlag, k);
    }
#pragma unroll
    for (u32 off = kSubLanes / 2; off > 0; off >>= 1) xh += (u32)__shfl_xor(xh, (int)off, kSubLanes);
    if (gl == 0) tri_add(tri, x, xh);
    wave_lds_sync();
  }
}

// ---- block class: one 1024-thread workgroup per (x, segment of partners) ------------
// N(x) is staged chunk by chunk (at most prm.chunk <= 16384 entries per chunk, 4096 by
// default so that the 128 KB LDS hash set stays at most 1/8 full).  For each chunk every
// partner list is cut at the chunk's largest ID (one binary search from the previous
// chunk's cut, only when N(x) needs several chunks) and padded out to whole 16-byte quads;
// the concatenated quad space is split into one contiguous range per wavefront.  A
// wavefront walks its range in windows of 64 quads, one quad (16-byte load) per lane,
// and keeps the current partner as it goes: the partner boundaries (quad prefix sums in
// LDS) that fall inside a window are applied with a few lane-uniform steps, so no
// per-lane search is needed.  Every partner element is probed exactly once, against the
// first chunk whose largest ID is not below it.
// What one pass of the workgroup kernel stages, streams and tallies:
//   kFull     : N(x) with level flags; each partner's whole list; c1, c2 and t2
//               (diagnostics and per-vertex counts);
//   kOther    : the other-level part of N(x); each partner's other-level part (hits
//               are the other-level apexes);
//   kSame     : the same-level part of N(x) above x; each partner's same-level part
//               above max(x, y) (hits are the same-level apexes above both ends);
//   kMember   : x's entries from sabove[x] on in one chunk; each partner record's range
//               (hits are the counted apexes of both kinds).
// A same-level apex w <= max(x, y) is never counted (the apex rule), so the pruned
// passes skip those list entries entirely and leave c2 uncounted.  kOther, kSame and
// kMember stage plain IDs, probe for membership only; kSame adds its hits to t2, kOther
// and kMember to s (with ST, kMember's hits in the range before the split point carried
// in place of y go to t2).
enum BlockMode { kFull = 0, kOther = 1, kSame = 2, kMember = 3 };

struct BlockShared {
  u32* table;
  u32* qincl;
  uint4* pinfo;
  u32* tmp;
  u32* ycnt;  // per-vertex counts: counted triangles per partner of the item (LDS)
};

// Per-vertex counts in the pruned hash passes: chunks of at most kPvChunk keys fill the
// lower half of the table, and the upper half (from kPvCnt) counts the hits of each
// slot's key, added to t(w) once per chunk.
constexpr u32 kPvCnt = kBigSlots / 2;
constexpr u32 kPvChunk = kPvCnt / 4;  // buckets at most a quarter full

// One pass over the partners of a work item.  The staged keys ga[gs .. ge) (ascending)
// go to LDS either as hash sets of at most prm.chunk keys (BM = false) or, for the
// level-specific pruned passes, as bitmaps of one 2^kWinBits-ID window each (BM = true,
// one bit per ID: these passes need membership only).  Partner `tid` < pn streams
// sa[plo .. phi), cut at each chunk's largest ID or window end.  All threads of the
// workgroup call it together.
constexpr u32 kWinBits = 20;  // 2^20 IDs per bitmap window = 128 KB of LDS

// PAD: the streamed array has at least 4 readable entries past its m counted ones, so
// every live quad is read in place and dead lanes only clamp their address.
// QU windows of 64 quads per wavefront are loaded before probing; FENCE keeps the
// scheduler from moving probe work between those loads (batched kernel).
template <bool PV, bool VEC, int MODE, bool BM, bool PAD = false, int QU = kQuadUnroll,
          bool ST = false, bool FENCE = false>
__device__ __forceinline__ void block_pass(
    const u32* __restrict__ sa, u32 m, const u32* __restrict__ st4, const u32* __restrict__ ga,
    u32 gs, u32 ge, const uint8_t* __restrict__ vinfo, u32 x, u32 px, u32 y, u32 pn, u32 plo,
    u32 phi, IsectParams prm, const BlockShared& sh, Tally& tl, Counts& c, u64* __restrict__ tri) {
  constexpr u32 NE = VEC ? 4 : 1;  // elements per quad (a quad is one element without VEC)
  const u32 tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
  static_assert(!BM || MODE == kOther || MODE == kSame, "bitmaps hold membership only");
  static_assert(!ST || MODE == kMember, "only the one-chunk member pass mixes both kinds");
  constexpr bool MEMBER = MODE == kOther || MODE == kSame || MODE == kMember;
  u32& hits = MODE == kSame ? tl.t2 : tl.s;  // same-level apexes above both ends: t2
  const u32 glen = ge - gs;
  static_assert(!PV || (MEMBER && !BM && !ST), "per-vertex counts: pruned hash passes only");
  const u32 chunk = PV ? min(prm.chunk, kPvChunk) : prm.chunk;
  u32 xh = 0;  // PV: this thread's counted triangles of x
  u32 yp = 0, ya = 0;  // PV: a partner index and its hits not yet in sh.ycnt
  if (PV && tid < pn) sh.ycnt[tid] = 0;
  // hash chunks by count, or bitmap windows by ID
  const u32 w_first = BM && glen ? ga[gs] >> kWinBits : 0u;
  const u32 nch = BM ? (glen ? (ga[ge - 1] >> kWinBits) - w_first + 1 : 0u)
                     : (glen + chunk - 1) / chunk;
  u32 lo = plo;  // cursor: elements below it were probed against earlier chunks
  u32 c0 = gs;   // first staged key of the chunk
  for (u32 ch = 0; ch < nch; ++ch) {
    const u32 wb = (w_first + ch) << kWinBits;  // BM: window [wb, wb + 2^kWinBits)
    u32 clen;
    if (BM) {
      clen = lower_bound_g(ga, c0, ge, wb + (1u << kWinBits)) - c0;
      if (clen == 0) continue;  // no staged key in this window (uniform)
    } else {
      clen = min(chunk, ge - c0);
    }
    const u32 mask = BM ? 0u : bucket_mask(clen, PV ? kPvCnt : (u32)kBigSlots);
    c.staged += tid == 0 ? clen : 0;
    if (BM) {
      uint4* t4 = reinterpret_cast<uint4*>(sh.table);
      for (u32 i = tid; i < (u32)kBigSlots / 4; i += blockDim.x) t4[i] = make_uint4(0, 0, 0, 0);
    } else {
      for (u32 i = tid; i < (mask + 1) * 4; i += blockDim.x) {
        sh.table[i] = kInf;
        if (PV) sh.table[kPvCnt + i] = 0;
      }
    }
    // this partner's elements up to the chunk's largest ID or the window's end (the
    // ones between two chunks are in no chunk and find nothing in either)
    u32 hi = phi;
    if (tid < pn && ch + 1 < nch)
      hi = lower_bound_g(sa, lo, phi, BM ? wb + (1u << kWinBits) : ga[c0 + clen - 1] + 1u);
    tl.probes += hi - lo;
    const u32 qa = VEC ? (lo & ~3u) : lo;
    const u32 nq = lo < hi ? (VEC ? (hi - qa + 3u) >> 2 : hi - lo) : 0u;
    u32 total;
    const u32 incl = block_incl_scan(nq, sh.tmp, &total);
    if (tid < pn) {
      sh.qincl[tid] = incl;
      sh.pinfo[tid] = make_uint4((VEC ? qa >> 2 : qa) - (incl - nq), lo, hi, y);
    }
    if (BM) {
      __syncthreads();  // the bitmap is cleared
      for (u32 i = tid; i < clen; i += blockDim.x) {
        const u32 k = ga[c0 + i] - wb;
        atomicOr(&sh.table[k >> 5], 1u << (k & 31u));
      }
    } else {
      for (u32 i = tid; i < clen; i += blockDim.x) {
        const u32 w = ga[c0 + i];
        if (MEMBER) {
          hash_insert_key(sh.table, mask, w, w);
        } else {
          const bool same = MODE == kFull && (vinfo[w] & 0x80u) == px;
          hash_insert(sh.table, mask, w, same ? 1u : 0u);
        }
      }
    }
    __syncthreads();
    // this wavefront's contiguous quad range, in whole windows
    const u32 per = (total + kBigWaves * kWave - 1) / (kBigWaves * kWave) * kWave;
    const u32 qs = min(wid * per, total), qe = min(qs + per, total);
    // partner of quad qs: smallest p with qincl[p] > qs (lane-uniform search)
    u32 pcur = 0;
    {
      u32 h = pn - 1;
      while (pcur < h) {
        const u32 mid = (pcur + h) >> 1;
        if (sh.qincl[mid] > qs) h = mid;
        else pcur = mid + 1;
      }
    }
    for (u32 qw = qs; qw < qe; qw += kWave * QU) {
      u32 e[QU][NE];
      uint4 inf[QU];
      u32 addr[QU];
      bool live[QU];
      u32 pidx[QU];  // PV: the quad's partner
#pragma unroll
      for (int u = 0; u < QU; ++u) {
        const u32 w0 = qw + u * kWave;        // first quad of this window
        const u32 q = w0 + lane;
        live[u] = q < qe;
        // partner of q: pcur plus the boundaries (qincl values) <= q in this window
        u32 p = pcur;
        while (true) {
          const u32 j = pcur + lane;
          const u32 bj = j < pn ? sh.qincl[j] : kInf;
          u64 bm = __ballot(bj <= w0 + kWave - 1);
          const u32 nb = (u32)__popcll(bm);
          while (bm) {
            const int jl = __ffsll((unsigned long long)bm) - 1;
            bm &= bm - 1;
            p += q >= (u32)__shfl(bj, jl, kWave) ? 1u : 0u;
          }
          pcur += nb;
          if (nb < (u32)kWave) break;
        }
        p = min(p, pn - 1);  // lanes past the range keep a valid index
        pidx[u] = p;
        inf[u] = sh.pinfo[p];
        addr[u] = (inf[u].x + q) * NE;
        if (VEC) {
          // one unconditional 16-byte load: a quad that would run past the end of the
          // streamed array (or a dead lane) reads the padded copy of its last partial quad,
          // or with PAD its own padded tail (a live quad starts at or below m - 1)
          const u32* src = PAD ? sa + min(addr[u], (m - 1) & ~3u)
                               : (live[u] && addr[u] + 3 < m) ? sa + addr[u] : st4;
          const uint4 v = *reinterpret_cast<const uint4*>(src);
          e[u][0] = v.x;
          e[u][NE > 1 ? 1 : 0] = v.y;
          e[u][NE > 2 ? 2 : 0] = v.z;
          e[u][NE > 3 ? 3 : 0] = v.w;
        } else {
          e[u][0] = sa[live[u] ? addr[u] : 0u];
        }
      }
      if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);  // as in subwave_vertex
#pragma unroll
      for (int u = 0; u < QU; ++u) {
        const u32 y2 = inf[u].w;
        const u32 vmax = max(x, y2);
        const u32 span = inf[u].z - inf[u].y;  // elements lo .. hi-1 are valid
        bool ok[NE];
#pragma unroll
        for (u32 i = 0; i < NE; ++i) ok[i] = live[u] && (addr[u] + i - inf[u].y) < span;
        if (BM) {
          // elements of earlier, skipped windows fall outside [wb, wb + 2^kWinBits)
#pragma unroll
          for (u32 i = 0; i < NE; ++i) {
            const u32 k = e[u][i] - wb;
            const bool in = ok[i] && k < (1u << kWinBits);
            const u32 kk = in ? k : 0u;
            hits += in ? (sh.table[kk >> 5] >> (kk & 31u)) & 1u : 0u;
          }
        } else if (ST) {
          bool sm[NE];
#pragma unroll
          for (u32 i = 0; i < NE; ++i) sm[i] = addr[u] + i < inf[u].w;
          hash_count_split_n<NE, true>(sh.table, mask, e[u], ok, sm, tl.s, tl.t2);
        } else if (MEMBER && PV) {
          // every hit is a counted apex: count it under its slot, its partner and x
          u32 sl[NE], qh = 0;
          hash_slots_n<NE>(sh.table, mask, e[u], ok, sl);
#pragma unroll
          for (u32 i = 0; i < NE; ++i) {
            if (sl[i] != kInf) {
              atomicAdd(&sh.table[kPvCnt + sl[i]], 1u);
              ++qh;
            }
          }
          if (qh) {
            // a lane's quads of one partner run on across windows: add to the partner's
            // counter when the partner changes
            if (pidx[u] != yp) {
              if (ya) atomicAdd(&sh.ycnt[yp], ya);
              yp = pidx[u];
              ya = 0;
            }
            ya += qh;
            xh += qh;
            hits += qh;
          }
        } else if (MEMBER) {
          hash_count_n<NE>(sh.table, mask, e[u], ok, hits);
        } else {
          u32 res[NE];
          hash_probe_n<NE>(sh.table, mask, e[u], ok, res);
#pragma unroll
          for (u32 i = 0; i < NE; ++i) {
            if (MODE == kFull) {
              tl.add(res[i], e[u][i], vmax);
            } else {
              tl.s += res[i] & 1u;  // other-level apex (c1)
              tl.t2 += res[i] >> 1;  // same-level apex above both endpoints
            }
          }
        }
      }
    }
    if (PV && ya) {
      atomicAdd(&sh.ycnt[yp], ya);
      ya = 0;
    }
    __syncthreads();
    if (PV) {
      // t(w) for the chunk's keys; the table is rebuilt only after every thread is done
      for (u32 i = tid; i < (mask + 1) * 4; i += blockDim.x) {
        const u32 k = sh.table[kPvCnt + i];
        if (k) tri_add(tri, sh.table[i] & ~kFlag, k);
      }
      __syncthreads();
    }
    lo = hi;
    c0 += clen;
  }
  if (PV) {
    // every partner's count is complete after the last chunk's barrier
    if (tid < pn) tri_add(tri, y, sh.ycnt[tid]);
    const u64 sx = wave_sum_u64(xh);
    if (lane == 0) tri_add(tri, x, sx);
  }
}

// Bitmap windows for the sorted keys a[s .. e) when they take fewer passes than hash
// chunks of `chunk` keys.
__device__ __forceinline__ bool use_bitmap(const u32* __restrict__ a, u32 s, u32 e, u32 chunk) {
  if (e - s <= chunk) return false;
  const u32 wins = (a[e - 1] >> kWinBits) - (a[s] >> kWinBits) + 1;
  return wins < (e - s + chunk - 1) / chunk;
}

// One work item of the full form: staged vertex x, partner segment `seg` (all threads
// call it together), one kFull pass over colidx.  m bounds the quad loads from colidx
// (beyond it the padded copy tail4 is read).
template <bool VEC, int HS = 1, int QU = kQuadUnroll>
__device__ __forceinline__ void block_item(
    const u32* __restrict__ rowptr, u32 cb, const u32* __restrict__ colidx, u32 m,
    const u32* __restrict__ tail4, const uint8_t* __restrict__ vinfo,
    const u32* __restrict__ hcnt, const u32* __restrict__ hadj, u32 x, u32 seg, IsectParams prm,
    const BlockShared& sh, Tally& tl, Counts& c) {
  const u32 tid = threadIdx.x;
  const u32 bx = cb + rowptr[x], ex = cb + rowptr[x + 1];
  const u32 px = vinfo[x] & 0x80u;
  const u32 hs = bx + seg * prm.seg;  // H+(x) sits in place of N(x)
  const u32 pn = min(prm.seg, hcnt[x] - seg * prm.seg);
  u32 y = 0, yr = 0, ye = 0;
  if (tid < pn) {
    y = hadj[(size_t)(hs + tid) * HS];
    yr = cb + rowptr[y];
    ye = cb + rowptr[y + 1];
  }
  block_pass<false, VEC, kFull, false, false, QU>(colidx, m, tail4, colidx, bx, ex, vinfo, x, px,
                                                  y, pn, yr, ye, prm, sh, tl, c, nullptr);
}

// One work item of the pruned count: x's entries from sabove[x] on are staged once,
// membership only.  When they fit one chunk, one kMember pass streams each partner's
// range .x .. .z; otherwise a kOther pass (x's other-level part against .y .. .z) and a
// kSame pass (x's same-level part above x against .x .. .y), each with hash chunks or
// bitmap windows, whichever takes fewer passes.  The ranges come from the partner records
// (PM = kPartRec, single graph: x's row from rowptr, sabove, split) or from the plain
// partner list with the per-vertex row records vrec = {row start, sabove, split, row
// end}, local to the graph whose entries start at cb (PM = kPartAbove, batched; see
// kPartAbove for why the hits agree).  PAD: colidx2 has 4 readable entries past its m2
// counted ones.  ST (kPartRec): the member pass tallies same-level and other-level hits
// apart (see block_pass).
template <bool VEC, bool PAD = false, bool ST = false, int PM = kPartRec, int QU = kQuadUnroll,
          bool PV = false>
__device__ __forceinline__ void block_item_rec(
    const u32* __restrict__ rowptr, u32 cb, const u32* __restrict__ colidx2, u32 m2,
    const u32* __restrict__ tail4b, const u32* __restrict__ split,
    const u32* __restrict__ sabove, const u32* __restrict__ hcnt,
    const uint4* __restrict__ hrec, const u32* __restrict__ hadj,
    const uint4* __restrict__ vrec, u32 x, u32 seg, IsectParams prm, const BlockShared& sh,
    Tally& tl, Counts& c, u64* __restrict__ tri = nullptr) {
  static_assert(PM == kPartRec || (PM == kPartAbove && !ST), "split tallies need records");
  static_assert(!PV || (PM == kPartRec && !ST), "per-vertex counts: records, no split tallies");
  constexpr bool kFence = PM == kPartAbove;
  const u32 tid = threadIdx.x;
  u32 bx, ex, gx, sx;
  if (PM == kPartRec) {
    bx = cb + rowptr[x];
    ex = cb + rowptr[x + 1];
    gx = cb + sabove[x];
    sx = cb + split[x];
  } else {
    const uint4 rx = vrec[x];
    bx = cb + rx.x;
    gx = cb + rx.y;
    sx = cb + rx.z;
    ex = cb + rx.w;
  }
  const u32 hs = bx + seg * prm.seg;  // the partners sit in place of N(x)
  const u32 pn = min(prm.seg, hcnt[x] - seg * prm.seg);
  uint4 r = make_uint4(0, 0, 0, 0);
  if (tid < pn) {
    if (PM == kPartRec) {
      r = hrec[hs + tid];
    } else {
      const u32 y = hadj[hs + tid];
      const uint4 ry = vrec[y];
      r = make_uint4(cb + ry.y, cb + ry.z, cb + ry.w, y);
    }
  }
  if (PV) {
    // per-vertex counts: hash chunks of at most kPvChunk keys (their slot counters fill
    // the other half of the table), never bitmaps
    if (ex - gx <= min(prm.chunk, kPvChunk)) {
      block_pass<true, VEC, kMember, false, PAD, QU>(colidx2, m2, tail4b, colidx2, gx, ex,
                                                     nullptr, x, 0, r.w, pn, r.x, r.z, prm, sh,
                                                     tl, c, tri);
    } else {
      block_pass<true, VEC, kOther, false, PAD, QU>(colidx2, m2, tail4b, colidx2, sx, ex,
                                                    nullptr, x, 0, r.w, pn, r.y, r.z, prm, sh,
                                                    tl, c, tri);
      block_pass<true, VEC, kSame, false, PAD, QU>(colidx2, m2, tail4b, colidx2, gx, sx,
                                                   nullptr, x, 0, r.w, pn, r.x, r.y, prm, sh,
                                                   tl, c, tri);
    }
  } else if (ex - gx <= prm.chunk) {
    block_pass<false, VEC, kMember, false, PAD, QU, ST, kFence>(
        colidx2, m2, tail4b, colidx2, gx, ex, nullptr, x, 0, ST ? r.y : r.w, pn, r.x, r.z, prm,
        sh, tl, c, nullptr);
  } else {
    if (use_bitmap(colidx2, sx, ex, prm.chunk))
      block_pass<false, VEC, kOther, true, PAD, QU, false, kFence>(colidx2, m2, tail4b, colidx2, sx, ex, nullptr,
                                                    x, 0, r.w, pn, r.y, r.z, prm, sh, tl, c,
                                                    nullptr);
    else
      block_pass<false, VEC, kOther, false, PAD, QU, false, kFence>(colidx2, m2, tail4b, colidx2, sx, ex, nullptr,
                                                     x, 0, r.w, pn, r.y, r.z, prm, sh, tl, c,
                                                     nullptr);
    if (use_bitmap(colidx2, gx, sx, prm.chunk))
      block_pass<false, VEC, kSame, true, PAD, QU, false, kFence>(colidx2, m2, tail4b, colidx2, gx, sx, nullptr,
                                                   x, 0, r.w, pn, r.x, r.y, prm, sh, tl, c,
                                                   nullptr);
    else
      block_pass<false, VEC, kSame, false, PAD, QU, false, kFence>(colidx2, m2, tail4b, colidx2, gx, sx, nullptr,
                                                    x, 0, r.w, pn, r.x, r.y, prm, sh, tl, c,
                                                    nullptr);
  }
}

// ---- level split of one row ------------------------------------------------------------
// The row of v (vx = vinfo[v]) at absolute offset lo is rewritten in colidx2 as
// [neighbours on v's level, ascending | the others, ascending], and the partners
// (same-level neighbours of smaller (degree class, ID) key) go to hadj from lo on.
constexpr u32 kSplitLane = 32;     // rows up to this length are split by one lane
constexpr u32 kSplitWave = 4096;   // rows up to this length by one wavefront; longer rows
                                   // by a whole workgroup (k_split_long)
constexpr u32 kSplitUnroll = 4;    // 64-entry steps per wavefront iteration

// Partition step over entries j0 .. j0 + 64 kSplitUnroll of the row at `lo` (d entries):
// counts (COUNT) or writes (!COUNT) the same-level entries, the other-level entries and
// the partners, advancing the running counts cs / co / ch, and cl, the same-level entries
// below v.
template <bool COUNT>
__device__ __forceinline__ void split_steps(const u32* __restrict__ colidx,
                                            const uint8_t* __restrict__ vinfo, u32 v, u32 vx,
                                            u32 lo, u32 j0, u32 jend, u32 same_base,
                                            u32 other_base, u32 part_base,
                                            u32* __restrict__ colidx2, u32* __restrict__ hadj,
                                            u32& cs, u32& co, u32& ch, u32& cl) {
  const u32 lane = lane_id();
  u32 w[kSplitUnroll], vw[kSplitUnroll];
#pragma unroll
  for (u32 u = 0; u < kSplitUnroll; ++u) {
    const u32 j = j0 + u * kWave + lane;
    w[u] = j < jend ? colidx[lo + j] : v;
  }
#pragma unroll
  for (u32 u = 0; u < kSplitUnroll; ++u) vw[u] = vinfo[w[u]];
#pragma unroll
  for (u32 u = 0; u < kSplitUnroll; ++u) {
    const u32 j = j0 + u * kWave + lane;
    const bool in = j < jend;
    const bool same = in && ((vw[u] ^ vx) & 0x80u) == 0;
    const bool part = same && key_less(vw[u] & 127u, w[u], vx & 127u, v);
    const u64 ms = __ballot(same), mo = __ballot(in && !same), mh = __ballot(part);
    if (!COUNT) {
      if (same) colidx2[lo + same_base + cs + mask_rank(ms)] = w[u];
      else if (in) colidx2[lo + other_base + co + mask_rank(mo)] = w[u];
      if (part) hadj[lo + part_base + ch + mask_rank(mh)] = w[u];
    }
    cs += (u32)__popcll(ms);
    co += (u32)__popcll(mo);
    ch += (u32)__popcll(mh);
    cl += (u32)__popcll(__ballot(same && w[u] < v));
  }
}

// A row of at most kSplitLane entries, by one lane, held in registers: every entry is
// loaded before the first vinfo gather and the same-level and partner flags are kept as
// bit masks, so the row costs one load and one gather round trip.  more[b]
// (wavefront-uniform) says whether any lane's row is longer than 8 b entries; blocks of
// 8 past every lane's row are skipped.  Returns the number of same-level entries in *ns,
// of partners in *nh and of same-level entries below v in *sr.
__device__ __forceinline__ void split_short_row(const u32* __restrict__ colidx,
                                                const uint8_t* __restrict__ vinfo, u32 v, u32 vx,
                                                u32 lo, u32 d, const bool* more,
                                                u32* __restrict__ colidx2,
                                                u32* __restrict__ hadj, u32* ns_out,
                                                u32* nh_out, u32* sr_out) {
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
  u32 sm = 0, pm = 0, lm = 0;  // same level, partner of v, same level below v
#pragma unroll
  for (u32 b = 0; b < NB; ++b) {
    if (more[b]) {
#pragma unroll
      for (u32 i = 0; i < B; ++i) {
        const u32 j = b * B + i;
        const u32 vw = vinfo[w[j]];
        const bool same = j < d && ((vw ^ vx) & 0x80u) == 0;
        sm |= (same ? 1u : 0u) << j;
        pm |= (same && key_less(vw & 127u, w[j], vx & 127u, v) ? 1u : 0u) << j;
        lm |= (same && w[j] < v ? 1u : 0u) << j;
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
  *sr_out = (u32)__popc(lm);
}

// A row of at most GL * U entries by one group of GL lanes (64 / GL rows per wavefront),
// held in registers: lane gl of the group holds entries GL u + gl, u < U, so the row
// costs one load and one gather round trip; the level, partner and below-v flags are kept
// as bit masks per lane and ranked by the group's bits of each ballot.  All 64 lanes call
// it together; a group without a row passes d = 0.  Returns the row's same-level entries
// in *ns, partners in *nh and same-level entries below v in *sr (on every lane of the
// group).
constexpr u32 kSplitGroup = 64;  // rows up to this length: 16-lane groups, 4 entries each

template <u32 GL, u32 U>
__device__ __forceinline__ void split_group_row(const u32* __restrict__ colidx,
                                                const uint8_t* __restrict__ vinfo, u32 v, u32 vx,
                                                u32 lo, u32 d, u32* __restrict__ colidx2,
                                                u32* __restrict__ hadj, u32* ns_out,
                                                u32* nh_out, u32* sr_out) {
  static_assert(GL == 16 || GL == 32, "groups of 16 or 32 lanes");
  static_assert(U <= 32, "flags are one 32-bit mask per lane");
  constexpr u64 gm = (1ull << GL) - 1ull;
  const u32 lane = lane_id(), gl = lane & (GL - 1u), gb = lane & ~(GL - 1u);
  const u64 below = (1ull << gl) - 1ull;
  u32 w[U];
#pragma unroll
  for (u32 u = 0; u < U; ++u) {
    const u32 j = u * GL + gl;
    w[u] = j < d ? colidx[lo + j] : v;
  }
  u32 sm = 0, pm = 0, lm = 0, im = 0;  // same level, partner, same level below v, in row
#pragma unroll
  for (u32 u = 0; u < U; ++u) {
    const u32 j = u * GL + gl;
    const u32 vw = vinfo[w[u]];
    const bool in = j < d;
    const bool same = in && ((vw ^ vx) & 0x80u) == 0;
    sm |= (same ? 1u : 0u) << u;
    pm |= (same && key_less(vw & 127u, w[u], vx & 127u, v) ? 1u : 0u) << u;
    lm |= (same && w[u] < v ? 1u : 0u) << u;
    im |= (in ? 1u : 0u) << u;
  }
  u32 ns = 0, nh = 0, sr = 0;
#pragma unroll
  for (u32 u = 0; u < U; ++u) {
    ns += (u32)__popcll((__ballot((sm >> u) & 1u) >> gb) & gm);
    nh += (u32)__popcll((__ballot((pm >> u) & 1u) >> gb) & gm);
    sr += (u32)__popcll((__ballot((lm >> u) & 1u) >> gb) & gm);
  }
  u32 cs = 0, co = 0, ch = 0;
#pragma unroll
  for (u32 u = 0; u < U; ++u) {
    const bool same = (sm >> u) & 1u, other = ((im & ~sm) >> u) & 1u, part = (pm >> u) & 1u;
    const u64 ms = (__ballot(same) >> gb) & gm, mo = (__ballot(other) >> gb) & gm;
    const u64 mp = (__ballot(part) >> gb) & gm;
    if (same) colidx2[lo + cs + (u32)__popcll(ms & below)] = w[u];
    else if (other) colidx2[lo + ns + co + (u32)__popcll(mo & below)] = w[u];
    if (part) hadj[lo + ch + (u32)__popcll(mp & below)] = w[u];
    cs += (u32)__popcll(ms);
    co += (u32)__popcll(mo);
    ch += (u32)__popcll(mp);
  }
  *ns_out = ns;
  *nh_out = nh;
  *sr_out = sr;
}

// A row of kSplitLane < d <= kSplitReg entries by one wavefront, held in registers (lane l
// holds entries 64 u + l): one load and one gather round trip, then the ballot-ranked
// writes.  Returns the number of same-level entries in *ns, of partners in *nh and of
// same-level entries below v in *sr.
constexpr u32 kSplitRegU = 16;
constexpr u32 kSplitReg = kSplitRegU * kWave;

__device__ __forceinline__ void split_wave_row(const u32* __restrict__ colidx,
                                               const uint8_t* __restrict__ vinfo, u32 v, u32 vx,
                                               u32 lo, u32 d, u32* __restrict__ colidx2,
                                               u32* __restrict__ hadj, u32* ns_out,
                                               u32* nh_out, u32* sr_out) {
  constexpr u32 U = kSplitRegU;
  const u32 lane = lane_id();
  const u32 nu = (d + kWave - 1) / kWave;  // wavefront-uniform
  u32 w[U];
#pragma unroll
  for (u32 u = 0; u < U; ++u) {
    if (u < nu) {
      const u32 j = u * kWave + lane;
      w[u] = j < d ? colidx[lo + j] : v;
    }
  }
  u32 sm = 0, pm = 0, lm = 0;
#pragma unroll
  for (u32 u = 0; u < U; ++u) {
    if (u < nu) {
      const u32 j = u * kWave + lane;
      const u32 vw = vinfo[w[u]];
      const bool same = j < d && ((vw ^ vx) & 0x80u) == 0;
      sm |= (same ? 1u : 0u) << u;
      pm |= (same && key_less(vw & 127u, w[u], vx & 127u, v) ? 1u : 0u) << u;
      lm |= (same && w[u] < v ? 1u : 0u) << u;
    }
  }
  u32 ns = 0, sr = 0;
#pragma unroll
  for (u32 u = 0; u < U; ++u) {
    if (u < nu) {
      ns += (u32)__popcll(__ballot((sm >> u) & 1u));
      sr += (u32)__popcll(__ballot((lm >> u) & 1u));
    }
  }
  u32 cs = 0, co = 0, ch = 0;
#pragma unroll
  for (u32 u = 0; u < U; ++u) {
    if (u < nu) {
      const bool in = u * kWave + lane < d;
      const bool same = (sm >> u) & 1u, part = (pm >> u) & 1u;
      const u64 ms = __ballot(same), mo = __ballot(in && !same), mh = __ballot(part);
      if (same) colidx2[lo + cs + mask_rank(ms)] = w[u];
      else if (in) colidx2[lo + ns + co + mask_rank(mo)] = w[u];
      if (part) hadj[lo + ch + mask_rank(mh)] = w[u];
      cs += (u32)__popcll(ms);
      co += (u32)__popcll(mo);
      ch += (u32)__popcll(mh);
    }
  }
  *ns_out = ns;
  *nh_out = ch;
  *sr_out = sr;
}

}  // namespace tc

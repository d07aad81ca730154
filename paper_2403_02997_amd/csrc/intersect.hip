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
#include "tc_device.h"
#include "tc_launch.h"

namespace tc {

static inline u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }

constexpr int kWaveSlots = 2048;   // LDS hash slots per wavefront (d(x) <= 512)
constexpr int kIsectThreads = 256;
constexpr int kUnroll = 4;         // independent list loads in flight per lane
static_assert(kUnroll == 4, "the wavefront kernel packs one mark byte per window in a word");
constexpr u32 kWaveClaim = 16;     // wavefront-class vertices claimed per counter atomic

// ---- lane class: one thread per cover edge ---------------------------------------------
template <bool PV>
__global__ void __launch_bounds__(kTileThreads) k_isect_lane(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx,
    const uint8_t* __restrict__ vinfo, const u32* __restrict__ hcnt, const u32* __restrict__ hadj,
    const u32* __restrict__ lane_x, u32 nlx, u64* __restrict__ ctr, u64* __restrict__ tri) {
  __shared__ u64 s_red[5 * (kTileThreads / kWave)];
  Counts c{0, 0, 0, 0, 0};
  const u32 stride = gridDim.x * blockDim.x;
  for (u32 t = blockIdx.x * blockDim.x + threadIdx.x; t < nlx; t += stride) {
    const u32 x = lane_x[t];
    const u32 bx = rowptr[x], ex = rowptr[x + 1], np = hcnt[x];
    const u32 px = vinfo[x] & 0x80u;
    for (u32 q = 0; q < np; ++q) {
      const u32 y = hadj[bx + q];
      u32 i = bx, j = rowptr[y];
      const u32 je = rowptr[y + 1];
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
            count_hit<PV>(r, a, x, y, vmax, c, tri);
            if (++i == ex || ++j == je) break;
            a = colidx[i];
            b = colidx[j];
          }
        }
      }
    }
  }
  block_flush_counts(c, 0, ctr, s_red);
}

// ---- wave class: one wavefront per staged vertex x ---------------------------------------
// N(x) goes to a per-wavefront LDS hash set.  The partners' lists are taken 64 at a time,
// padded out to whole 16-byte quads (VEC) and concatenated; each lane then loads one quad
// per window, so a lane has 4 * kUnroll list elements in flight.  The partner of a quad
// comes from the partners' quad ends: those inside the current windows mark their
// positions in LDS, and a ballot plus a population count gives every lane its partner.
template <bool PV, bool VEC>
__global__ void __launch_bounds__(kIsectThreads) k_isect_wave(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx, u32 m,
    const u32* __restrict__ tail4, const uint8_t* __restrict__ vinfo,
    const u32* __restrict__ hcnt, const u32* __restrict__ hadj, const u32* __restrict__ wave_x,
    u32 nwx, Plan* __restrict__ plan, u64* __restrict__ ctr, u64* __restrict__ tri) {
  constexpr int kW = kIsectThreads / kWave;
  constexpr u32 NE = VEC ? 4 : 1;  // elements per quad
  __shared__ __align__(16) u32 s_table[kW][kWaveSlots];
  __shared__ uint4 s_pinfo[kW][kWave];  // {quad base, lo, hi, y} of each compacted partner
  __shared__ u32 s_end[kW][kWave];
  __shared__ u32 s_mark[kW][kWave];
  __shared__ u64 s_red[5 * kW];
  const u32 wid = threadIdx.x / kWave, lane = lane_id();
  u32* table = s_table[wid];
  const u64 le = lane == kWave - 1 ? ~0ull : (2ull << lane) - 1;
  Counts c{0, 0, 0, 0, 0};
  // Vertices are claimed kWaveClaim at a time: one counter atomic per vertex would
  // serialise hundreds of thousands of same-address atomics at the L2.
  u32 idx = 0, idx_end = 0;
  while (true) {
    if (idx == idx_end) {
      u32 c0 = 0;
      if (lane == 0) c0 = atomicAdd(&plan->next_wave, kWaveClaim);
      idx = __shfl(c0, 0, kWave);
      idx_end = min(idx + kWaveClaim, nwx);
    }
    if (idx >= nwx) break;
    const u32 x = wave_x[idx++];
    const u32 bx = rowptr[x], dx = rowptr[x + 1] - bx;
    const u32 hs = bx, np = hcnt[x];  // H+(x) sits in place of N(x)
    const u32 px = vinfo[x] & 0x80u;
    const u32 mask = bucket_mask(dx, kWaveSlots);
    c.staged += lane == 0 ? dx : 0;
    for (u32 i = lane; i < (mask + 1) * 4; i += kWave) table[i] = kInf;
    wave_lds_sync();
    for (u32 i = lane; i < dx; i += kWave) {
      const u32 w = colidx[bx + i];
      const u32 same = ((vinfo[w] & 0x80u) == px) ? 1u : 0u;
      hash_insert(table, mask, w, same);
    }
    wave_lds_sync();
    Tally tl{0, 0, 0, 0};
    for (u32 pb = 0; pb < np; pb += kWave) {
      const u32 p = pb + lane;
      u32 y = 0, lo = 0, hi = 0;
      if (p < np) {
        y = hadj[hs + p];
        lo = rowptr[y];
        hi = rowptr[y + 1];
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
        s_pinfo[wid][r] = make_uint4((VEC ? qa >> 2 : qa) - (incl - nq), lo, hi, y);
        s_end[wid][r] = incl;
      }
      wave_lds_sync();
      const u32 my_end = lane < npc ? s_end[wid][lane] : kInf;  // quad end of partner `lane`
      for (u32 k0 = 0; k0 < total; k0 += kWave * kUnroll) {
        // Quad q belongs to partner #{r : end_r <= q}.  Partner ends strictly inside one
        // of the kUnroll windows of 64 quads from k0 mark their position (byte u of word
        // j for position 64 u + j); ends at a window start count in that window's base.
        s_mark[wid][lane] = 0;
        wave_lds_sync();
        const u32 t = my_end - k0;
        if (my_end > k0 && t < kWave * kUnroll && (t & (kWave - 1)) != 0)
          reinterpret_cast<uint8_t*>(s_mark[wid])[(t & (kWave - 1)) * 4 + t / kWave] = 1;
        wave_lds_sync();
        const u32 word = s_mark[wid][lane];
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
          inf[u] = s_pinfo[wid][l];
          addr[u] = (inf[u].x + q) * NE;
          if (VEC) {
            // one unconditional 16-byte load: a quad that would run past the end of
            // colidx (or a dead lane) reads the padded copy of the last partial quad
            const u32* src = (live[u] && addr[u] + 3 < m) ? colidx + addr[u] : tail4;
            const uint4 v = *reinterpret_cast<const uint4*>(src);
            e[u][0] = v.x;
            e[u][NE > 1 ? 1 : 0] = v.y;
            e[u][NE > 2 ? 2 : 0] = v.z;
            e[u][NE > 3 ? 3 : 0] = v.w;
          } else {
            e[u][0] = colidx[live[u] ? addr[u] : 0u];
          }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const u32 y2 = inf[u].w;
          const u32 vmax = max(x, y2);
          const u32 span = inf[u].z - inf[u].y;  // elements lo .. hi-1 are valid
          bool ok[NE];
#pragma unroll
          for (u32 i = 0; i < NE; ++i) ok[i] = live[u] && (addr[u] + i - inf[u].y) < span;
          u32 res[NE];
          hash_probe_n<NE>(table, mask, e[u], ok, res);
#pragma unroll
          for (u32 i = 0; i < NE; ++i) {
            tl.add(res[i], e[u][i], vmax);
            if (PV) attribute(tri, res[i], e[u][i], x, y2, vmax);
          }
        }
      }
      wave_lds_sync();
    }
    tl.fold(c);
  }
  block_flush_counts(c, 1, ctr, s_red);
}

// ---- block class: one 1024-thread workgroup per (x, segment of partners) ----------------
// N(x) is staged chunk by chunk (at most prm.chunk <= 16384 entries per chunk, 4096 by
// default so that the 128 KB LDS hash set stays at most 1/8 full).  For each chunk every
// partner list is cut at the chunk's largest ID (one binary search from the previous
// chunk's cut, only when N(x) needs several chunks) and padded out to whole 16-byte quads; the concatenated quad space is split into one contiguous range per
// wavefront.  A wavefront walks its range in windows of 64 quads, one quad (16-byte load)
// per lane, and keeps the current partner as it goes: the partner boundaries (quad prefix
// sums in LDS) that fall inside a window are applied with a few lane-uniform steps, so
// no per-lane search is needed.  Every partner element is probed exactly once, against
// the first chunk whose largest ID is not below it.
constexpr int kBigThreads = 1024;
constexpr int kBigWaves = kBigThreads / kWave;
constexpr int kBigSlots = 32768;   // 128 KB of LDS
constexpr int kBigSeg = 1024;      // partners per work item (one per thread for set-up)
constexpr int kQuadUnroll = 4;     // windows per wavefront loaded before probing

// What one pass of the workgroup kernel stages, streams and tallies:
//   kFull     : N(x) with level flags; each partner's whole list; c1, c2 and t2
//               (diagnostics and per-vertex counts);
//   kPrunedOne: N(x) with level flags in one chunk; each partner's same-level
//               neighbours above max(x, y) and its other-level ones (one contiguous
//               range of the level-split rows); c1 and t2;
//   kOther    : the other-level part of N(x); each partner's other-level part; c1;
//   kSame     : the same-level part of N(x) above x; each partner's same-level part
//               above max(x, y); t2 (every hit is a same-level apex above both ends).
// A same-level apex w <= max(x, y) is never counted (the apex rule), so the pruned
// passes skip those list entries entirely and leave c2 uncounted.
enum BlockMode { kFull = 0, kPrunedOne = 1, kOther = 2, kSame = 3 };

struct BlockShared {
  u32* table;
  u32* qincl;
  uint4* pinfo;
  u32* tmp;
};

// One pass over the partners of a work item.  The staged keys ga[gs .. ge) (ascending)
// go to LDS either as hash sets of at most prm.chunk keys (BM = false) or, for the
// level-specific pruned passes, as bitmaps of one 2^kWinBits-ID window each (BM = true,
// one bit per ID: these passes need membership only).  Partner `tid` < pn streams
// sa[plo .. phi), cut at each chunk's largest ID or window end.  All threads of the
// workgroup call it together.
constexpr u32 kWinBits = 20;  // 2^20 IDs per bitmap window = 128 KB of LDS

template <bool PV, bool VEC, int MODE, bool BM>
__device__ __forceinline__ void block_pass(
    const u32* __restrict__ sa, u32 m, const u32* __restrict__ st4, const u32* __restrict__ ga,
    u32 gs, u32 ge, const uint8_t* __restrict__ vinfo, u32 x, u32 px, u32 y, u32 pn, u32 plo,
    u32 phi, IsectParams prm, const BlockShared& sh, Tally& tl, Counts& c, u64* __restrict__ tri) {
  constexpr u32 NE = VEC ? 4 : 1;  // elements per quad (a quad is one element without VEC)
  const u32 tid = threadIdx.x, lane = lane_id(), wid = tid / kWave;
  static_assert(!BM || MODE == kOther || MODE == kSame, "bitmaps hold membership only");
  const u32 glen = ge - gs;
  // hash chunks by count, or bitmap windows by ID
  const u32 w_first = BM && glen ? ga[gs] >> kWinBits : 0u;
  const u32 nch = BM ? (glen ? (ga[ge - 1] >> kWinBits) - w_first + 1 : 0u)
                     : (glen + prm.chunk - 1) / prm.chunk;
  u32 lo = plo;  // cursor: elements below it were probed against earlier chunks
  u32 c0 = gs;   // first staged key of the chunk
  for (u32 ch = 0; ch < nch; ++ch) {
    const u32 wb = (w_first + ch) << kWinBits;  // BM: window [wb, wb + 2^kWinBits)
    u32 clen;
    if (BM) {
      clen = lower_bound_g(ga, c0, ge, wb + (1u << kWinBits)) - c0;
      if (clen == 0) continue;  // no staged key in this window (uniform)
    } else {
      clen = min(prm.chunk, ge - c0);
    }
    const u32 mask = BM ? 0u : bucket_mask(clen, kBigSlots);
    c.staged += tid == 0 ? clen : 0;
    if (BM) {
      uint4* t4 = reinterpret_cast<uint4*>(sh.table);
      for (u32 i = tid; i < (u32)kBigSlots / 4; i += blockDim.x) t4[i] = make_uint4(0, 0, 0, 0);
    } else {
      for (u32 i = tid; i < (mask + 1) * 4; i += blockDim.x) sh.table[i] = kInf;
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
        const u32 same = (MODE == kFull || MODE == kPrunedOne) && (vinfo[w] & 0x80u) == px;
        hash_insert(sh.table, mask, w, same ? 1u : 0u);
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
    for (u32 qw = qs; qw < qe; qw += kWave * kQuadUnroll) {
      u32 e[kQuadUnroll][NE];
      uint4 inf[kQuadUnroll];
      u32 addr[kQuadUnroll];
      bool live[kQuadUnroll];
#pragma unroll
      for (int u = 0; u < kQuadUnroll; ++u) {
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
        inf[u] = sh.pinfo[p];
        addr[u] = (inf[u].x + q) * NE;
        if (VEC) {
          // one unconditional 16-byte load: a quad that would run past the end of the
          // streamed array (or a dead lane) reads the padded copy of its last partial quad
          const u32* src = (live[u] && addr[u] + 3 < m) ? sa + addr[u] : st4;
          const uint4 v = *reinterpret_cast<const uint4*>(src);
          e[u][0] = v.x;
          e[u][NE > 1 ? 1 : 0] = v.y;
          e[u][NE > 2 ? 2 : 0] = v.z;
          e[u][NE > 3 ? 3 : 0] = v.w;
        } else {
          e[u][0] = sa[live[u] ? addr[u] : 0u];
        }
      }
#pragma unroll
      for (int u = 0; u < kQuadUnroll; ++u) {
        const u32 y2 = inf[u].w;
        const u32 vmax = max(x, y2);
        const u32 span = inf[u].z - inf[u].y;  // elements lo .. hi-1 are valid
        bool ok[NE];
#pragma unroll
        for (u32 i = 0; i < NE; ++i) ok[i] = live[u] && (addr[u] + i - inf[u].y) < span;
        u32 res[NE];
        if (BM) {
          // elements of earlier, skipped windows fall outside [wb, wb + 2^kWinBits)
#pragma unroll
          for (u32 i = 0; i < NE; ++i) {
            const u32 k = e[u][i] - wb;
            const bool in = ok[i] && k < (1u << kWinBits);
            const u32 kk = in ? k : 0u;
            res[i] = in ? (sh.table[kk >> 5] >> (kk & 31u)) & 1u : 0u;
          }
        } else {
          hash_probe_n<NE>(sh.table, mask, e[u], ok, res);
        }
#pragma unroll
        for (u32 i = 0; i < NE; ++i) {
          if (MODE == kFull) {
            tl.add(res[i], e[u][i], vmax);
            if (PV) attribute(tri, res[i], e[u][i], x, y2, vmax);
          } else if (MODE == kPrunedOne) {
            tl.s += res[i] & 1u;  // other-level apex (c1)
            tl.t2 += res[i] >> 1;  // same-level apex above both endpoints
          } else if (MODE == kOther) {
            tl.s += res[i];
          } else {
            tl.t2 += res[i];
          }
        }
      }
    }
    __syncthreads();
    lo = hi;
    c0 += clen;
  }
}

// Bitmap windows for the sorted keys a[s .. e) when they take fewer passes than hash
// chunks of `chunk` keys.
__device__ __forceinline__ bool use_bitmap(const u32* __restrict__ a, u32 s, u32 e, u32 chunk) {
  if (e - s <= chunk) return false;
  const u32 wins = (a[e - 1] >> kWinBits) - (a[s] >> kWinBits) + 1;
  return wins < (e - s + chunk - 1) / chunk;
}

// PRUNED = false: kFull pass over colidx.  PRUNED = true: the level-split rows colidx2
// (split[v] = start of v's other-level neighbours), one kPrunedOne pass when N(x) fits
// one chunk, else a kOther and a kSame pass.
template <bool PV, bool VEC, bool PRUNED>
__global__ void __launch_bounds__(kBigThreads) k_isect_block(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx, u32 m,
    const u32* __restrict__ tail4, const u32* __restrict__ colidx2,
    const u32* __restrict__ split, const u32* __restrict__ tail4b,
    const uint8_t* __restrict__ vinfo, const u32* __restrict__ hcnt, const u32* __restrict__ hadj,
    const Item* __restrict__ items, u32 nitems, IsectParams prm, Plan* __restrict__ plan,
    u64* __restrict__ ctr, u64* __restrict__ tri) {
  __shared__ __align__(16) u32 s_table[kBigSlots];
  __shared__ u32 s_qincl[kBigSeg];
  __shared__ uint4 s_pinfo[kBigSeg];  // {quad base, lo, hi, y} of each partner
  __shared__ u32 s_tmp[kBigWaves];
  __shared__ u64 s_red[5 * kBigWaves];
  __shared__ u32 s_item;
  const BlockShared sh{s_table, s_qincl, s_pinfo, s_tmp};
  const u32 tid = threadIdx.x;
  Counts c{0, 0, 0, 0, 0};
  Tally tl{0, 0, 0, 0};
  while (true) {
    if (tid == 0) s_item = atomicAdd(&plan->next_item, 1u);
    __syncthreads();
    const u32 it = s_item;
    if (it >= nitems) break;
    const Item item = items[it];
    const u32 x = item.x;
    const u32 bx = rowptr[x], ex = rowptr[x + 1], dx = ex - bx;
    const u32 px = vinfo[x] & 0x80u;
    const u32 hs = bx + item.seg * prm.seg;  // H+(x) sits in place of N(x)
    const u32 pn = min(prm.seg, hcnt[x] - item.seg * prm.seg);
    u32 y = 0, yr = 0, ye = 0;
    if (tid < pn) {
      y = hadj[hs + tid];
      yr = rowptr[y];
      ye = rowptr[y + 1];
    }
    if (!PRUNED) {
      block_pass<PV, VEC, kFull, false>(colidx, m, tail4, colidx, bx, ex, vinfo, x, px, y, pn, yr,
                                        ye, prm, sh, tl, c, tri);
    } else {
      u32 ys = 0, lb = 0;
      if (tid < pn) {
        ys = split[y];
        lb = lower_bound_g(colidx2, yr, ys, max(x, y) + 1u);  // same-level part above max
      }
      if (dx <= prm.chunk) {
        block_pass<false, VEC, kPrunedOne, false>(colidx2, m, tail4b, colidx, bx, ex, vinfo, x, px,
                                                  y, pn, lb, ye, prm, sh, tl, c, tri);
      } else {
        const u32 sx = split[x];
        const u32 gx = lower_bound_g(colidx2, bx, sx, x + 1u);  // same-level part above x
        // bitmap windows where they need fewer passes than hash chunks
        if (use_bitmap(colidx2, sx, ex, prm.chunk))
          block_pass<false, VEC, kOther, true>(colidx2, m, tail4b, colidx2, sx, ex, vinfo, x, px, y,
                                               pn, ys, ye, prm, sh, tl, c, tri);
        else
          block_pass<false, VEC, kOther, false>(colidx2, m, tail4b, colidx2, sx, ex, vinfo, x, px,
                                                y, pn, ys, ye, prm, sh, tl, c, tri);
        if (use_bitmap(colidx2, gx, sx, prm.chunk))
          block_pass<false, VEC, kSame, true>(colidx2, m, tail4b, colidx2, gx, sx, vinfo, x, px, y,
                                              pn, lb, ys, prm, sh, tl, c, tri);
        else
          block_pass<false, VEC, kSame, false>(colidx2, m, tail4b, colidx2, gx, sx, vinfo, x, px, y,
                                               pn, lb, ys, prm, sh, tl, c, tri);
      }
    }
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
                       const u32* hcnt, const u32* hadj, const u32* lane_x, u32 nlx, u64* ctr,
                       u64* tri, hipStream_t s) {
  if (nlx == 0) return;
  const u32 g = min(cdiv(nlx, kTileThreads), resident_blocks(8));
  if (tri)
    hipLaunchKernelGGL(k_isect_lane<true>, dim3(g), dim3(kTileThreads), 0, s, rowptr, colidx,
                       vinfo, hcnt, hadj, lane_x, nlx, ctr, tri);
  else
    hipLaunchKernelGGL(k_isect_lane<false>, dim3(g), dim3(kTileThreads), 0, s, rowptr, colidx,
                       vinfo, hcnt, hadj, lane_x, nlx, ctr, tri);
}

void launch_isect_wave(const u32* rowptr, const u32* colidx, u32 m, const u32* tail4,
                       const uint8_t* vinfo, const u32* hcnt, const u32* hadj, const u32* wave_x,
                       u32 nwx, Plan* plan, u64* ctr, u64* tri, hipStream_t s) {
  if (nwx == 0) return;
  const u32 g = min(cdiv(nwx, kIsectThreads / kWave), resident_blocks(8));
  const bool vec = ((uintptr_t)colidx & 15u) == 0;
#define TC_LAUNCH_WAVE(PV, VEC)                                                                \
  hipLaunchKernelGGL((k_isect_wave<PV, VEC>), dim3(g), dim3(kIsectThreads), 0, s, rowptr,       \
                     colidx, m, tail4, vinfo, hcnt, hadj, wave_x, nwx, plan, ctr, tri)
  if (tri) {
    if (vec) TC_LAUNCH_WAVE(true, true);
    else TC_LAUNCH_WAVE(true, false);
  } else {
    if (vec) TC_LAUNCH_WAVE(false, true);
    else TC_LAUNCH_WAVE(false, false);
  }
#undef TC_LAUNCH_WAVE
}

void launch_isect_block(const u32* rowptr, const u32* colidx, u32 m, const u32* tail4,
                        const u32* colidx2, const u32* split, const u32* tail4b,
                        const uint8_t* vinfo, const u32* hcnt, const u32* hadj, const Item* items,
                        u32 nitems, IsectParams p, Plan* plan, u64* ctr, u64* tri, bool pruned,
                        hipStream_t s) {
  if (nitems == 0) return;
  const u32 g = min(nitems, resident_blocks(1));
  const bool vec = ((uintptr_t)colidx & 15u) == 0 && ((uintptr_t)colidx2 & 15u) == 0;
#define TC_LAUNCH_BLOCK(PV, VEC, PR)                                                           \
  hipLaunchKernelGGL((k_isect_block<PV, VEC, PR>), dim3(g), dim3(kBigThreads), 0, s, rowptr,    \
                     colidx, m, tail4, colidx2, split, tail4b, vinfo, hcnt, hadj, items, nitems, \
                     p, plan, ctr, tri)
  if (tri) {
    if (vec) TC_LAUNCH_BLOCK(true, true, false);
    else TC_LAUNCH_BLOCK(true, false, false);
  } else if (pruned) {
    if (vec) TC_LAUNCH_BLOCK(false, true, true);
    else TC_LAUNCH_BLOCK(false, false, true);
  } else {
    if (vec) TC_LAUNCH_BLOCK(false, true, false);
    else TC_LAUNCH_BLOCK(false, false, false);
  }
#undef TC_LAUNCH_BLOCK
}

void launch_finalize(const u64* ctr, u64* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, ctr, out);
}

}  // namespace tc

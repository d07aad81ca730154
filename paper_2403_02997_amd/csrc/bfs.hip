// Level-synchronous, direction-optimising BFS from every component root at once.
//
// The paper's CETC-Seq restarts BFS(G, v) from every unvisited vertex; with candidate
// roots taken in ascending ID, each component is searched from its smallest vertex ID.
// Components are disjoint, so one multi-source BFS seeded with all those roots at level
// 0 assigns every vertex exactly the distance to its own component's root.
//
// Each level is one launch of k_bfs_level.  The expansion direction follows Beamer,
// Asanović & Patterson (SC 2012): top-down while the frontier's edges m_f stay below
// m_u / 14 (m_u = edges of unvisited vertices), bottom-up until the frontier shrinks
// below n / 24.  The last block of each level takes that decision on the device, so the
// host enqueues many levels without waiting and only polls `done` between batches.
// Blocks leave their totals in their own slots of `part` and take one ticket atomic;
// the last block sums the slots with all its threads.
//
// Top-down levels expand the frontier queue, short lists per lane and lists of up to
// kBfsBig entries per wavefront; longer lists are also kept in a small queue of big
// vertices, whose lists every workgroup shares in kBfsChunk-entry pieces, so that one
// hub on the frontier does not leave its whole list to a single wavefront.  Bottom-up
// levels test the first four entries of every unvisited row together before any row
// goes on, so most vertices find their parent in two memory round trips.
// Each level's frontier is also kept as a bitmap (n bits, small enough to stay in the
// L2): bottom-up steps test neighbours against it instead of gathering their levels.
// Three bitmaps rotate: level k reads bitmap k mod 3, fills (k + 1) mod 3 and clears
// (k + 2) mod 3, the frontier of level k - 1, which level k + 1 fills next.
#include "tc_device.h"
#include "tc_launch.h"

namespace tc {

static inline u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }

constexpr int kBfsThreads = 256;
constexpr u32 kBfsLaneMax = 32;    // top-down: frontier lists up to this length per lane
constexpr u32 kBfsBig = 1024;      // top-down: longer frontier lists are shared by the grid
constexpr u32 kBfsChunk = 1024;    // entries of a big list per workgroup task
constexpr u32 kBfsVisit = 4;       // top-down: neighbours per lane claimed together
constexpr u32 kBfsPer = 8;         // vertices per thread and pass in the vertex sweeps
constexpr u32 kBfsBlocksPerCu = 2;

// Stores the frontier bits of 32 consecutive vertices v0 .. v0 + 31 handled by one half
// of a wavefront (v0 a multiple of 32), which no other thread writes in this sweep.
__device__ __forceinline__ void store_bits_half(u32* bm, u32 v, bool set, u32 n) {
  const u64 b = __ballot(set);
  const u32 lane = lane_id();
  if ((lane & 31u) == 0 && v < n) bm[v >> 5] = (u32)(b >> (lane & 32u));
}

__global__ void __launch_bounds__(kBfsThreads) k_bfs_init(const u32* __restrict__ rowptr,
                                                          const u32* __restrict__ parent, u32 n,
                                                          u32* __restrict__ level,
                                                          u32* __restrict__ queue0,
                                                          u32* __restrict__ bigq0,
                                                          u32* __restrict__ fb0,
                                                          BfsCtl* __restrict__ ctl, u32 keep) {
  __shared__ u32 s_tmp[kBfsThreads / kWave];
  __shared__ u32 s_base;
  u64 mu = 0;
  u32 roots = 0;
  const u32 span = kBfsPer * blockDim.x;
  for (u32 base = blockIdx.x * span; base < n; base += gridDim.x * span) {
    u32 bits = 0, cnt = 0;
#pragma unroll
    for (u32 k = 0; k < kBfsPer; ++k) {
      const u32 v = base + k * blockDim.x + threadIdx.x;
      if (v < n) {
        const u32 d = rowptr[v + 1] - rowptr[v];
        // keep: a vertex an earlier search reached keeps its level and takes no part
        const bool reached = keep && level[v] != kInf;
        const bool root = !reached && parent[v] == v;
        if (!reached) level[v] = root ? 0u : kInf;
        roots += root;
        if (!root && !reached) mu += d;
        if (root && d > 0) {
          bits |= 1u << k;
          ++cnt;
          if (d > kBfsBig) bigq0[atomicAdd(&ctl->bqlen[0], 1u)] = v;
        }
      }
      store_bits_half(fb0, v, (bits >> k) & 1u, n);
    }
    u32 tot;
    const u32 incl = block_incl_scan(cnt, s_tmp, &tot);
    if (threadIdx.x == 0) s_base = tot ? atomicAdd(&ctl->qlen[0], tot) : 0u;
    __syncthreads();
    u32 pos = s_base + incl - cnt;
#pragma unroll
    for (u32 k = 0; k < kBfsPer; ++k)
      if (bits & (1u << k)) queue0[pos++] = base + k * blockDim.x + threadIdx.x;
    __syncthreads();  // s_base is rewritten by the next pass
  }
  // one atomic per workgroup and counter
  __shared__ u64 s_mu[kBfsThreads / kWave];
  __shared__ u32 s_roots[kBfsThreads / kWave];
  mu = wave_sum_u64(mu);
  roots = wave_sum_u32(roots);
  if (lane_id() == 0) {
    s_mu[threadIdx.x / kWave] = mu;
    s_roots[threadIdx.x / kWave] = roots;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 a = 0;
    u32 b = 0;
    for (u32 w = 0; w < blockDim.x / kWave; ++w) {
      a += s_mu[w];
      b += s_roots[w];
    }
    if (a) atomicAdd((unsigned long long*)&ctl->mu, (unsigned long long)a);
    if (b) atomicAdd(&ctl->num_roots, b);
  }
}

// Claim y for level k+1 (top-down).  Returns true for exactly one claimant.
__device__ __forceinline__ bool bfs_claim(u32* level, u32 y, u32 next) {
  if (load_coherent(&level[y]) != kInf) return false;
  return atomicCAS(&level[y], kInf, next) == kInf;
}

// Where a level's output goes: the next frontier queue (and its length), the queue of
// big vertices among it, and the next frontier bitmap.
struct BfsOut {
  u32* q;
  u32* qlen;
  u32* bq;
  u32* bqlen;
  u32* bits;  // null: no frontier bitmap (persistent top-down levels)
};

// Top-down visit of the neighbours y[i] with act[i] of every lane; all lanes of the
// wavefront call it together.  Their level loads, then their claims, are issued
// together, and the claimed ones join the next frontier with one queue atomic per
// wavefront.
__device__ __forceinline__ void td_visit(const u32 (&y)[kBfsVisit], const bool (&act)[kBfsVisit],
                                         u32 next, const u32* __restrict__ rowptr,
                                         u32* __restrict__ level, const BfsOut& o, u64& mf,
                                         u64& mu_dec) {
  u32 lv[kBfsVisit];
#pragma unroll
  for (u32 i = 0; i < kBfsVisit; ++i) lv[i] = act[i] ? load_coherent(&level[y[i]]) : 0u;
  bool cl[kBfsVisit];
  u32 cnt = 0;
#pragma unroll
  for (u32 i = 0; i < kBfsVisit; ++i) {
    cl[i] = act[i] && lv[i] == kInf && atomicCAS(&level[y[i]], kInf, next) == kInf;
    cnt += cl[i] ? 1u : 0u;
  }
  const u32 incl = wave_incl_scan(cnt);
  const u32 total = __shfl(incl, kWave - 1, kWave);
  if (total == 0) return;  // uniform
  u32 base = 0;
  if (lane_id() == 0) base = atomicAdd(o.qlen, total);
  u32 pos = __shfl(base, 0, kWave) + incl - cnt;
#pragma unroll
  for (u32 i = 0; i < kBfsVisit; ++i) {
    if (cl[i]) {
      o.q[pos++] = y[i];
      if (o.bits) atomicOr(&o.bits[y[i] >> 5], 1u << (y[i] & 31));
      const u32 dy = rowptr[y[i] + 1] - rowptr[y[i]];
      mf += dy;
      mu_dec += dy;
      if (dy > kBfsBig) o.bq[atomicAdd(o.bqlen, 1u)] = y[i];
    }
  }
}

__global__ void __launch_bounds__(kBfsThreads) k_bfs_level(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx, u32 n, u32 k,
    u32* __restrict__ level, u32* __restrict__ queue0, u32* __restrict__ queue1,
    u32* __restrict__ bigq0, u32* __restrict__ bigq1, u32* __restrict__ fb,
    BfsCtl* __restrict__ ctl, u64* __restrict__ part) {
  __shared__ u64 s_red[2 * (kBfsThreads / kWave)];
  __shared__ bool s_last;
  if (load_coherent(&ctl->done)) return;  // uniform across the grid
  const u32 mode = load_coherent(&ctl->mode);
  const u32* qin = (k & 1) ? queue1 : queue0;
  const u32* bqin = (k & 1) ? bigq1 : bigq0;
  const u32 next = k + 1;
  const u32 nw = (n + 31) / 32;
  const u32* fcur = fb + (k % 3) * (size_t)nw;
  const BfsOut o{(k & 1) ? queue0 : queue1, &ctl->qlen[(k + 1) & 1], (k & 1) ? bigq0 : bigq1,
                 &ctl->bqlen[(k + 1) & 1], fb + ((k + 1) % 3) * (size_t)nw};
  u64 mf = 0, mu_dec = 0;
  const u32 lane = lane_id();
  const u32 stride = gridDim.x * blockDim.x;
  u32* fold = fb + ((k + 2) % 3) * (size_t)nw;
  for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += stride) fold[i] = 0;

  if (mode == 0) {
    // ---- top-down: expand the frontier queue ----
    const u32 qn = load_coherent(&ctl->qlen[k & 1]);
    const u32 qr = (qn + kWave - 1) / kWave * kWave;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < qr; i += stride) {
      u32 x = 0, lo = 0, d = 0;
      if (i < qn) {
        x = qin[i];
        lo = rowptr[x];
        d = rowptr[x + 1] - lo;
        if (d > kBfsBig) d = 0;  // shared by the grid below
      }
      const bool big = d > kBfsLaneMax;
      // small frontier vertices: each lane walks its own list in lockstep
      u32 dl = big ? 0 : d;
      u32 dmax = dl;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) dmax = max(dmax, (u32)__shfl_xor(dmax, off, kWave));
      for (u32 j = 0; j < dmax; j += kBfsVisit) {
        u32 y[kBfsVisit];
        bool act[kBfsVisit];
#pragma unroll
        for (u32 i = 0; i < kBfsVisit; ++i) {
          act[i] = j + i < dl;
          y[i] = act[i] ? colidx[lo + j + i] : 0u;
        }
        td_visit(y, act, next, rowptr, level, o, mf, mu_dec);
      }
      // larger frontier vertices: the whole wavefront strides each list
      u64 bigmask = __ballot(big);
      while (bigmask) {
        const int b = __ffsll((unsigned long long)bigmask) - 1;
        bigmask &= bigmask - 1;
        const u32 blo = __shfl(lo, b, kWave), bd = __shfl(d, b, kWave);
        for (u32 j0 = 0; j0 < bd; j0 += kWave * kBfsVisit) {
          u32 y[kBfsVisit];
          bool act[kBfsVisit];
#pragma unroll
          for (u32 i = 0; i < kBfsVisit; ++i) {
            const u32 j = j0 + i * kWave + lane;
            act[i] = j < bd;
            y[i] = act[i] ? colidx[blo + j] : 0u;
          }
          td_visit(y, act, next, rowptr, level, o, mf, mu_dec);
        }
      }
    }
    // big frontier vertices: piece c of the bi-th list goes to workgroup (c + 131 bi) % grid
    const u32 nb = load_coherent(&ctl->bqlen[k & 1]);
    for (u32 bi = 0; bi < nb; ++bi) {
      const u32 x = bqin[bi];
      const u32 lo = rowptr[x], d = rowptr[x + 1] - lo;
      const u32 nch = (d + kBfsChunk - 1) / kBfsChunk;
      const u32 shift = (u32)(((u64)bi * 131u) % gridDim.x);
      for (u32 c = (blockIdx.x + gridDim.x - shift) % gridDim.x; c < nch; c += gridDim.x) {
        const u32 ce = min(d, (c + 1) * kBfsChunk);
        for (u32 j0 = c * kBfsChunk; j0 < ce; j0 += blockDim.x * kBfsVisit) {
          u32 y[kBfsVisit];
          bool act[kBfsVisit];
#pragma unroll
          for (u32 i = 0; i < kBfsVisit; ++i) {
            const u32 j = j0 + i * blockDim.x + threadIdx.x;
            act[i] = j < ce;
            y[i] = act[i] ? colidx[lo + j] : 0u;
          }
          td_visit(y, act, next, rowptr, level, o, mf, mu_dec);
        }
      }
    }
  } else {
    // ---- bottom-up: every unvisited vertex looks for a neighbour on level k ----
    __shared__ u32 s_tmp[kBfsThreads / kWave];
    __shared__ u32 s_base;
    const u32 span = kBfsPer * blockDim.x;
    for (u32 base = blockIdx.x * span; base < n; base += gridDim.x * span) {
      u32 lo[kBfsPer], d[kBfsPer];
      u32 act = 0;  // bit kk: vertex kk is unvisited
#pragma unroll
      for (u32 kk = 0; kk < kBfsPer; ++kk) {
        const u32 v = base + kk * blockDim.x + threadIdx.x;
        lo[kk] = 0;
        d[kk] = 0;
        if (v < n) {
          const u32 lv = level[v];
          const u32 r0 = rowptr[v], r1 = rowptr[v + 1];
          if (lv == kInf) {
            act |= 1u << kk;
            lo[kk] = r0;
            d[kk] = r1 - r0;
          }
        }
      }
      // the first four entries of every unvisited row, all loaded before any test
      u32 w[kBfsPer][4];
#pragma unroll
      for (u32 kk = 0; kk < kBfsPer; ++kk)
#pragma unroll
        for (u32 i = 0; i < 4; ++i) w[kk][i] = i < d[kk] ? colidx[lo[kk] + i] : 0u;
      u32 found = 0;
#pragma unroll
      for (u32 kk = 0; kk < kBfsPer; ++kk) {
        bool f = false;
#pragma unroll
        for (u32 i = 0; i < 4; ++i)
          f |= i < d[kk] && ((fcur[w[kk][i] >> 5] >> (w[kk][i] & 31)) & 1u);
        found |= (f ? 1u : 0u) << kk;
      }
      u32 bits = 0, cnt = 0;
#pragma unroll
      for (u32 kk = 0; kk < kBfsPer; ++kk) {
        const u32 v = base + kk * blockDim.x + threadIdx.x;
        const u32 lk = lo[kk], dk = d[kk];
        bool fk = (found >> kk) & 1u;
        // the rest of a short row, four neighbours per step
        const bool big = dk > kBfsLaneMax;
        if (!big) {
          for (u32 j = 4; j < dk && !fk; j += 4) {
            u32 ww[4];
#pragma unroll
            for (u32 i = 0; i < 4; ++i) ww[i] = j + i < dk ? colidx[lk + j + i] : 0u;
#pragma unroll
            for (u32 i = 0; i < 4; ++i)
              fk |= j + i < dk && ((fcur[ww[i] >> 5] >> (ww[i] & 31)) & 1u);
          }
        }
        // the rest of a long row: the whole wavefront, 64 neighbours per step
        u64 bm = __ballot(big && !fk);
        while (bm) {
          const int b = __ffsll((unsigned long long)bm) - 1;
          bm &= bm - 1;
          const u32 blo = __shfl(lk, b, kWave), bd = __shfl(dk, b, kWave);
          bool bf = false;
          for (u32 j0 = 4; j0 < bd && !bf; j0 += kWave) {
            const u32 j = j0 + lane;
            bool hit = false;
            if (j < bd) {
              const u32 ww = colidx[blo + j];
              hit = (fcur[ww >> 5] >> (ww & 31)) & 1u;
            }
            bf = __ballot(hit) != 0;
          }
          if ((int)lane == b) fk = bf;
        }
        if (fk) {
          level[v] = next;
          bits |= 1u << kk;
          ++cnt;
          mf += dk;
          mu_dec += dk;
          if (dk > kBfsBig) o.bq[atomicAdd(o.bqlen, 1u)] = v;
        }
        store_bits_half(o.bits, v, fk, n);
      }
      u32 tot;
      const u32 incl = block_incl_scan(cnt, s_tmp, &tot);
      if (threadIdx.x == 0) s_base = tot ? atomicAdd(o.qlen, tot) : 0u;
      __syncthreads();
      u32 pos = s_base + incl - cnt;
#pragma unroll
      for (u32 kk = 0; kk < kBfsPer; ++kk)
        if (bits & (1u << kk)) o.q[pos++] = base + kk * blockDim.x + threadIdx.x;
      __syncthreads();  // s_base is rewritten by the next pass
    }
  }

  // ---- block totals, then the last block decides the next level ----
  mf = wave_sum_u64(mf);
  mu_dec = wave_sum_u64(mu_dec);
  const u32 wid = threadIdx.x / kWave;
  if (lane == 0) {
    s_red[2 * wid] = mf;
    s_red[2 * wid + 1] = mu_dec;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 a = 0, b = 0;
    for (u32 w = 0; w < blockDim.x / kWave; ++w) {
      a += s_red[2 * w];
      b += s_red[2 * w + 1];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
    __threadfence();
    const u32 ticket = atomicAdd(&ctl->blocks_done, 1u);
    s_last = ticket == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;  // uniform within the block
  __threadfence();
  u64 a = 0, b = 0;
  for (u32 i = threadIdx.x; i < gridDim.x; i += blockDim.x) {
    a += __hip_atomic_load(&part[2 * i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    b += __hip_atomic_load(&part[2 * i + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  a = wave_sum_u64(a);
  b = wave_sum_u64(b);
  if (lane == 0) {  // thread 0 read s_red before the last barrier
    s_red[2 * wid] = a;
    s_red[2 * wid + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 mfs = 0, dec = 0;
    for (u32 w = 0; w < blockDim.x / kWave; ++w) {
      mfs += s_red[2 * w];
      dec += s_red[2 * w + 1];
    }
    const u32 nf = __hip_atomic_load(o.qlen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const u64 mus = __hip_atomic_load(&ctl->mu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - dec;
    ctl->mu = mus;
    if (mode == 1) ctl->bu_levels += 1;
    if (nf == 0) {
      ctl->done = 1;
    } else {
      ctl->depth = next;
      u32 nm = mode;
      if (mode == 0 && mfs > mus / 14) nm = 1;
      else if (mode == 1 && (u64)nf * 24 < (u64)n) nm = 0;
      ctl->mode = nm;
    }
    // this level's input queues are the next level's output
    ctl->qlen[k & 1] = 0;
    ctl->bqlen[k & 1] = 0;
    ctl->blocks_done = 0;
    __threadfence();
  }
}

// ---- persistent top-down levels (long searches) -------------------------------------
// A search still running after the first batch of levels (a large diameter: grids,
// road-like graphs, paths) continues in one cooperative launch that runs consecutive
// top-down levels with a grid barrier between them, instead of one launch, one ticket and
// one last-workgroup decision per level.  Every workgroup is resident (cooperative
// launch), takes every decision from the same values read after a barrier, and so
// passes the same barriers and leaves at the same level.  The kernel keeps the frontier
// queues, the big-vertex queues, the unvisited degree sum mu and the Beamer switch of
// k_bfs_level; it stops at an empty frontier (done), when the switch picks bottom-up for
// the next level, or after max_levels levels, and then writes the state k_bfs_level
// resumes from (the frontier bitmaps are rebuilt by k_bfs_bitmap first).  Per-level
// counters rotate over four slots: the frontier length of level k is appended during
// level k - 1 and read up to the barrier that ends level k + 1 (every workgroup reads the
// level's totals right after the barrier that ends level k), so slot k mod 4 is cleared
// during level k + 2, before level k + 3 appends to it again.
constexpr u32 kRunSlots = 4;

struct BfsRun {
  u32 bar;                // barrier arrivals of this launch (zeroed before it)
  u32 next_k;             // out: level of the frontier left in the queues
  u32 qcnt[kRunSlots];    // frontier lengths by level mod 4
  u32 bcnt[kRunSlots];    // big-vertex queue lengths by level mod 4
  u64 mf[kRunSlots];      // frontier edges of the level, by level mod 4
  u64 dec[kRunSlots];     // degree of the vertices claimed in the level, by level mod 4
};

static_assert(sizeof(BfsRun) <= kBfsRunMaxBytes, "host copies of the run state are this large");
size_t bfs_run_bytes() { return sizeof(BfsRun); }

// All workgroups arrive once per barrier; `target` = barriers so far x grid size.
__device__ __forceinline__ void bfs_grid_sync(u32* bar, u32 target) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(bar, 1u);
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target)
      __builtin_amdgcn_s_sleep(1);
    __threadfence();
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kBfsThreads) k_bfs_run(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx, u32 n, u32 k0,
    u32 max_levels, u32* __restrict__ level, u32* __restrict__ queue0,
    u32* __restrict__ queue1, u32* __restrict__ bigq0, u32* __restrict__ bigq1,
    BfsCtl* __restrict__ ctl, BfsRun* __restrict__ st) {
  __shared__ u64 s_red[2 * (kBfsThreads / kWave)];
  // entry state, written by earlier kernels: the same values in every workgroup
  if (load_coherent(&ctl->done) || load_coherent(&ctl->mode) != 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->next_k = k0;
    return;
  }
  const u32 g = gridDim.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->qcnt[k0 % kRunSlots] = load_coherent(&ctl->qlen[k0 & 1]);
    st->bcnt[k0 % kRunSlots] = load_coherent(&ctl->bqlen[k0 & 1]);
  }
  u32 nbar = 1;
  bfs_grid_sync(&st->bar, nbar * g);
  u64 mus = __hip_atomic_load(&ctl->mu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  u32 depth = load_coherent(&ctl->depth);
  const u32 lane = lane_id(), wid = threadIdx.x / kWave;
  const u32 stride = g * blockDim.x;
  u32 k = k0, mode = 0, done = 0;
  while (true) {
    const u32 qn = load_coherent(&st->qcnt[k % kRunSlots]);
    if (qn == 0) {
      done = 1;
      break;
    }
    if (k == k0 + max_levels) break;
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // the slot of level k - 2 (and k + 2)
      const u32 r = (k + 2) % kRunSlots;
      __hip_atomic_store(&st->qcnt[r], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&st->bcnt[r], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store((unsigned long long*)&st->mf[r], 0ull, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store((unsigned long long*)&st->dec[r], 0ull, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    const u32* qin = (k & 1) ? queue1 : queue0;
    const u32* bqin = (k & 1) ? bigq1 : bigq0;
    const u32 next = k + 1;
    const BfsOut o{(k & 1) ? queue0 : queue1, &st->qcnt[next % kRunSlots],
                   (k & 1) ? bigq0 : bigq1, &st->bcnt[next % kRunSlots], nullptr};
    u64 mf = 0, mu_dec = 0;
    const u32 qr = (qn + kWave - 1) / kWave * kWave;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < qr; i += stride) {
      u32 x = 0, lo = 0, d = 0;
      if (i < qn) {
        x = qin[i];
        lo = rowptr[x];
        d = rowptr[x + 1] - lo;
        if (d > kBfsBig) d = 0;  // shared by the grid below
      }
      const bool big = d > kBfsLaneMax;
      u32 dl = big ? 0 : d;
      u32 dmax = dl;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) dmax = max(dmax, (u32)__shfl_xor(dmax, off, kWave));
      for (u32 j = 0; j < dmax; j += kBfsVisit) {
        u32 y[kBfsVisit];
        bool act[kBfsVisit];
#pragma unroll
        for (u32 t = 0; t < kBfsVisit; ++t) {
          act[t] = j + t < dl;
          y[t] = act[t] ? colidx[lo + j + t] : 0u;
        }
        td_visit(y, act, next, rowptr, level, o, mf, mu_dec);
      }
      u64 bigmask = __ballot(big);
      while (bigmask) {
        const int b = __ffsll((unsigned long long)bigmask) - 1;
        bigmask &= bigmask - 1;
        const u32 blo = __shfl(lo, b, kWave), bd = __shfl(d, b, kWave);
        for (u32 j0 = 0; j0 < bd; j0 += kWave * kBfsVisit) {
          u32 y[kBfsVisit];
          bool act[kBfsVisit];
#pragma unroll
          for (u32 t = 0; t < kBfsVisit; ++t) {
            const u32 j = j0 + t * kWave + lane;
            act[t] = j < bd;
            y[t] = act[t] ? colidx[blo + j] : 0u;
          }
          td_visit(y, act, next, rowptr, level, o, mf, mu_dec);
        }
      }
    }
    const u32 nbq = load_coherent(&st->bcnt[k % kRunSlots]);
    for (u32 bi = 0; bi < nbq; ++bi) {
      const u32 x = bqin[bi];
      const u32 lo = rowptr[x], d = rowptr[x + 1] - lo;
      const u32 nch = (d + kBfsChunk - 1) / kBfsChunk;
      const u32 shift = (u32)(((u64)bi * 131u) % g);
      for (u32 c = (blockIdx.x + g - shift) % g; c < nch; c += g) {
        const u32 ce = min(d, (c + 1) * kBfsChunk);
        for (u32 j0 = c * kBfsChunk; j0 < ce; j0 += blockDim.x * kBfsVisit) {
          u32 y[kBfsVisit];
          bool act[kBfsVisit];
#pragma unroll
          for (u32 t = 0; t < kBfsVisit; ++t) {
            const u32 j = j0 + t * blockDim.x + threadIdx.x;
            act[t] = j < ce;
            y[t] = act[t] ? colidx[lo + j] : 0u;
          }
          td_visit(y, act, next, rowptr, level, o, mf, mu_dec);
        }
      }
    }
    // the level's totals: one atomic per workgroup and counter
    mf = wave_sum_u64(mf);
    mu_dec = wave_sum_u64(mu_dec);
    if (lane == 0) {
      s_red[2 * wid] = mf;
      s_red[2 * wid + 1] = mu_dec;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      u64 a = 0, b = 0;
      for (u32 w = 0; w < blockDim.x / kWave; ++w) {
        a += s_red[2 * w];
        b += s_red[2 * w + 1];
      }
      if (a) atomicAdd((unsigned long long*)&st->mf[k % kRunSlots], (unsigned long long)a);
      if (b) atomicAdd((unsigned long long*)&st->dec[k % kRunSlots], (unsigned long long)b);
    }
    ++nbar;
    bfs_grid_sync(&st->bar, nbar * g);
    // every workgroup takes the same decision from the same totals
    const u32 nf = load_coherent(&st->qcnt[next % kRunSlots]);
    const u64 mfs =
        __hip_atomic_load(&st->mf[k % kRunSlots], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    mus -= __hip_atomic_load(&st->dec[k % kRunSlots], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    k = next;
    if (nf == 0) {
      done = 1;
      break;
    }
    depth = next;
    if (mfs > mus / 14) {
      mode = 1;
      break;
    }
  }
  // the state k_bfs_level resumes from (level k's frontier in queue[k & 1])
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const u32 qk = load_coherent(&st->qcnt[k % kRunSlots]);
    const u32 bk = load_coherent(&st->bcnt[k % kRunSlots]);
    __hip_atomic_store(&ctl->qlen[k & 1], done ? 0u : qk, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctl->qlen[(k + 1) & 1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctl->bqlen[k & 1], done ? 0u : bk, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctl->bqlen[(k + 1) & 1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store((unsigned long long*)&ctl->mu, (unsigned long long)mus, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctl->depth, depth, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctl->mode, mode, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctl->done, done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st->next_k, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
  }
}

// The three frontier bitmaps for level k after k_bfs_run: bitmap k mod 3 holds the
// frontier in queue[k & 1] (qn vertices), the other two are cleared.
__global__ void __launch_bounds__(kBfsThreads) k_bfs_bitmap(u32 n, u32 k,
                                                            const u32* __restrict__ queue0,
                                                            const u32* __restrict__ queue1,
                                                            const BfsCtl* __restrict__ ctl,
                                                            u32* __restrict__ fb, u32 phase) {
  const u32 nw = (n + 31) / 32;
  const u32 stride = gridDim.x * blockDim.x;
  if (phase == 0) {
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < 3 * nw; i += stride) fb[i] = 0;
  } else {
    const u32 qn = ctl->qlen[k & 1];
    const u32* q = (k & 1) ? queue1 : queue0;
    u32* bits = fb + (k % 3) * (size_t)nw;
    for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < qn; i += stride)
      atomicOr(&bits[q[i] >> 5], 1u << (q[i] & 31u));
  }
}

u32 bfs_grid(u32 n) {
  return max(1u, min(cdiv(n, kBfsThreads * kBfsPer), (u32)num_cus() * kBfsBlocksPerCu));
}
size_t bfs_part_words() { return 2 * (size_t)num_cus() * kBfsBlocksPerCu; }
size_t bfs_big_cap(u32 n, u64 m) { return (size_t)min((u64)n, m / (kBfsBig + 1) + 1); }

void launch_bfs_init(const u32* rowptr, const u32* parent, u32 n, u32* level, u32* queue0,
                     u32* bigq0, u32* fb, BfsCtl* ctl, hipStream_t s, bool keep) {
  // each workgroup adds its totals with same-address atomics
  const u32 g = max(1u, min(cdiv(n, kBfsThreads), (u32)num_cus() * kBfsBlocksPerCu));
  hipLaunchKernelGGL(k_bfs_init, dim3(g), dim3(kBfsThreads), 0, s, rowptr, parent, n, level,
                     queue0, bigq0, fb, ctl, keep ? 1u : 0u);
}

void launch_bfs_level(const u32* rowptr, const u32* colidx, u32 n, u32 k, u32* level,
                      u32* queue0, u32* queue1, u32* bigq0, u32* bigq1, u32* fb, BfsCtl* ctl,
                      u64* part, u32 grid, hipStream_t s) {
  hipLaunchKernelGGL(k_bfs_level, dim3(grid), dim3(kBfsThreads), 0, s, rowptr, colidx, n, k,
                     level, queue0, queue1, bigq0, bigq1, fb, ctl, part);
}

// Grid of the persistent levels: at most 32 workgroups, fewer for small graphs.  The
// levels these searches run are thin, and each barrier costs more with more workgroups
// (measured: 2.0 us with 32, 5.4 us with 128, 13.7 us with 256); on the 4096 x 4096 grid
// the BFS took 78.8, 74.5, 88.0 and 102.6 ms with 16, 32, 64 and 128 workgroups.  A
// small grid also leaves room for concurrent searches on other streams.
constexpr u32 kBfsRunMaxGrid = 32;

u32 bfs_run_grid(u32 n) {
  return max(1u, min(cdiv(n, kBfsThreads * kBfsPer), min(kBfsRunMaxGrid, (u32)num_cus())));
}

bool launch_bfs_run(const u32* rowptr, const u32* colidx, u32 n, u32 k0, u32 max_levels,
                    u32* level, u32* queue0, u32* queue1, u32* bigq0, u32* bigq1, BfsCtl* ctl,
                    void* run_state, u32 grid, hipStream_t s) {
  BfsRun* st = (BfsRun*)run_state;
  if (hipMemsetAsync(st, 0, sizeof(BfsRun), s) != hipSuccess) return false;
  void* args[] = {(void*)&rowptr, (void*)&colidx, (void*)&n, (void*)&k0, (void*)&max_levels,
                  (void*)&level, (void*)&queue0, (void*)&queue1, (void*)&bigq0, (void*)&bigq1,
                  (void*)&ctl, (void*)&st};
  return hipLaunchCooperativeKernel((const void*)k_bfs_run, dim3(grid), dim3(kBfsThreads), args,
                                    0, s) == hipSuccess;
}

u32 bfs_run_next_level(const void* run_state) {
  return ((const BfsRun*)run_state)->next_k;
}

void launch_bfs_bitmap(u32 n, u32 k, const u32* queue0, const u32* queue1, const BfsCtl* ctl,
                       u32* fb, hipStream_t s) {
  const u32 g = max(1u, min(cdiv(3 * ((n + 31) / 32), kBfsThreads), (u32)num_cus() * 4));
  hipLaunchKernelGGL(k_bfs_bitmap, dim3(g), dim3(kBfsThreads), 0, s, n, k, queue0, queue1, ctl,
                     fb, 0u);
  hipLaunchKernelGGL(k_bfs_bitmap, dim3(g), dim3(kBfsThreads), 0, s, n, k, queue0, queue1, ctl,
                     fb, 1u);
}

}  // namespace tc

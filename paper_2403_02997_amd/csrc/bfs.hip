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
// Each level's frontier is also kept as a bitmap (n bits, small enough to stay in the
// L2): bottom-up steps test neighbours against it instead of gathering their levels.
// Three bitmaps rotate: level k reads bitmap k mod 3, fills (k + 1) mod 3 and clears
// (k + 2) mod 3, the frontier of level k - 1, which level k + 1 fills next.
#include "tc_device.h"
#include "tc_launch.h"

namespace tc {

static inline u32 cdiv(u64 a, u64 b) { return (u32)((a + b - 1) / b); }

constexpr int kBfsThreads = 256;
constexpr u32 kBfsLaneMax = 32;  // frontier vertices up to this degree expand per lane
constexpr u32 kBfsPer = 8;       // vertices per thread and pass in the vertex sweeps

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
                                                          u32* __restrict__ fb0,
                                                          BfsCtl* __restrict__ ctl) {
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
        const bool root = parent[v] == v;
        level[v] = root ? 0u : kInf;
        roots += root;
        if (!root) mu += d;
        if (root && d > 0) {
          bits |= 1u << k;
          ++cnt;
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

__global__ void __launch_bounds__(kBfsThreads) k_bfs_level(
    const u32* __restrict__ rowptr, const u32* __restrict__ colidx, u32 n, u32 k,
    u32* __restrict__ level, u32* __restrict__ queue0, u32* __restrict__ queue1,
    u32* __restrict__ fb, BfsCtl* __restrict__ ctl) {
  __shared__ u64 s_red[2 * (kBfsThreads / kWave)];
  __shared__ bool s_last;
  if (load_coherent(&ctl->done)) return;  // uniform across the grid
  const u32 mode = load_coherent(&ctl->mode);
  const u32* qin = (k & 1) ? queue1 : queue0;
  u32* qout = (k & 1) ? queue0 : queue1;
  u32* qlen_out = &ctl->qlen[(k + 1) & 1];
  const u32 next = k + 1;
  u64 mf = 0, mu_dec = 0;
  const u32 lane = lane_id();
  const u32 stride = gridDim.x * blockDim.x;
  const u32 nw = (n + 31) / 32;
  const u32* fcur = fb + (k % 3) * (size_t)nw;
  u32* fnext = fb + ((k + 1) % 3) * (size_t)nw;
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
      }
      const bool big = d > kBfsLaneMax;
      // small frontier vertices: each lane walks its own list in lockstep
      u32 dl = big ? 0 : d;
      u32 dmax = dl;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) dmax = max(dmax, (u32)__shfl_xor(dmax, off, kWave));
      for (u32 j = 0; j < dmax; ++j) {
        bool claimed = false;
        u32 y = 0;
        if (j < dl) {
          y = colidx[lo + j];
          claimed = bfs_claim(level, y, next);
        }
        const u32 pos = wave_append(qlen_out, claimed);
        if (claimed) {
          qout[pos] = y;
          atomicOr(&fnext[y >> 5], 1u << (y & 31));
          const u32 dy = rowptr[y + 1] - rowptr[y];
          mf += dy;
          mu_dec += dy;
        }
      }
      // large frontier vertices: the whole wavefront strides each list
      u64 bigmask = __ballot(big);
      while (bigmask) {
        const int b = __ffsll((unsigned long long)bigmask) - 1;
        bigmask &= bigmask - 1;
        const u32 blo = __shfl(lo, b, kWave), bd = __shfl(d, b, kWave);
        for (u32 j0 = 0; j0 < bd; j0 += kWave) {
          const u32 j = j0 + lane;
          bool claimed = false;
          u32 y = 0;
          if (j < bd) {
            y = colidx[blo + j];
            claimed = bfs_claim(level, y, next);
          }
          const u32 pos = wave_append(qlen_out, claimed);
          if (claimed) {
            qout[pos] = y;
            atomicOr(&fnext[y >> 5], 1u << (y & 31));
            const u32 dy = rowptr[y + 1] - rowptr[y];
            mf += dy;
            mu_dec += dy;
          }
        }
      }
    }
  } else {
    // ---- bottom-up: every unvisited vertex looks for a neighbour on level k ----
    __shared__ u32 s_tmp[kBfsThreads / kWave];
    __shared__ u32 s_base;
    const u32 span = kBfsPer * blockDim.x;
    for (u32 base = blockIdx.x * span; base < n; base += gridDim.x * span) {
      u32 bits = 0, cnt = 0;
#pragma unroll
      for (u32 kk = 0; kk < kBfsPer; ++kk) {
        const u32 v = base + kk * blockDim.x + threadIdx.x;
        u32 lo = 0, d = 0;
        if (v < n && level[v] == kInf) {
          lo = rowptr[v];
          d = rowptr[v + 1] - lo;
        }
        bool found = false;
        // short lists: per lane, four neighbours per step
        const bool big = d > kBfsLaneMax;
        if (!big) {
          for (u32 j = 0; j < d && !found; j += 4) {
            u32 w[4];
#pragma unroll
            for (u32 i = 0; i < 4; ++i) w[i] = j + i < d ? colidx[lo + j + i] : 0u;
#pragma unroll
            for (u32 i = 0; i < 4; ++i) found |= j + i < d && ((fcur[w[i] >> 5] >> (w[i] & 31)) & 1u);
          }
        }
        // long lists: the whole wavefront, 64 neighbours per step
        u64 bm = __ballot(big);
        while (bm) {
          const int b = __ffsll((unsigned long long)bm) - 1;
          bm &= bm - 1;
          const u32 blo = __shfl(lo, b, kWave), bd = __shfl(d, b, kWave);
          bool bf = false;
          for (u32 j0 = 0; j0 < bd && !bf; j0 += kWave) {
            const u32 j = j0 + lane;
            bool hit = false;
            if (j < bd) {
              const u32 w = colidx[blo + j];
              hit = (fcur[w >> 5] >> (w & 31)) & 1u;
            }
            bf = __ballot(hit) != 0;
          }
          if ((int)lane == b) found = bf;
        }
        if (found) {
          level[v] = next;
          bits |= 1u << kk;
          ++cnt;
          mf += d;
          mu_dec += d;
        }
        store_bits_half(fnext, v, found, n);
      }
      u32 tot;
      const u32 incl = block_incl_scan(cnt, s_tmp, &tot);
      if (threadIdx.x == 0) s_base = tot ? atomicAdd(qlen_out, tot) : 0u;
      __syncthreads();
      u32 pos = s_base + incl - cnt;
#pragma unroll
      for (u32 kk = 0; kk < kBfsPer; ++kk)
        if (bits & (1u << kk)) qout[pos++] = base + kk * blockDim.x + threadIdx.x;
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
    if (a) atomicAdd((unsigned long long*)&ctl->mf, (unsigned long long)a);
    if (b) atomicAdd((unsigned long long*)&ctl->mu, (unsigned long long)(0 - b));
    __threadfence();
    const u32 ticket = atomicAdd(&ctl->blocks_done, 1u);
    s_last = ticket == gridDim.x - 1;
  }
  __syncthreads();
  if (s_last && threadIdx.x == 0) {
    __threadfence();
    const u32 nf = __hip_atomic_load(qlen_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const u64 mfs = __hip_atomic_load(&ctl->mf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const u64 mus = __hip_atomic_load(&ctl->mu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    ctl->qlen[k & 1] = 0;  // this level's input queue is the next level's output
    ctl->mf = 0;
    ctl->blocks_done = 0;
    __threadfence();
  }
}

// Two workgroups per CU: the per-level totals cost three same-address atomics per
// workgroup.
u32 bfs_grid(u32 n) { return max(1u, min(cdiv(n, kBfsThreads), (u32)num_cus() * 2)); }

void launch_bfs_init(const u32* rowptr, const u32* parent, u32 n, u32* level, u32* queue0,
                     u32* fb, BfsCtl* ctl, hipStream_t s) {
  const u32 g = bfs_grid(n);
  hipLaunchKernelGGL(k_bfs_init, dim3(g), dim3(kBfsThreads), 0, s, rowptr, parent, n, level,
                     queue0, fb, ctl);
}

void launch_bfs_level(const u32* rowptr, const u32* colidx, u32 n, u32 k, u32* level,
                      u32* queue0, u32* queue1, u32* fb, BfsCtl* ctl, u32 grid, hipStream_t s) {
  hipLaunchKernelGGL(k_bfs_level, dim3(grid), dim3(kBfsThreads), 0, s, rowptr, colidx, n, k,
                     level, queue0, queue1, fb, ctl);
}

}  // namespace tc

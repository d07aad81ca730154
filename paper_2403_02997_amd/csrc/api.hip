// C ABI of the cover-edge triangle-counting library (declared in include/tc.h) and the
// host-side orchestration of the single-graph path:
//
//   component roots (union-find, smallest ID)          CETC-Seq BFS restart loop
//   level BFS from all roots, direction-optimising      Def. BFS-Edge
//   per-vertex info byte (level parity, degree class)
//   cover-edge extraction: horizontal edges, oriented    Theorem Gen-CES
//   planning of the intersection classes
//   intersections with the apex rule                    CETC-Seq / CETC-SM
//   reduction of the per-block counters
//
// The graph is read-only and already resident on the device.  Scratch memory comes from
// the device's stream-ordered pool and is returned before the call completes.
#include <stdint.h>
#include <string.h>

#include <mutex>

#include "../../include/tc.h"
#include "tc_device.h"
#include "host_api.h"
#include "tc_launch.h"

namespace tc {

thread_local tc_call_info t_last_info{};  // see tc_last_call_info
thread_local bool t_side_on = true;  // see set_thread_side_stream

// A caller's device arena from which the calling thread's calls take their workspaces in
// place of the stream-ordered allocator (see set_thread_arena).
struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0;
};
thread_local Arena t_arena;
void set_thread_side_stream(bool on) { t_side_on = on; }


namespace {

constexpr int kVersion = 10000;  // 1.0.0

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Carves aligned sub-buffers out of one allocation.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = (T*)(base + off);
    off += sizeof(T) * count;
    return p;
  }
};

struct Layout {
  size_t bytes;
};

std::mutex g_pool_mu;
bool g_pool_ready[64];

// Keep freed stream-ordered memory in the device pool between calls.
void prepare_pool() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (g_pool_ready[dev]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  g_pool_ready[dev] = true;
}

// Fork / join of a second stream (default priority) on which the wavefront class and the
// hub count run beside the workgroup class.  The stream lives for one call only: a
// process has few hardware queues (four by default), and a stream kept alive would take
// one of them for good, so that other long-lived streams (a server's workers) could end
// up sharing a queue and waiting behind each other's kernels.  create() makes it (early
// in the call, while the GPU runs the BFS); start() orders it after the work queued on
// the main stream; join() (also run on destruction, before the workspace is released)
// orders the main stream after everything queued on it.  If anything fails, the caller
// stays on its own stream.
struct SideFork {
  hipStream_t s = nullptr, s2 = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool active = false;
  // Creates the stream and its two events (done early, while the host would otherwise
  // wait on the GPU).  False if any of them cannot be made.
  bool create() {
    if (s2) return true;
    if (!t_side_on) return false;
    if (hipStreamCreateWithFlags(&s2, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      s2 = nullptr;
      return false;
    }
    for (hipEvent_t& e : ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        e = nullptr;
        return false;
      }
    return true;
  }
  bool start(hipStream_t main) {
    s = main;
    if (!create()) return false;
    if (hipEventRecord(ev[0], s) != hipSuccess || hipStreamWaitEvent(s2, ev[0], 0) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    active = true;
    return true;
  }
  bool join() {
    if (!active) return true;
    active = false;
    return hipEventRecord(ev[1], s2) == hipSuccess && hipStreamWaitEvent(s, ev[1], 0) == hipSuccess;
  }
  ~SideFork() {
    if (!join()) (void)hipGetLastError();
    for (hipEvent_t e : ev)
      if (e) hipEventDestroy(e);
    if (s2) hipStreamDestroy(s2);  // its work is ordered before the main stream's next work
  }
};

// Calls below this many stored entries stay on one stream (the fork costs more than the
// overlap saves).
constexpr u32 kSideMinEntries = 1u << 22;

// Top-down levels per cooperative BFS launch at most.
constexpr u32 kBfsRunLevels = 1u << 16;

std::mutex g_coop_mu;  // serialises the cooperative BFS launches of concurrent calls

struct DevAlloc {
  void* p = nullptr;
  hipStream_t s = nullptr;
  bool owned = false;  // false: taken from the thread's arena
  ~DevAlloc() {
    if (p && owned) hipFreeAsync(p, s);
  }
};

#define TC_HIP(call)                          \
  do {                                        \
    if ((call) != hipSuccess) {               \
      (void)hipGetLastError();                \
      return TC_ERR_HIP;                      \
    }                                         \
  } while (0)

#define TC_LAUNCHED()                         \
  do {                                        \
    if (hipGetLastError() != hipSuccess) return TC_ERR_HIP; \
  } while (0)

int alloc_async(DevAlloc& a, size_t bytes, hipStream_t s) {
  a.s = s;
  if (bytes == 0) bytes = 256;
  if (t_arena.base) {
    const size_t off = (t_arena.used + 255) / 256 * 256;
    if (off > t_arena.size || bytes > t_arena.size - off) return TC_ERR_OUT_OF_MEMORY;
    a.p = t_arena.base + off;
    t_arena.used = off + bytes;
    return TC_OK;
  }
  a.owned = true;
  hipError_t e = hipMallocAsync(&a.p, bytes, s);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    a.p = nullptr;
    return TC_ERR_OUT_OF_MEMORY;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    a.p = nullptr;
    return TC_ERR_HIP;
  }
  return TC_OK;
}

// lane_max 8: with the pruned wavefront path, rows of 9..16 entries count faster four
// per wavefront (16-lane groups) than by one lane's full merge (4096-graph batch 108.0 ->
// 104.8 ms; R-MAT 22, er22 and the grid unchanged; 4 slowed the grid's lane-class edges)
IsectParams default_params() {
  IsectParams p;
  p.lane_max = 8;
  p.wave_max = 512;
  p.chunk = 4096;
  p.seg = 1024;
  return p;
}

IsectParams g_params = default_params();

// Host copy of the device degree class (4 steps per octave).
u32 host_degree_class(u32 d) {
  if (d == 0) return 0;
  u32 lg = 31;
  while (!((d >> lg) & 1u)) --lg;
  const u32 frac = lg >= 2 ? (d >> (lg - 2)) & 3u : ((d << (2 - lg)) & 3u);
  const u32 c = 1u + 4u * lg + frac;
  return c > 127u ? 127u : c;
}

// Hub pass: up to 256 hubs of degree at least 4096 (by class).
constexpr u32 kDefaultHubs = kMaxHubs;
constexpr u32 kDefaultHubDegree = 4096;
constexpr u64 kHubEntriesPerDegree = 1024;
u32 g_hub_max = kDefaultHubs;
u32 g_hub_min_degree = kDefaultHubDegree;

// CETC-Seq-FE's covering-ratio threshold.  The paper's experiments use 0.7; here the
// switch is off by default (a value above 1), because the forward ordering streams as
// much as the pruned pass and costs a second extraction (measured on ER 2^14 with
// degree 256: 2.32 ms switched against 1.92 ms kept).
constexpr double kDefaultForwardThreshold = 2.0;
double g_fe_threshold = kDefaultForwardThreshold;

struct RunOut {
  u64 c[kNumCtr];  // see kNumCtr: c1, c2, t2, streamed[3], staged[3]
  u64 cover_edges;
  BfsCtl ctl;
};

// ---- step timing (diagnostics) ----------------------------------------------------------
// When enabled, the single-graph path records HIP events on its own stream at every step
// boundary and accumulates the elapsed time of each step.
enum Step { kStepRoots, kStepBfs, kStepExtract, kStepPlan, kStepLane, kStepBlock, kStepWave,
            kStepHub, kStepReduce, kNumSteps };
const char* kStepNames[kNumSteps] = {"roots", "bfs", "extract", "plan", "isect_lane",
                                     "isect_block", "isect_wave", "isect_hub", "reduce"};
std::mutex g_prof_mu;
bool g_prof_on = false;
double g_prof_ms[kNumSteps];
u64 g_prof_calls = 0;

struct StepTimer {
  bool on;
  hipStream_t s;
  hipEvent_t ev[kNumSteps + 1];
  int next = 0;
  StepTimer(hipStream_t st) : s(st) {
    {
      std::lock_guard<std::mutex> lk(g_prof_mu);
      on = g_prof_on;
    }
    if (on)
      for (int i = 0; i <= kNumSteps; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) on = false;
  }
  // Marks the end of the previous step (and the start of the next one).
  void mark() {
    if (on && next <= kNumSteps) hipEventRecord(ev[next++], s);
  }
  // Called after the stream has been synchronised.
  void collect() {
    if (!on || next != kNumSteps + 1) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (int i = 0; i < kNumSteps; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) g_prof_ms[i] += ms;
    }
    g_prof_calls += 1;
  }
  ~StepTimer() {
    if (on)
      for (int i = 0; i <= kNumSteps; ++i) hipEventDestroy(ev[i]);
  }
};

size_t hub_item_cap(u32 n, u32 m) { return (size_t)n + m / kHubChunk + 1; }

// Device workspace of one single-graph call, carved from `base` in this order (every
// array 256-byte aligned).  The control block (ctl .. outc) is contiguous so that one
// memset clears it.  Returns the bytes needed; with base = nullptr only sizes.
struct SingleWs {
  u32 *parent, *level, *q0, *q1, *fb;
  size_t fb_words;
  u64* bfs_part;
  u32* bigq0;
  uint8_t* bfs_run;
  uint8_t* vinfo;
  u32 *hcnt, *split, *sabove, *hcur, *scan_tmp;
  uint4* hrec;
  u32 *colidx2, *lane_x, *wave_x, *block_x, *bitems;
  uint8_t* hubidx;
  u32 *hublist, *hy, *hubmask;
  uint2* hitems;
  u32* hcuts;
  BfsCtl* ctl;
  Plan* plan;
  u32* chist;
  u64 *ctr, *outc;
  u32 *tail4, *tail4b, *cc_mode;
};

size_t carve_single(void* base, u32 n, u32 m, bool hub_on, SingleWs* out) {
  SingleWs w;
  Carver c(base);
  w.parent = c.take<u32>(n);
  w.level = c.take<u32>(n);
  w.q0 = c.take<u32>(n);
  w.q1 = c.take<u32>(n);                        // BFS queue, then the list of long rows
  w.fb_words = 3 * (((size_t)n + 31) / 32);     // three frontier bitmaps
  w.fb = c.take<u32>(w.fb_words);
  w.bfs_part = c.take<u64>(bfs_part_words());   // per-workgroup BFS level totals
  w.bigq0 = c.take<u32>(2 * bfs_big_cap(n, m));  // queues of big frontier vertices
  w.bfs_run = c.take<uint8_t>(bfs_run_bytes());  // state of the cooperative BFS launch
  w.vinfo = c.take<uint8_t>(n);
  w.hcnt = c.take<u32>(n);
  w.split = c.take<u32>(n);
  w.sabove = c.take<u32>(n);
  w.hcur = c.take<u32>(n);                      // record cursors
  w.scan_tmp = c.take<u32>(scan_tmp_words(n));
  w.hrec = c.take<uint4>(m);                    // partner records in place of the rows
  w.colidx2 = c.take<u32>((size_t)m + 4);       // level-split rows, 4 readable padding entries
  w.lane_x = c.take<u32>(n);
  w.wave_x = c.take<u32>(n);
  w.block_x = c.take<u32>(n);
  w.bitems = c.take<u32>((size_t)n + 1);        // block items / offsets
  w.hubidx = c.take<uint8_t>(hub_on ? n : 0);
  w.hublist = c.take<u32>(hub_on ? kMaxHubs : 0);
  w.hy = reinterpret_cast<u32*>(c.take<uint4>(hub_on ? (size_t)n * kHubWords / 4 : 0));
  w.hubmask = reinterpret_cast<u32*>(c.take<uint4>(hub_on ? (size_t)n * kHubWords / 4 : 0));
  w.hitems = c.take<uint2>(hub_on ? hub_item_cap(n, m) : 0);
  w.hcuts = c.take<u32>(hub_on ? hub_cut_words(kMaxHubs, n) : 0);
  w.ctl = c.take<BfsCtl>(1);
  w.plan = c.take<Plan>(1);
  w.chist = c.take<u32>(128);                   // degree-class histogram
  w.ctr = c.take<u64>(kCounterSlots * kNumCtr);
  w.outc = c.take<u64>(kNumCtr);
  w.tail4 = c.take<u32>(4);
  w.tail4b = c.take<u32>(4);                    // padded last quad of colidx2
  w.cc_mode = c.take<u32>(4);
  if (out) *out = w;
  return c.off + 256;
}

// The whole single-graph pipeline.  `level_out` (device) may be null; `tri` (device,
// zeroed by the caller) selects per-vertex attribution.  split_stats (with pruned): the
// pruned kernels tally same-level apexes in t2 and other-level ones in c1.
int run_single(const u32* rowptr, const u32* colidx, u32 n, u32 m, hipStream_t s,
               u32* level_out, u64* tri, bool pruned, RunOut* out, bool split_stats = false) {
  prepare_pool();
  const IsectParams prm = g_params;
  // the hub pass serves the pruned count and per-vertex counts only (c1 / c2 tallies stay
  // per cover edge), on graphs of at least kHubEntriesPerDegree stored entries per unit of the hub
  // degree floor (smaller ones cannot give hubs enough partners to pay for the pass)
  const bool hub_size = (u64)m >= (u64)kHubEntriesPerDegree * g_hub_min_degree;
  const HubParams hp{pruned && hub_size ? g_hub_max : 0u,
                     host_degree_class(g_hub_min_degree)};
  const bool hub_on = hp.max_hubs > 0;
  const size_t hub_cap = hub_on ? hub_item_cap(n, m) : 0;
  const u32 max_s = m / 2;
  // ---- workspace ----
  const size_t bytes = carve_single(nullptr, n, m, hub_on, nullptr);
  DevAlloc ws;
  int rc = alloc_async(ws, bytes, s);
  if (rc) return rc;
  SingleWs w;
  carve_single(ws.p, n, m, hub_on, &w);
  u32* parent = w.parent;
  u32* level = w.level;
  u32* q0 = w.q0;
  u32* q1 = w.q1;
  const size_t fb_words = w.fb_words;
  u32* fb = w.fb;
  u64* bfs_part = w.bfs_part;
  u32* bigq0 = w.bigq0;
  u32* bigq1 = bigq0 + bfs_big_cap(n, m);
  uint8_t* bfs_run = w.bfs_run;
  uint8_t* vinfo = w.vinfo;
  u32* hcnt = w.hcnt;
  u32* split = w.split;
  u32* sabove = w.sabove;
  u32* hcur = w.hcur;
  u32* scan_tmp = w.scan_tmp;
  uint4* hrec = w.hrec;
  u32* colidx2 = w.colidx2;
  u32* lane_x = w.lane_x;
  u32* wave_x = w.wave_x;
  u32* block_x = w.block_x;
  u32* bitems = w.bitems;
  uint8_t* hubidx = w.hubidx;
  u32* hublist = w.hublist;
  u32* hy = w.hy;
  u32* hubmask = w.hubmask;
  uint2* hitems = w.hitems;
  u32* hcuts = w.hcuts;
  BfsCtl* ctl = w.ctl;
  Plan* plan = w.plan;
  u32* chist = w.chist;
  u64* ctr = w.ctr;
  u64* outc = w.outc;
  const size_t ctl_bytes = (char*)(outc + kNumCtr) - (char*)ctl;
  u32* tail4 = w.tail4;
  u32* tail4b = w.tail4b;
  u32* cc_mode = w.cc_mode;
  if (level_out) level = level_out;

  TC_HIP(hipMemsetAsync(ctl, 0, ctl_bytes, s));
  TC_HIP(hipMemsetAsync(fb, 0, sizeof(u32) * fb_words, s));
  TC_HIP(hipMemsetAsync(bitems, 0, sizeof(u32) * ((size_t)n + 1), s));
  StepTimer timer(s);

  // ---- a1: component roots ----
  // The first search runs from v0, the smallest vertex with neighbours (the first root of
  // the ascending restart loop); a union-find over the vertices it does not reach gives
  // the roots of the other components, which a second search then covers.  A graph
  // whose non-isolated vertices form one component needs no union-find at all.
  timer.mark();
  launch_first_root(rowptr, n, parent, cc_mode, s);
  TC_LAUNCHED();

  // ---- a2: level BFS ----
  timer.mark();
  SideFork fork;  // its stream is made while the first BFS levels run
  const bool want_side = !timer.on && m >= kSideMinEntries;
  BfsCtl hc;
  // One search from the roots in parent[] (keep: vertices already reached keep their
  // levels).  Batches of one launch per level, with a poll of the control block after
  // each; a search still in top-down mode after a batch (a large diameter) continues in
  // one cooperative launch that runs its top-down levels back to back (launch_bfs_run),
  // and resumes with per-level launches only for bottom-up levels.
  auto search = [&](bool keep) -> int {
    launch_bfs_init(rowptr, parent, n, level, q0, bigq0, fb, ctl, s, keep);
    TC_LAUNCHED();
    const u32 grid = bfs_grid(n);
    bool run_ok = true;  // cleared if the device refuses the cooperative launch
    u32 k = 0, batch = 8;  // low-diameter graphs finish within one poll
    while (true) {
      for (u32 i = 0; i < batch; ++i)
        launch_bfs_level(rowptr, colidx, n, k + i, level, q0, q1, bigq0, bigq1, fb, ctl, bfs_part,
                         grid, s);
      TC_LAUNCHED();
      if (k == 0 && want_side && !keep) fork.create();
      k += batch;
      TC_HIP(hipMemcpyAsync(&hc, ctl, sizeof(BfsCtl), hipMemcpyDeviceToHost, s));
      TC_HIP(hipStreamSynchronize(s));
      if (hc.done) break;
      if ((u64)k > (u64)n + 2) return TC_ERR_INTERNAL;  // a BFS has at most n levels
      batch = batch < 64 ? batch * 2 : 64;
      if (hc.mode != 0 || !run_ok) continue;
      alignas(16) char hr[kBfsRunMaxBytes];
      {
        // one cooperative launch at a time per process: the launch and its completion
        // stay under the lock, so concurrent searches on other threads never hold part
        // of the device each while waiting at their barriers
        std::lock_guard<std::mutex> lk(g_coop_mu);
        run_ok = launch_bfs_run(rowptr, colidx, n, k, kBfsRunLevels, level, q0, q1, bigq0,
                                bigq1, ctl, bfs_run, bfs_run_grid(n), s);
        if (!run_ok) {
          (void)hipGetLastError();
          continue;
        }
        TC_HIP(hipMemcpyAsync(hr, bfs_run, bfs_run_bytes(), hipMemcpyDeviceToHost, s));
        TC_HIP(hipMemcpyAsync(&hc, ctl, sizeof(BfsCtl), hipMemcpyDeviceToHost, s));
        TC_HIP(hipStreamSynchronize(s));
      }
      const u32 nk = bfs_run_next_level(hr);
      if (nk < k || (u64)nk > (u64)n + 2) return TC_ERR_INTERNAL;
      k = nk;
      if (hc.done) break;
      launch_bfs_bitmap(n, k, q0, q1, ctl, fb, s);  // per-level launches resume at level k
    }
    return TC_OK;
  };
  rc = search(false);
  if (rc) return rc;
  // the vertices the first search did not reach, if any: their roots, then their search
  launch_rest_init(level, n, parent, cc_mode, s);
  TC_LAUNCHED();
  u32 h_rest = 0;
  TC_HIP(hipMemcpyAsync(&h_rest, cc_mode + 2, sizeof(u32), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  BfsCtl first_ctl = hc;  // the first search's depth, roots and bottom-up levels
  bool two = false;
  if (h_rest > 0) {
    two = true;
    // a few unreached vertices (small components): join just their edges; many (v0 sat
    // in a small component): the sampled union-find over the whole graph, whose roots of
    // the reached vertices are v0 as well
    if (h_rest <= n / 8) launch_rest_links(rowptr, colidx, n, parent, cc_mode, s);
    else launch_cc(rowptr, colidx, n, m, parent, cc_mode, s);
    TC_HIP(hipMemsetAsync(ctl, 0, sizeof(BfsCtl), s));
    TC_HIP(hipMemsetAsync(fb, 0, sizeof(u32) * fb_words, s));
    TC_LAUNCHED();
    rc = search(true);
    if (rc) return rc;
  }
  timer.mark();
  // ---- a3: cover-edge extraction and planning ----
  // level_par = nullptr puts every vertex on one level (the forward ordering below)
  const HubView hv{&plan->hub_lim, hubidx, hy, hitems, &plan->num_hub_items, (u32)hub_cap};
  u32 h_items = 0;
  Plan h_plan;
  auto extract = [&](const u32* level_par) -> int {
    launch_vinfo(rowptr, level_par, n, vinfo, hcur, hub_on ? chist : nullptr, hp.min_class, s);
    if (hub_on) launch_hub_select(vinfo, n, chist, hp, hubidx, hublist, plan, s);
    // the BFS queues are free again: q1 lists the long rows
    launch_split_rows(rowptr, colidx, vinfo, n, m, colidx2, split, sabove, hcnt, hcur, hrec, q1,
                      &plan->num_long, hv, s);
    if (level_par) timer.mark();  // a second extraction is timed as planning
    launch_plan(rowptr, hcnt, hcur, n, prm, lane_x, wave_x, block_x, bitems, plan, s);
    launch_scan(bitems, bitems, n, scan_tmp, s);
    // padded last quads of both rows arrays, queued before the host waits for the plan
    launch_tail4(colidx, m, tail4, s);
    launch_tail4(colidx2, m, tail4b, s);
    TC_LAUNCHED();
    TC_HIP(hipMemcpyAsync(&h_items, bitems + n, sizeof(u32), hipMemcpyDeviceToHost, s));
    TC_HIP(hipMemcpyAsync(&h_plan, plan, sizeof(Plan), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    // a graph that is not symmetric can leave partner records unwritten: stop before
    // any intersection reads them
    if (h_plan.bad_records) return TC_ERR_INVALID_GRAPH;
    if (h_plan.num_cover > max_s) return TC_ERR_INTERNAL;
    if (h_plan.num_hubs > hp.max_hubs || h_plan.num_hub_items > hub_cap) return TC_ERR_INTERNAL;
    return TC_OK;
  };
  rc = extract(level);
  if (rc) return rc;
  const u32 h_ns = h_plan.num_cover;  // |S| under the BFS levels
  // CETC-Seq-FE (Alg. 11): with a covering ratio c = |S| / |E| at or above the threshold,
  // count by the forward algorithm instead.  With every vertex on one level every edge
  // is a cover edge and the apex rule keeps exactly the apexes above both endpoints, so
  // the same kernels then run the ID-ordered forward count (Alg. 5 with Alg. 6's hashed
  // intersections).  The first extraction is the computation of c; the counting call
  // only (per-vertex counts and the statistics keep the BFS levels).
  const bool forward = pruned && !tri && !split_stats && m > 0 &&
                       (double)h_ns >= g_fe_threshold * (double)(m / 2);
  if (forward) {
    TC_HIP(hipMemsetAsync(plan, 0, sizeof(Plan), s));
    TC_HIP(hipMemsetAsync(chist, 0, sizeof(u32) * 128, s));
    TC_HIP(hipMemsetAsync(bitems, 0, sizeof(u32) * ((size_t)n + 1), s));
    rc = extract(nullptr);
    if (rc) return rc;
  }

  // ---- a4: intersections ----
  DevAlloc items_mem;
  Item* items = nullptr;
  if (h_items) {
    rc = alloc_async(items_mem, sizeof(Item) * (size_t)h_items, s);
    if (rc) return rc;
    items = (Item*)items_mem.p;
    launch_fill_items(rowptr, hcnt, block_x, bitems, h_plan.num_block_x, prm, items, s);
  }
  const SplitView sv{colidx2, split, sabove, hcnt, hrec, tail4b};
  // the hub masks are built before the fork: their window kernel needs more LDS than a
  // compute unit has left beside a workgroup-class workgroup, so beside it it would wait
  // for the workgroup class to drain (with step timing on they run in the hub step)
  const bool hubs = h_plan.num_hubs > 0 && h_plan.num_hub_items > 0;
  if (hubs && !timer.on)
    launch_hub_masks(rowptr, colidx2, split, sabove, hublist, h_plan.num_hubs, n, hcuts, hubmask,
                     s);
  TC_LAUNCHED();
  // The workgroup class is bound by HBM streaming, the wavefront class and the hub count
  // by latency: the latter two run on the side stream, beside it (all on the caller's
  // stream, one after another, while step timing is on).
  const hipStream_t sw = want_side && fork.start(s) ? fork.s2 : s;
  if (sw != s) {
    // side stream first: the hub count and the wavefront class take compute units while
    // the workgroup class (persistent workgroups that hold their units to the end) ramps up
    if (hubs)
      launch_hub_count(rowptr, colidx2, sabove, split, h_plan.num_hubs, hy, hubmask, hitems,
                       h_plan.num_hub_items, ctr, split_stats, hublist, tri, sw);
    launch_isect_wave(rowptr, colidx, m, tail4, vinfo, sv, wave_x, h_plan.num_wave_x, plan, ctr,
                      tri, pruned, split_stats, sw);
    launch_isect_lane(rowptr, colidx, vinfo, sv, lane_x, h_plan.num_lane_x, ctr, tri, s);
    launch_isect_block(rowptr, colidx, m, tail4, vinfo, sv, items, h_items, prm, plan, ctr, tri,
                       pruned, split_stats, s);
  } else {
    timer.mark();
    launch_isect_lane(rowptr, colidx, vinfo, sv, lane_x, h_plan.num_lane_x, ctr, tri, s);
    timer.mark();
    launch_isect_block(rowptr, colidx, m, tail4, vinfo, sv, items, h_items, prm, plan, ctr, tri,
                       pruned, split_stats, s);
    timer.mark();
    launch_isect_wave(rowptr, colidx, m, tail4, vinfo, sv, wave_x, h_plan.num_wave_x, plan, ctr,
                      tri, pruned, split_stats, s);
    timer.mark();
    if (hubs && timer.on)
      launch_hub_masks(rowptr, colidx2, split, sabove, hublist, h_plan.num_hubs, n, hcuts, hubmask,
                       s);
    if (hubs)
      launch_hub_count(rowptr, colidx2, sabove, split, h_plan.num_hubs, hy, hubmask, hitems,
                       h_plan.num_hub_items, ctr, split_stats, hublist, tri, s);
    timer.mark();
  }
  TC_LAUNCHED();
  if (!fork.join()) {
    (void)hipGetLastError();
    return TC_ERR_HIP;
  }
  // ---- a5: reduction ----
  launch_finalize(ctr, outc, s);
  timer.mark();
  TC_LAUNCHED();
  TC_HIP(hipMemcpyAsync(out->c, outc, sizeof(u64) * kNumCtr, hipMemcpyDeviceToHost, s));
  TC_HIP(hipMemcpyAsync(&out->ctl, ctl, sizeof(BfsCtl), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  timer.collect();
  if (two) {  // both searches' statistics
    out->ctl.depth = std::max(out->ctl.depth, first_ctl.depth);
    out->ctl.num_roots += first_ctl.num_roots;
    out->ctl.bu_levels += first_ctl.bu_levels;
  }
  out->cover_edges = h_ns;
  // Two independent tallies of the same-level apexes must agree (CETC-SM: c2 / 3); the
  // pruned count does not tally c2.
  if (!pruned && (out->c[1] % 3 != 0 || out->c[1] / 3 != out->c[2])) return TC_ERR_INTERNAL;
  tc_call_info info{};
  info.cover_edges = h_ns;
  info.lane_vertices = h_plan.num_lane_x;
  info.wave_vertices = h_plan.num_wave_x;
  info.block_vertices = h_plan.num_block_x;
  info.block_items = h_items;
  info.hubs = hubs ? h_plan.num_hubs : 0u;
  info.hub_items = hubs ? h_plan.num_hub_items : 0u;
  info.side_stream = sw != s ? 1u : 0u;
  info.forward = forward ? 1u : 0u;
  t_last_info = info;
  return TC_OK;
}

int check_args(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n, uint64_t m) {
  if (n >= 0x40000000u) return TC_ERR_TOO_LARGE;  // LDS hash keys hold (w << 1) | same < 2^31
  // 32-bit entry offsets: tile ends (e0 + kTile) and rounded-up tile counts need headroom
  // below 2^32, so m stops 2^20 short of it.
  if (m > kMaxEntries) return TC_ERR_TOO_LARGE;
  if (n > 0 && !rowptr) return TC_ERR_INVALID_ARG;
  if (m > 0 && (!colidx || n == 0)) return TC_ERR_INVALID_ARG;
  return TC_OK;
}

}  // namespace

IsectParams current_isect_params() { return g_params; }

void set_thread_arena(void* base, size_t bytes) {
  t_arena.base = base ? static_cast<char*>(base) : nullptr;
  t_arena.size = base ? bytes : 0;
  t_arena.used = 0;
}

size_t single_call_bytes(u32 n, u64 m) {
  const IsectParams prm = g_params;
  const size_t items = (size_t)n + m / prm.seg + 1;  // workgroup items (allocated after planning)
  return carve_single(nullptr, n, (u32)m, g_hub_max > 0, nullptr) + sizeof(Item) * items + 256;
}

}  // namespace tc

using namespace tc;

extern "C" {

int tc_version(void) { return kVersion; }

const char* tc_status_string(int status) {
  switch (status) {
    case TC_OK: return "ok";
    case TC_ERR_INVALID_ARG: return "invalid argument";
    case TC_ERR_OUT_OF_MEMORY: return "device out of memory";
    case TC_ERR_HIP: return "HIP runtime error";
    case TC_ERR_INVALID_GRAPH: return "graph violates the CSR contract";
    case TC_ERR_TOO_LARGE: return "graph too large (n >= 2^30 or m > 2^32 - 2^20)";
    case TC_ERR_INTERNAL: return "internal consistency check failed";
    default: return "unknown status";
  }
}

int tc_count_ex(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n, uint64_t m,
                hipStream_t stream, uint64_t* count, uint32_t* level_out, tc_stats* stats) {
  int rc = check_args(rowptr, colidx, n, m);
  if (rc) return rc;
  if (!count && !stats) return TC_ERR_INVALID_ARG;
  tc_stats st;
  memset(&st, 0, sizeof(st));
  if (n == 0 || m == 0) {
    t_last_info = tc_call_info{};
    if (level_out && n > 0) {
      TC_HIP(hipMemsetAsync(level_out, 0, sizeof(uint32_t) * n, stream));
      TC_HIP(hipStreamSynchronize(stream));
    }
    st.num_roots = n;
  } else {
    RunOut ro;
    memset(&ro, 0, sizeof(ro));
    // without statistics the pruned count runs (no c2); with them every tally is kept
    rc = run_single(rowptr, colidx, n, (u32)m, stream, level_out, nullptr, stats == nullptr, &ro);
    if (rc) return rc;
    st.c1 = ro.c[0];
    st.c2 = ro.c[1];
    st.triangles = ro.c[0] + ro.c[2];
    st.probes = ro.c[3] + ro.c[4] + ro.c[5];
    for (int i = 0; i < 3; ++i) {
      st.class_streamed[i] = ro.c[3 + i];
      st.class_staged[i] = ro.c[6 + i];
    }
    st.cover_edges = ro.cover_edges;
    st.depth = ro.ctl.depth;
    st.num_roots = ro.ctl.num_roots;
    st.bfs_levels_bottom_up = ro.ctl.bu_levels;
  }
  if (count) *count = st.triangles;
  if (stats) *stats = st;
  return TC_OK;
}

int tc_count(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n, uint64_t m,
             hipStream_t stream, uint64_t* count) {
  if (!count) return TC_ERR_INVALID_ARG;
  return tc_count_ex(rowptr, colidx, n, m, stream, count, nullptr, nullptr);
}

int tc_count_split(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n, uint64_t m,
                   hipStream_t stream, uint64_t* t0_t1) {
  int rc = check_args(rowptr, colidx, n, m);
  if (rc) return rc;
  if (!t0_t1) return TC_ERR_INVALID_ARG;
  if (n == 0 || m == 0) {
    t_last_info = tc_call_info{};
    t0_t1[0] = 0;
    t0_t1[1] = 0;
    return TC_OK;
  }
  RunOut ro;
  memset(&ro, 0, sizeof(ro));
  rc = run_single(rowptr, colidx, n, (u32)m, stream, nullptr, nullptr, true, &ro, true);
  if (rc) return rc;
  t0_t1[0] = ro.c[2];  // same-level apexes above both ends: the triangles inside G0
  t0_t1[1] = ro.c[0];  // other-level apexes: the triangles with an edge in G1
  return TC_OK;
}

int tc_count_per_vertex(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n,
                        uint64_t m, hipStream_t stream, uint64_t* tri_out) {
  int rc = check_args(rowptr, colidx, n, m);
  if (rc) return rc;
  if (n > 0 && !tri_out) return TC_ERR_INVALID_ARG;
  if (n == 0 || m == 0) t_last_info = tc_call_info{};
  if (n == 0) return TC_OK;
  TC_HIP(hipMemsetAsync(tri_out, 0, sizeof(uint64_t) * n, stream));
  if (m == 0) {
    TC_HIP(hipStreamSynchronize(stream));
    return TC_OK;
  }
  RunOut ro;
  memset(&ro, 0, sizeof(ro));
  return run_single(rowptr, colidx, n, (u32)m, stream, nullptr, (u64*)tri_out, true, &ro);
}

int tc_validate_csr(const uint32_t* rowptr, const uint32_t* colidx, uint32_t n, uint64_t m,
                    hipStream_t stream) {
  int rc = check_args(rowptr, colidx, n, m);
  if (rc) return rc;
  if (n == 0) return m == 0 ? TC_OK : TC_ERR_INVALID_GRAPH;
  prepare_pool();
  const u32 ntiles = (u32)((m + kTile - 1) / kTile);
  DevAlloc ws;
  rc = alloc_async(ws, sizeof(u32) * (ntiles + 1) + 256 + 256, stream);
  if (rc) return rc;
  Carver c(ws.p);
  u32* flag = c.take<u32>(1);
  u32* tile_row = c.take<u32>(ntiles + 1);
  TC_HIP(hipMemsetAsync(flag, 0, sizeof(u32), stream));
  if (!validate_rowptr_ok(rowptr, n, (u32)m, flag, stream)) {
    TC_HIP(hipGetLastError());
    return TC_ERR_INVALID_GRAPH;
  }
  if (m == 0) return TC_OK;
  launch_tile_rows(rowptr, n, (u32)m, tile_row, stream);
  launch_validate(rowptr, colidx, tile_row, n, (u32)m, flag, stream);
  TC_LAUNCHED();
  u32 h = 0;
  TC_HIP(hipMemcpyAsync(&h, flag, sizeof(u32), hipMemcpyDeviceToHost, stream));
  TC_HIP(hipStreamSynchronize(stream));
  return h ? TC_ERR_INVALID_GRAPH : TC_OK;
}

size_t tc_count_batch_workspace_size(uint32_t num_graphs, uint64_t total_rows,
                                     uint64_t total_cols) {
  return batch_workspace_bytes(num_graphs, total_rows, total_cols);
}

int tc_count_batch(const uint32_t* rowptr_cat, const uint32_t* colidx_cat,
                   const int64_t* row_off, const int64_t* col_off, uint32_t num_graphs,
                   uint64_t total_rows, uint64_t total_cols, void* workspace,
                   size_t workspace_bytes, hipStream_t stream, uint64_t* counts) {
  if (num_graphs == 0) return TC_OK;
  if (!rowptr_cat || !row_off || !col_off || !counts || total_rows < num_graphs ||
      (total_cols > 0 && !colidx_cat))
    return TC_ERR_INVALID_ARG;
  if (total_cols > kMaxEntries || total_rows > kMaxEntries) return TC_ERR_TOO_LARGE;
  const IsectParams prm = g_params;
  const size_t need = batch_workspace_bytes(num_graphs, total_rows, total_cols);
  if (workspace) {
    if (workspace_bytes < need) return TC_ERR_INVALID_ARG;
    launch_batch(rowptr_cat, colidx_cat, row_off, col_off, num_graphs, total_rows, total_cols,
                 workspace, prm, (u64*)counts, stream);
    TC_LAUNCHED();
    return TC_OK;
  }
  prepare_pool();
  DevAlloc ws;
  int rc = alloc_async(ws, need, stream);
  if (rc) return rc;
  launch_batch(rowptr_cat, colidx_cat, row_off, col_off, num_graphs, total_rows, total_cols,
               ws.p, prm, (u64*)counts, stream);
  TC_LAUNCHED();
  return TC_OK;
}

// Intersection class thresholds (used by the autotuner).  Returns TC_ERR_INVALID_ARG for
// values outside the ranges the LDS tables are sized for.
int tc_set_isect_params(uint32_t lane_max, uint32_t wave_max, uint32_t chunk, uint32_t seg) {
  if (wave_max > 512 || lane_max > wave_max || chunk == 0 || chunk > 16384 || seg == 0 ||
      seg > 1024)
    return TC_ERR_INVALID_ARG;
  g_params.lane_max = lane_max;
  g_params.wave_max = wave_max;
  g_params.chunk = chunk;
  g_params.seg = seg;
  return TC_OK;
}

int tc_set_hub_params(uint32_t max_hubs, uint32_t min_degree) {
  if (max_hubs > kMaxHubs) return TC_ERR_INVALID_ARG;
  g_hub_max = max_hubs;
  g_hub_min_degree = min_degree;
  return TC_OK;
}

int tc_set_forward_threshold(double threshold) {
  if (!(threshold >= 0.0) || threshold != threshold || threshold > 1e300) return TC_ERR_INVALID_ARG;
  g_fe_threshold = threshold;
  return TC_OK;
}

double tc_get_forward_threshold(void) { return g_fe_threshold; }

int tc_get_hub_params(uint32_t* out2) {
  if (!out2) return TC_ERR_INVALID_ARG;
  out2[0] = g_hub_max;
  out2[1] = g_hub_min_degree;
  return TC_OK;
}

int tc_last_call_info(tc_call_info* out) {
  if (!out) return TC_ERR_INVALID_ARG;
  *out = t_last_info;
  return TC_OK;
}

int tc_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return TC_OK;
}

int tc_profile_read(double* ms_out, uint32_t cap, uint64_t* calls, int reset) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (ms_out)
    for (uint32_t i = 0; i < cap && i < (uint32_t)kNumSteps; ++i) ms_out[i] = g_prof_ms[i];
  if (calls) *calls = g_prof_calls;
  if (reset) {
    for (int i = 0; i < kNumSteps; ++i) g_prof_ms[i] = 0.0;
    g_prof_calls = 0;
  }
  return kNumSteps;
}

const char* tc_profile_step_name(int step) {
  return step >= 0 && step < kNumSteps ? kStepNames[step] : "";
}

int tc_get_isect_params(uint32_t* out4) {
  if (!out4) return TC_ERR_INVALID_ARG;
  out4[0] = g_params.lane_max;
  out4[1] = g_params.wave_max;
  out4[2] = g_params.chunk;
  out4[3] = g_params.seg;
  return TC_OK;
}

}  // extern "C"

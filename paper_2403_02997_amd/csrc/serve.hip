// Continuous-batching server over the counting path (declared in include/tc.h).
//
// Requests arrive as HOST CSR arrays and are routed at once, by size, to one of three
// paths, each driven by its own host thread and HIP stream so that they overlap on the
// device and a small request never waits behind the upload of a large one:
//   batched : at most `small_max_entries` stored entries.  Whenever the previous batch
//             has completed, everything queued since is packed into one concatenated
//             CSR (uploaded once, resident until its counts are back) and counted by one
//             tc_count_batch launch;
//   medium  : up to `large_min_entries`, one tc_count call each, in arrival order;
//   large   : the rest, one tc_count call each, smallest first (a request that has
//             waited kLargeMaxWait seconds since submission goes next).
// Device memory: each path keeps one device buffer for its jobs (CSR, offsets, results
// and the counting workspace, which tc_count takes from it through the thread's arena
// instead of allocating), grown when a job needs more and kept between jobs, so that a
// steady stream of requests allocates nothing.  The buffers are held against the HBM
// budget: a path that must grow gives its buffer back and reserves the new size, waiting,
// in the order the paths asked, while it does not fit beside the other paths' buffers;
// while a path waits, the others give theirs back as soon as they are idle (the waiting
// path frees those of idle paths itself) or their current job ends.  An idle path also
// gives back a buffer above kIdleKeepBytes.  Queued requests hold no device memory, so a
// backlog on one path never keeps the others from starting.  (Allocating and freeing
// every job's memory through the stream-ordered allocator, with three streams doing so
// at once, stalled single allocations for up to 1.5 s.)
//
// The paths' uploads overlap with each other and with the counting, but the counting
// itself runs one job at a time: a path takes the device before its first kernel and
// hands it back after its result has been read.  Every count already fills the device
// (persistent grids, one 1024-thread workgroup per compute unit with most of its LDS),
// so kernels of two paths cannot share compute units; launched side by side, each
// path's short kernels waited behind the other paths' long ones, and the three paths
// together ran at well under half the rate of the same jobs run one by one.  The device
// goes to the waiting path of smallest jobs (batched, then medium, then large), except
// that a path that has waited kDeviceMaxWait seconds for it goes first.
// Results carry the request's submit, start (admit) and completion times on the server
// clock.
// Requests come from callers, so their bounds are checked before any kernel reads them:
// rowptr[0] = 0 and rowptr[n] = m at submission, the rest of the bounds (rowptr
// non-decreasing, every ID < n) on the host for batched requests and on the device for
// the others; a request that breaks them completes with TC_ERR_INVALID_GRAPH.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/tc.h"
#include "host_api.h"
#include "tc_launch.h"

namespace tc {
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket;
  const uint32_t* rowptr;
  const uint32_t* colidx;
  uint32_t n;
  uint64_t m;
  uint64_t footprint;
  double t_submit, t_admit, t_count;
};

// The large path serves the smallest queued request first (by stored entries), so a
// stream of scale-22..24 requests does not queue behind a scale-26 one; a request that
// has waited this long since submission is served next regardless.
constexpr double kLargeMaxWait = 2.0;  // seconds

// A path that has waited this long for the device takes it next, whatever its rank.
constexpr double kDeviceMaxWait = 0.5;  // seconds

// An idle path keeps a buffer up to this size for its next job.
constexpr uint64_t kIdleKeepBytes = 4ull << 30;

inline size_t up256(size_t x) { return (x + 255) / 256 * 256; }

// Buffer of a single-graph job: rowptr, colidx, the bounds-check flag, then the arena of
// the tc_count call.
struct SingleJobLayout {
  size_t o_ci, o_flag, o_ws, ws, total;
  SingleJobLayout(uint32_t n, uint64_t m) {
    o_ci = up256(4ull * ((uint64_t)n + 1));
    o_flag = o_ci + up256(4ull * std::max<uint64_t>(m, 1));
    o_ws = o_flag + 256;
    ws = single_call_bytes(n, m);
    total = o_ws + up256(ws);
  }
};

// Buffer of a batched job: concatenated rowptrs and colidx, row and entry offsets, counts,
// then the tc_count_batch workspace.
struct BatchJobLayout {
  size_t o_ci, o_ro, o_co, o_cnt, o_ws, ws, total;
  BatchJobLayout(uint32_t G, uint64_t rows, uint64_t cols) {
    o_ci = up256(4 * rows);
    o_ro = o_ci + up256(4 * cols);
    o_co = o_ro + up256(8 * ((size_t)G + 1));
    o_cnt = o_co + up256(8 * ((size_t)G + 1));
    o_ws = o_cnt + up256(8 * (size_t)G);
    ws = tc_count_batch_workspace_size(G, rows, cols);
    total = o_ws + up256(ws);
  }
};

// The bounds a request must keep before any kernel reads it: rowptr non-decreasing from 0
// to m and every neighbour ID below n.  A batched request that broke them would send the
// batch kernel into other members' slices or past the workspace, so small requests are
// checked here on the host (at most small_max_entries entries each); the single-graph
// paths check the same on the device after the upload (check_csr_bounds).
bool host_bounds_ok(const Request& r) {
  if (r.rowptr[0] != 0 || r.rowptr[r.n] != r.m) return false;
  for (uint32_t v = 0; v < r.n; ++v)
    if (r.rowptr[v + 1] < r.rowptr[v]) return false;
  uint32_t mx = 0;
  for (uint64_t e = 0; e < r.m; ++e) mx = std::max(mx, r.colidx[e]);
  return r.m == 0 || mx < r.n;
}

}  // namespace
}  // namespace tc

using namespace tc;

struct tc_server {
  int device = 0;
  tc_serve_config cfg{};
  Clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_path[3], cv_mem, cv_dev, cv_done;
  std::deque<Request> ready[3];  // routed, not started: [0] batched, [1] medium, [2] large
  std::deque<int> mem_wait;      // paths waiting for device memory, in the order they asked
  std::deque<tc_serve_result> done;
  tc_serve_stats st{};
  uint64_t next_ticket = 1;
  bool stop = false;

  // each path's device buffer; `running` while a job uses it
  struct PathBuf {
    char* p = nullptr;
    size_t bytes = 0;
    bool running = false;
  } buf[3];

  int dev_owner = -1;                       // the path whose job is counting, or -1
  double dev_since = 0;                     // when the owner took the device
  double dev_wait_since[3] = {-1, -1, -1};  // when each path began to wait for the device

  hipStream_t stream[3] = {nullptr, nullptr, nullptr};
  std::thread th[3];

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  int path_of(uint64_t m) const {
    return m <= cfg.small_max_entries ? 0 : m >= cfg.large_min_entries ? 2 : 1;
  }

  // Buffer bytes a request needs on its own (what submission checks against the budget).
  uint64_t footprint(uint32_t n, uint64_t m) const {
    return path_of(m) == 0 ? BatchJobLayout(1, (uint64_t)n + 1, m).total
                           : SingleJobLayout(n, m).total;
  }

  // ---- device memory -----------------------------------------------------------------

  // Gives path k's buffer back (its stream has no work left).  Caller holds mu.
  void free_buf_locked(int k) {
    if (!buf[k].p) return;
    (void)hipFreeAsync(buf[k].p, stream[k]);
    st.hbm_in_use -= buf[k].bytes;
    buf[k].p = nullptr;
    buf[k].bytes = 0;
    cv_mem.notify_all();
  }

  // Takes `bytes` of the budget for path k.  A path that cannot have them at once queues
  // behind the paths already waiting; when it is first in line it frees the buffers of
  // idle paths, and running paths give theirs back when their job ends, so it takes them
  // once they fit: every wait ends.  Caller holds lk.
  void reserve(std::unique_lock<std::mutex>& lk, int k, uint64_t bytes) {
    mem_wait.push_back(k);
    while (true) {
      if (mem_wait.front() == k) {
        if (st.hbm_in_use + bytes > st.hbm_budget)
          for (int j = 0; j < 3; ++j)
            if (j != k && !buf[j].running) free_buf_locked(j);
        if (st.hbm_in_use + bytes <= st.hbm_budget) break;
      }
      cv_mem.wait(lk);
    }
    mem_wait.pop_front();
    cv_mem.notify_all();  // the next waiter may fit as well
    st.hbm_in_use += bytes;
    st.hbm_peak = std::max(st.hbm_peak, st.hbm_in_use);
  }

  // Makes path k's buffer at least `need` bytes (need <= budget) and marks it running.
  // Returns TC_OK, or TC_ERR_OUT_OF_MEMORY when the device refuses the allocation.
  // Caller holds lk; it is released while the allocation is made.
  int take_buf(std::unique_lock<std::mutex>& lk, int k, size_t need) {
    // (a job checked at submission can outgrow the budget only if the counting settings
    // changed meanwhile)
    if (need > st.hbm_budget) return TC_ERR_OUT_OF_MEMORY;
    if (buf[k].bytes < need) {
      free_buf_locked(k);
      // some headroom, so that a run of slightly larger jobs does not grow it each time
      const size_t want =
          std::max<size_t>(need, std::min<uint64_t>(st.hbm_budget, up256(need + need / 8)));
      reserve(lk, k, want);
      buf[k].bytes = want;
      buf[k].running = true;
      lk.unlock();
      char* p = nullptr;
      const bool ok = hipMallocAsync((void**)&p, want, stream[k]) == hipSuccess;
      if (!ok) (void)hipGetLastError();
      lk.lock();
      if (!ok) {
        st.hbm_in_use -= want;
        buf[k].bytes = 0;
        buf[k].running = false;
        cv_mem.notify_all();
        return TC_ERR_OUT_OF_MEMORY;
      }
      buf[k].p = p;
      return TC_OK;
    }
    buf[k].running = true;
    return TC_OK;
  }

  // After a job of path k: its buffer goes back if another path waits for memory, or if
  // the path is idle and the buffer is large.  Caller holds mu.
  void end_job_locked(int k) {
    buf[k].running = false;
    if (!mem_wait.empty() || (ready[k].empty() && buf[k].bytes > kIdleKeepBytes))
      free_buf_locked(k);
  }

  // ---- the device --------------------------------------------------------------------

  // The path that takes the device next: one that has waited kDeviceMaxWait (the
  // longest waiting first), else the lowest-numbered waiting path, else -1.  Caller
  // holds mu.
  int next_device_path() const {
    const double t = now();
    int pick = -1;
    for (int k = 0; k < 3; ++k)
      if (dev_wait_since[k] >= 0 && t - dev_wait_since[k] >= kDeviceMaxWait &&
          (pick < 0 || dev_wait_since[k] < dev_wait_since[pick]))
        pick = k;
    if (pick >= 0) return pick;
    for (int k = 0; k < 3; ++k)
      if (dev_wait_since[k] >= 0) return k;
    return -1;
  }

  // Path k takes the device for one job's counting; returns when it took it.  The device
  // is handed from owner to owner: release_device names the next one, so while it is free
  // nobody waits for it.
  double acquire_device(int k) {
    std::unique_lock<std::mutex> lk(mu);
    if (dev_owner < 0) {
      dev_owner = k;
      dev_since = now();
      return dev_since;
    }
    dev_wait_since[k] = now();
    cv_dev.wait(lk, [&] { return dev_owner == k; });
    return dev_since;
  }

  void release_device() {
    std::lock_guard<std::mutex> lk(mu);
    const double t = now();
    st.device_s[dev_owner] += t - dev_since;
    dev_owner = next_device_path();
    dev_since = t;
    if (dev_owner >= 0) dev_wait_since[dev_owner] = -1;
    cv_dev.notify_all();
  }

  void finish_locked(const Request& r, int status, uint64_t tri, uint32_t path) {
    tc_serve_result res{};
    res.ticket = r.ticket;
    res.triangles = status == TC_OK ? tri : 0;
    res.status = status;
    res.path = path;
    res.input_edges = r.m / 2;
    res.submit_s = r.t_submit;
    res.admit_s = r.t_admit;
    res.count_s = r.t_count;
    res.done_s = now();
    done.push_back(res);
    st.in_flight -= 1;
    st.completed += 1;
    cv_done.notify_all();
  }

  // ---- batched path ------------------------------------------------------------------
  // Uploads the batch into the path's buffer, takes the device, counts, reads the counts.
  int run_batch(const std::vector<Request>& b, const BatchJobLayout& L, uint64_t rows,
                uint64_t cols, std::vector<uint64_t>& counts, double* t_count) {
    const hipStream_t s = stream[0];
    char* const dev = buf[0].p;
    const uint32_t G = (uint32_t)b.size();
    std::vector<int64_t> row_off(G + 1), col_off(G + 1);
    row_off[0] = col_off[0] = 0;
    for (uint32_t i = 0; i < G; ++i) {
      row_off[i + 1] = row_off[i] + b[i].n + 1;
      col_off[i + 1] = col_off[i] + (int64_t)b[i].m;
    }
    int rc = TC_OK;
    for (uint32_t i = 0; i < G && rc == TC_OK; ++i) {
      if (hipMemcpyAsync(dev + 4 * row_off[i], b[i].rowptr, 4ull * (b[i].n + 1),
                         hipMemcpyHostToDevice, s) != hipSuccess)
        rc = TC_ERR_HIP;
      if (rc == TC_OK && b[i].m &&
          hipMemcpyAsync(dev + L.o_ci + 4 * col_off[i], b[i].colidx, 4ull * b[i].m,
                         hipMemcpyHostToDevice, s) != hipSuccess)
        rc = TC_ERR_HIP;
    }
    if (rc == TC_OK &&
        (hipMemcpyAsync(dev + L.o_ro, row_off.data(), 8 * ((size_t)G + 1),
                        hipMemcpyHostToDevice, s) != hipSuccess ||
         hipMemcpyAsync(dev + L.o_co, col_off.data(), 8 * ((size_t)G + 1),
                        hipMemcpyHostToDevice, s) != hipSuccess))
      rc = TC_ERR_HIP;
    // the upload completes before the device is taken for the count
    if (hipStreamSynchronize(s) != hipSuccess && rc == TC_OK) rc = TC_ERR_HIP;
    *t_count = acquire_device(0);
    if (rc == TC_OK)
      rc = tc_count_batch((const uint32_t*)dev, (const uint32_t*)(dev + L.o_ci),
                          (const int64_t*)(dev + L.o_ro), (const int64_t*)(dev + L.o_co), G,
                          rows, cols, dev + L.o_ws, L.ws, s, (uint64_t*)(dev + L.o_cnt));
    counts.assign(G, 0);
    if (rc == TC_OK && hipMemcpyAsync(counts.data(), dev + L.o_cnt, 8 * (size_t)G,
                                      hipMemcpyDeviceToHost, s) != hipSuccess)
      rc = TC_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess && rc == TC_OK) rc = TC_ERR_HIP;
    release_device();
    (void)hipGetLastError();
    return rc;
  }

  void batch_loop() {
    (void)hipSetDevice(device);
    while (true) {
      std::vector<Request> b;
      uint64_t rows = 0, cols = 0;
      int rc = TC_OK;
      double t_start = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_path[0].wait(lk, [&] { return stop || !ready[0].empty(); });
        if (stop) return;
        // everything queued, up to the batch limits and the whole budget (a request
        // alone always fits it: larger ones are rejected at submission)
        while (!ready[0].empty() && b.size() < cfg.batch_max_graphs) {
          const Request& r = ready[0].front();
          if (!b.empty() &&
              (cols + r.m > cfg.batch_max_entries ||
               BatchJobLayout((uint32_t)b.size() + 1, rows + r.n + 1, cols + r.m).total >
                   st.hbm_budget))
            break;
          rows += r.n + 1;
          cols += r.m;
          b.push_back(r);
          ready[0].pop_front();
        }
        st.queued -= b.size();
        st.batches += 1;
        rc = take_buf(lk, 0, BatchJobLayout((uint32_t)b.size(), rows, cols).total);
        t_start = now();
        for (Request& r : b) r.t_admit = r.t_count = t_start;
      }
      std::vector<Request> bad;
      size_t kept = 0;
      for (size_t i = 0; i < b.size(); ++i) {
        if (host_bounds_ok(b[i])) b[kept++] = b[i];
        else bad.push_back(b[i]);
      }
      b.resize(kept);
      rows = cols = 0;
      for (const Request& r : b) {
        rows += r.n + 1;
        cols += r.m;
      }
      std::vector<uint64_t> counts;
      if (rc == TC_OK && !b.empty()) {
        double t_count = t_start;
        rc = run_batch(b, BatchJobLayout((uint32_t)b.size(), rows, cols), rows, cols, counts,
                       &t_count);
        for (Request& r : b) r.t_count = t_count;
      }
      std::lock_guard<std::mutex> lk(mu);
      st.busy_s[0] += now() - t_start;
      if (buf[0].running) end_job_locked(0);
      for (const Request& r : bad) finish_locked(r, TC_ERR_INVALID_GRAPH, 0, 0);
      for (size_t i = 0; i < b.size(); ++i)
        finish_locked(b[i], rc, rc == TC_OK ? counts[i] : 0, 0);
    }
  }

  // ---- single-graph paths ------------------------------------------------------------
  // Uploads the request into path k's buffer, takes the device, checks the bounds and
  // counts with the buffer's arena as tc_count's workspace.
  int run_single(const Request& r, int k, uint64_t* tri, double* t_count) {
    const hipStream_t s = stream[k];
    char* const dev = buf[k].p;
    const SingleJobLayout L(r.n, r.m);
    int rc = TC_OK;
    if (hipMemcpyAsync(dev, r.rowptr, 4ull * (r.n + 1), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        (r.m && hipMemcpyAsync(dev + L.o_ci, r.colidx, 4ull * r.m, hipMemcpyHostToDevice, s) !=
                    hipSuccess))
      rc = TC_ERR_HIP;
    // the upload completes before the device is taken for the bounds check and the count
    if (hipStreamSynchronize(s) != hipSuccess && rc == TC_OK) rc = TC_ERR_HIP;
    *t_count = acquire_device(k);
    if (rc == TC_OK) {
      const int b = check_csr_bounds((const uint32_t*)dev, (const uint32_t*)(dev + L.o_ci), r.n,
                                     (uint32_t)r.m, (uint32_t*)(dev + L.o_flag), s);
      rc = b == 0 ? TC_OK : (b == -4 ? TC_ERR_INVALID_GRAPH : TC_ERR_HIP);
    }
    if (rc == TC_OK) {
      set_thread_arena(dev + L.o_ws, buf[k].bytes - L.o_ws);
      rc = tc_count((const uint32_t*)dev, (const uint32_t*)(dev + L.o_ci), r.n, r.m, s, tri);
      set_thread_arena(nullptr, 0);
    }
    if (hipStreamSynchronize(s) != hipSuccess && rc == TC_OK) rc = TC_ERR_HIP;
    release_device();
    (void)hipGetLastError();
    return rc;
  }

  // k = 1 medium, k = 2 large
  void single_loop(int k) {
    (void)hipSetDevice(device);
    set_thread_side_stream(false);  // this thread's stream is one of the server's three
    while (true) {
      Request r;
      int rc;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_path[k].wait(lk, [&] { return stop || !ready[k].empty(); });
        if (stop) return;
        std::deque<Request>& q = ready[k];
        auto pick = q.begin();
        if (k == 2 && now() - q.front().t_submit < kLargeMaxWait) {
          // shortest first by stored entries, unless the oldest has waited too long
          for (auto it = q.begin(); it != q.end(); ++it)
            if (it->m < pick->m) pick = it;
        }
        r = *pick;
        q.erase(pick);
        st.queued -= 1;
        st.singles += 1;
        rc = take_buf(lk, k, SingleJobLayout(r.n, r.m).total);
        r.t_admit = r.t_count = now();
      }
      uint64_t tri = 0;
      if (rc == TC_OK) rc = run_single(r, k, &tri, &r.t_count);
      std::lock_guard<std::mutex> lk(mu);
      st.busy_s[k] += now() - r.t_admit;
      if (buf[k].running) end_job_locked(k);
      finish_locked(r, rc, tri, k == 1 ? 1u : 3u);
    }
  }
};

extern "C" {

int tc_serve_create(const tc_serve_config* cfg, tc_server** out) {
  if (!out) return TC_ERR_INVALID_ARG;
  tc_server* s = new tc_server();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return TC_ERR_HIP;
  }
  if (cfg) s->cfg = *cfg;
  if (!s->cfg.small_max_entries) s->cfg.small_max_entries = 1ull << 18;
  if (!s->cfg.batch_max_graphs) s->cfg.batch_max_graphs = 4096;
  if (!s->cfg.batch_max_entries) s->cfg.batch_max_entries = 1ull << 28;
  if (!s->cfg.large_min_entries) s->cfg.large_min_entries = 1ull << 25;
  if (!s->cfg.hbm_budget_bytes) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      delete s;
      return TC_ERR_HIP;
    }
    s->cfg.hbm_budget_bytes = (uint64_t)(free_b / 10 * 8);
  }
  s->st.hbm_budget = s->cfg.hbm_budget_bytes;
  for (int i = 0; i < 3; ++i) {
    if (hipStreamCreateWithFlags(&s->stream[i], hipStreamNonBlocking) != hipSuccess) {
      for (int j = 0; j < i; ++j) hipStreamDestroy(s->stream[j]);
      delete s;
      return TC_ERR_HIP;
    }
  }
  s->t0 = Clock::now();
  s->th[0] = std::thread([s] { s->batch_loop(); });
  for (int k = 1; k < 3; ++k) s->th[k] = std::thread([s, k] { s->single_loop(k); });
  *out = s;
  return TC_OK;
}

int tc_serve_submit(tc_server* s, const uint32_t* rowptr, const uint32_t* colidx, uint32_t n,
                    uint64_t m, uint64_t* ticket) {
  if (!s || !ticket || !rowptr || (m > 0 && !colidx)) return TC_ERR_INVALID_ARG;
  if (n >= 0x40000000u || m > tc::kMaxEntries) return TC_ERR_TOO_LARGE;
  if (rowptr[0] != 0 || rowptr[n] != m) return TC_ERR_INVALID_GRAPH;
  Request r{};
  r.rowptr = rowptr;
  r.colidx = colidx;
  r.n = n;
  r.m = m;
  r.footprint = s->footprint(n, m);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return TC_ERR_INVALID_ARG;
  r.ticket = s->next_ticket++;
  r.t_submit = s->now();
  *ticket = r.ticket;
  s->st.submitted += 1;
  if (r.footprint > s->st.hbm_budget) {
    // can never start: completed at once with an error
    s->st.rejected += 1;
    s->st.in_flight += 1;
    r.t_admit = r.t_count = r.t_submit;
    s->finish_locked(r, TC_ERR_OUT_OF_MEMORY, 0, 2);
    return TC_OK;
  }
  s->st.in_flight += 1;
  s->st.queued += 1;
  const int k = s->path_of(m);
  s->ready[k].push_back(r);
  s->cv_path[k].notify_one();
  return TC_OK;
}

int tc_serve_footprint(const tc_server* s, uint32_t n, uint64_t m, uint64_t* bytes) {
  if (!s || !bytes) return TC_ERR_INVALID_ARG;
  if (n >= 0x40000000u || m > tc::kMaxEntries) return TC_ERR_TOO_LARGE;
  *bytes = s->footprint(n, m);
  return TC_OK;
}

int tc_serve_poll(tc_server* s, tc_serve_result* out, uint32_t cap, uint32_t* got,
                  int32_t timeout_ms) {
  if (!s || !got || (cap > 0 && !out)) return TC_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && timeout_ms != 0) {
    auto ready = [&] { return !s->done.empty(); };
    if (timeout_ms < 0) s->cv_done.wait(lk, ready);
    else s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
  }
  uint32_t k = 0;
  while (k < cap && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *got = k;
  return TC_OK;
}

int tc_serve_get_stats(tc_server* s, tc_serve_stats* stats) {
  if (!s || !stats) return TC_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *stats = s->st;
  return TC_OK;
}

int tc_serve_destroy(tc_server* s) {
  if (!s) return TC_ERR_INVALID_ARG;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    // drain: every admitted or waiting request completes before the threads stop
    s->cv_done.wait(lk, [&] { return s->st.in_flight == 0; });
    s->stop = true;
  }
  for (int k = 0; k < 3; ++k) s->cv_path[k].notify_all();
  for (int k = 0; k < 3; ++k) s->th[k].join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (int k = 0; k < 3; ++k) s->free_buf_locked(k);
  }
  for (int k = 0; k < 3; ++k) {
    hipStreamSynchronize(s->stream[k]);
    hipStreamDestroy(s->stream[k]);
  }
  delete s;
  return TC_OK;
}

}  // extern "C"

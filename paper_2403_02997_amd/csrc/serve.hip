// Continuous-batching server over the counting path (declared in include/tc.h).
//
// Requests arrive as HOST CSR arrays.  A request is admitted when its device footprint
// (its CSR plus the scratch its path needs) fits the server's HBM budget; admission is
// first-fit in arrival order, except that while the oldest waiting request does not fit,
// later requests are admitted only if the oldest would still fit beside them, so a large
// request cannot be starved by a stream of small ones.
//
// Admitted requests take one of three paths, each driven by its own host thread and HIP
// stream so that they overlap on the device and a small request never waits behind the
// upload of a large one:
//   batched : at most `small_max_entries` stored entries.  Whenever the previous batch
//             has completed, everything admitted since is packed into one concatenated
//             CSR (uploaded once, resident until its counts are back) and counted by one
//             tc_count_batch launch;
//   medium  : up to `large_min_entries`, one tc_count call each, in arrival order;
//   large   : the rest, one tc_count call each, smallest first (a request that has
//             waited kLargeMaxWait seconds goes next).
// Results carry the request's submit, admit and completion times on the server clock.
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
  double t_submit, t_admit;
};

// The large path serves the smallest admitted request first (by stored entries), so
// a stream of scale-22..24 requests does not queue behind a scale-26 one; a request
// that has waited this long since admission is served next regardless.
constexpr double kLargeMaxWait = 2.0;  // seconds

inline uint64_t csr_bytes(uint32_t n, uint64_t m) { return 4ull * ((uint64_t)n + 1) + 4ull * m; }

// Device bytes a request holds while admitted: its CSR and, on the single-graph path,
// what the tc_count call allocates.
inline uint64_t single_footprint(uint32_t n, uint64_t m) {
  return csr_bytes(n, m) + single_call_bytes(n, m);
}
inline uint64_t batched_footprint(uint32_t n, uint64_t m) {
  return csr_bytes(n, m) + 21ull * ((uint64_t)n + 1) + 8ull * m + 64;
}

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
  std::condition_variable cv_small, cv_single[2], cv_done;
  std::deque<Request> waiting, small_ready, single_ready[2];  // [0] medium, [1] large
  std::deque<tc_serve_result> done;
  tc_serve_stats st{};
  uint64_t next_ticket = 1;
  bool stop = false;

  hipStream_t s_batch = nullptr, s_single[2] = {nullptr, nullptr};
  std::thread th_batch, th_single[2];

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

  // Moves waiting requests that fit into the ready queues.  Caller holds mu.
  void admit_locked() {
    bool woke_small = false, woke_single[2] = {false, false};
    uint64_t head_need = 0;
    for (auto it = waiting.begin(); it != waiting.end();) {
      const uint64_t need = it->footprint + (it == waiting.begin() ? 0 : head_need);
      if (st.hbm_in_use + need <= st.hbm_budget) {
        Request r = *it;
        r.t_admit = now();
        st.hbm_in_use += r.footprint;
        st.hbm_peak = std::max(st.hbm_peak, st.hbm_in_use);
        if (r.m <= cfg.small_max_entries) {
          small_ready.push_back(r);
          woke_small = true;
        } else {
          const int k = r.m >= cfg.large_min_entries ? 1 : 0;
          single_ready[k].push_back(r);
          woke_single[k] = true;
        }
        it = waiting.erase(it);
      } else {
        if (it == waiting.begin()) head_need = it->footprint;
        ++it;
      }
    }
    st.queued = waiting.size();
    if (woke_small) cv_small.notify_one();
    for (int k = 0; k < 2; ++k)
      if (woke_single[k]) cv_single[k].notify_one();
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
    res.done_s = now();
    done.push_back(res);
    st.hbm_in_use -= r.footprint;
    st.in_flight -= 1;
    st.completed += 1;
    admit_locked();
    cv_done.notify_all();
  }

  // ---- batched path ------------------------------------------------------------------
  int run_batch(const std::vector<Request>& b, std::vector<uint64_t>& counts) {
    const uint32_t G = (uint32_t)b.size();
    std::vector<int64_t> row_off(G + 1), col_off(G + 1);
    row_off[0] = col_off[0] = 0;
    for (uint32_t i = 0; i < G; ++i) {
      row_off[i + 1] = row_off[i] + b[i].n + 1;
      col_off[i + 1] = col_off[i] + (int64_t)b[i].m;
    }
    const uint64_t rows = (uint64_t)row_off[G], cols = (uint64_t)col_off[G];
    const size_t ws_bytes = tc_count_batch_workspace_size(G, rows, cols);
    char* dev = nullptr;
    const size_t o_rp = 0;
    const size_t o_ci = (o_rp + 4 * rows + 255) / 256 * 256;
    const size_t o_ro = (o_ci + 4 * cols + 255) / 256 * 256;
    const size_t o_co = (o_ro + 8 * ((size_t)G + 1) + 255) / 256 * 256;
    const size_t o_cnt = (o_co + 8 * ((size_t)G + 1) + 255) / 256 * 256;
    const size_t o_ws = (o_cnt + 8 * (size_t)G + 255) / 256 * 256;
    const size_t total = o_ws + ws_bytes;
    if (hipMallocAsync((void**)&dev, total, s_batch) != hipSuccess) {
      (void)hipGetLastError();
      return TC_ERR_OUT_OF_MEMORY;
    }
    int rc = TC_OK;
    for (uint32_t i = 0; i < G && rc == TC_OK; ++i) {
      if (hipMemcpyAsync(dev + o_rp + 4 * row_off[i], b[i].rowptr, 4ull * (b[i].n + 1),
                         hipMemcpyHostToDevice, s_batch) != hipSuccess)
        rc = TC_ERR_HIP;
      if (rc == TC_OK && b[i].m &&
          hipMemcpyAsync(dev + o_ci + 4 * col_off[i], b[i].colidx, 4ull * b[i].m,
                         hipMemcpyHostToDevice, s_batch) != hipSuccess)
        rc = TC_ERR_HIP;
    }
    if (rc == TC_OK &&
        (hipMemcpyAsync(dev + o_ro, row_off.data(), 8 * ((size_t)G + 1), hipMemcpyHostToDevice,
                        s_batch) != hipSuccess ||
         hipMemcpyAsync(dev + o_co, col_off.data(), 8 * ((size_t)G + 1), hipMemcpyHostToDevice,
                        s_batch) != hipSuccess))
      rc = TC_ERR_HIP;
    if (rc == TC_OK)
      rc = tc_count_batch((const uint32_t*)(dev + o_rp), (const uint32_t*)(dev + o_ci),
                          (const int64_t*)(dev + o_ro), (const int64_t*)(dev + o_co), G, rows,
                          cols, dev + o_ws, ws_bytes, s_batch, (uint64_t*)(dev + o_cnt));
    counts.assign(G, 0);
    if (rc == TC_OK && hipMemcpyAsync(counts.data(), dev + o_cnt, 8 * (size_t)G,
                                      hipMemcpyDeviceToHost, s_batch) != hipSuccess)
      rc = TC_ERR_HIP;
    if (hipFreeAsync(dev, s_batch) != hipSuccess && rc == TC_OK) rc = TC_ERR_HIP;
    if (hipStreamSynchronize(s_batch) != hipSuccess && rc == TC_OK) rc = TC_ERR_HIP;
    (void)hipGetLastError();
    return rc;
  }

  void batch_loop() {
    (void)hipSetDevice(device);
    while (true) {
      std::vector<Request> b;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_small.wait(lk, [&] { return stop || !small_ready.empty(); });
        if (stop) return;
        uint64_t entries = 0;
        while (!small_ready.empty() && b.size() < cfg.batch_max_graphs) {
          const Request& r = small_ready.front();
          if (!b.empty() && entries + r.m > cfg.batch_max_entries) break;
          entries += r.m;
          b.push_back(r);
          small_ready.pop_front();
        }
        st.batches += 1;
      }
      std::vector<Request> bad;
      size_t kept = 0;
      for (size_t i = 0; i < b.size(); ++i) {
        if (host_bounds_ok(b[i])) b[kept++] = b[i];
        else bad.push_back(b[i]);
      }
      b.resize(kept);
      std::vector<uint64_t> counts;
      const int rc = b.empty() ? TC_OK : run_batch(b, counts);
      std::lock_guard<std::mutex> lk(mu);
      for (const Request& r : bad) finish_locked(r, TC_ERR_INVALID_GRAPH, 0, 0);
      for (size_t i = 0; i < b.size(); ++i) finish_locked(b[i], rc, rc == TC_OK ? counts[i] : 0, 0);
    }
  }

  // ---- single-graph path -------------------------------------------------------------
  int run_single(const Request& r, hipStream_t s_single, uint64_t* tri) {
    char* dev = nullptr;
    const size_t o_ci = (4ull * (r.n + 1) + 255) / 256 * 256;
    const size_t o_flag = o_ci + (4ull * std::max<uint64_t>(r.m, 1) + 255) / 256 * 256;
    if (hipMallocAsync((void**)&dev, o_flag + 256, s_single) != hipSuccess) {
      (void)hipGetLastError();
      return TC_ERR_OUT_OF_MEMORY;
    }
    int rc = TC_OK;
    if (hipMemcpyAsync(dev, r.rowptr, 4ull * (r.n + 1), hipMemcpyHostToDevice, s_single) !=
            hipSuccess ||
        (r.m && hipMemcpyAsync(dev + o_ci, r.colidx, 4ull * r.m, hipMemcpyHostToDevice,
                               s_single) != hipSuccess))
      rc = TC_ERR_HIP;
    if (rc == TC_OK) {
      const int b = check_csr_bounds((const uint32_t*)dev, (const uint32_t*)(dev + o_ci), r.n,
                                     (uint32_t)r.m, (uint32_t*)(dev + o_flag), s_single);
      rc = b == 0 ? TC_OK : (b == -4 ? TC_ERR_INVALID_GRAPH : TC_ERR_HIP);
    }
    if (rc == TC_OK)
      rc = tc_count((const uint32_t*)dev, (const uint32_t*)(dev + o_ci), r.n, r.m, s_single, tri);
    if (hipFreeAsync(dev, s_single) != hipSuccess && rc == TC_OK) rc = TC_ERR_HIP;
    if (hipStreamSynchronize(s_single) != hipSuccess && rc == TC_OK) rc = TC_ERR_HIP;
    (void)hipGetLastError();
    return rc;
  }

  void single_loop(int k) {
    (void)hipSetDevice(device);
    set_thread_side_stream(false);  // this thread's stream is one of the server's three
    while (true) {
      Request r;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_single[k].wait(lk, [&] { return stop || !single_ready[k].empty(); });
        if (stop) return;
        std::deque<Request>& q = single_ready[k];
        auto pick = q.begin();
        if (k == 1 && now() - q.front().t_admit < kLargeMaxWait) {
          // shortest first by stored entries, unless the oldest has waited too long
          for (auto it = q.begin(); it != q.end(); ++it)
            if (it->m < pick->m) pick = it;
        }
        r = *pick;
        q.erase(pick);
        st.singles += 1;
      }
      uint64_t tri = 0;
      const int rc = run_single(r, s_single[k], &tri);
      std::lock_guard<std::mutex> lk(mu);
      finish_locked(r, rc, tri, k == 0 ? 1u : 3u);
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
  hipStream_t* streams[3] = {&s->s_batch, &s->s_single[0], &s->s_single[1]};
  for (int i = 0; i < 3; ++i) {
    if (hipStreamCreateWithFlags(streams[i], hipStreamNonBlocking) != hipSuccess) {
      for (int j = 0; j < i; ++j) hipStreamDestroy(*streams[j]);
      delete s;
      return TC_ERR_HIP;
    }
  }
  s->t0 = Clock::now();
  s->th_batch = std::thread([s] { s->batch_loop(); });
  s->th_single[0] = std::thread([s] { s->single_loop(0); });
  s->th_single[1] = std::thread([s] { s->single_loop(1); });
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
  r.footprint = m <= s->cfg.small_max_entries ? batched_footprint(n, m) : single_footprint(n, m);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return TC_ERR_INVALID_ARG;
  r.ticket = s->next_ticket++;
  r.t_submit = s->now();
  *ticket = r.ticket;
  s->st.submitted += 1;
  if (r.footprint > s->st.hbm_budget) {
    // can never be admitted: completed at once with an error
    s->st.rejected += 1;
    s->st.in_flight += 1;
    s->st.hbm_in_use += r.footprint;  // balanced by finish_locked
    r.t_admit = r.t_submit;
    s->finish_locked(r, TC_ERR_OUT_OF_MEMORY, 0, 2);
    return TC_OK;
  }
  s->st.in_flight += 1;
  s->waiting.push_back(r);
  s->admit_locked();
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
  s->cv_small.notify_all();
  for (int k = 0; k < 2; ++k) s->cv_single[k].notify_all();
  s->th_batch.join();
  for (int k = 0; k < 2; ++k) s->th_single[k].join();
  hipStreamDestroy(s->s_batch);
  for (int k = 0; k < 2; ++k) hipStreamDestroy(s->s_single[k]);
  delete s;
  return TC_OK;
}

}  // extern "C"

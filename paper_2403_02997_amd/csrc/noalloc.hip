// Allocation-free batched counting: tc_count_batch_noalloc runs the batched kernels of
// tc_count_batch with their workspace in a fixed device array of this library, for
// callers that cannot allocate device memory (code under HIP graph capture, serving
// loops that forbid allocation after start-up).
//
// `scratch` is a file-scope device array: every GPU the library runs on holds its own
// copy, at its own address, until the process ends.  In host code its name is only a
// stand-in for the symbol, never a device address, so its address on each device is
// looked up once (hipGetSymbolAddress, with that device current) and kept per device;
// the kernels get that address as their workspace argument.  Calls on one GPU share the
// array: calls that overlap in time on one GPU race (the caller serialises them, e.g. by
// issuing them on one stream).  The batched kernels write every workspace word they read
// and reset their own control block, so the array needs no clearing between calls.
#include <mutex>

#include "../../include/tc.h"
#include "host_api.h"
#include "tc_launch.h"

namespace tc {

static_assert(TC_NOALLOC_SCRATCH_BYTES % 256 == 0, "the scratch size is whole 256-byte units");

static __device__ __align__(256) unsigned char scratch[TC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device, once looked up

// Device address of this device's copy of `scratch`, or nullptr on failure.
void* scratch_on_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace tc

using namespace tc;

extern "C" int tc_count_batch_noalloc(const uint32_t* rowptr_cat, const uint32_t* colidx_cat,
                                      const int64_t* row_off, const int64_t* col_off,
                                      uint32_t num_graphs, uint64_t total_rows,
                                      uint64_t total_cols, hipStream_t stream,
                                      uint64_t* counts) {
  if (num_graphs == 0) return TC_OK;
  if (!rowptr_cat || !row_off || !col_off || !counts || total_rows < num_graphs ||
      (total_cols > 0 && !colidx_cat))
    return TC_ERR_INVALID_ARG;
  if (total_cols > kMaxEntries || total_rows > kMaxEntries) return TC_ERR_TOO_LARGE;
  if (batch_workspace_bytes(num_graphs, total_rows, total_cols) > TC_NOALLOC_SCRATCH_BYTES)
    return TC_ERR_TOO_LARGE;
  void* ws = scratch_on_current_device();
  if (!ws) return TC_ERR_HIP;
  launch_batch(rowptr_cat, colidx_cat, row_off, col_off, num_graphs, total_rows, total_cols, ws,
               current_isect_params(), (u64*)counts, stream);
  if (hipGetLastError() != hipSuccess) return TC_ERR_HIP;
  return TC_OK;
}

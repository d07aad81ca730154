// Host-side orchestration shared by the C ABI (api.hip) and the server (serve.hip): no
// kernel and no launch shape is declared here.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace tc {

// Largest number of stored entries (and of concatenated rows or entries in a batch) the
// entry points accept: entry offsets are 32-bit, and the tile arithmetic over them (a
// tile end e0 + 1024, a tile count rounded up) needs headroom below 2^32.
constexpr uint64_t kMaxEntries = 0x100000000ull - 0x100000ull;  // 2^32 - 2^20

// Whether the single-graph path of the calling thread may run the wavefront class and
// the hub count on a second stream (default on).  A thread whose own stream is one of
// several long-lived streams that already fill the device's few hardware queues (the
// server's workers) turns it off, so that no call adds a stream beside them.
void set_thread_side_stream(bool on);

// Device bytes one tc_count call on n vertices and m stored entries allocates (its
// workspace and its workgroup items), under the current settings.
size_t single_call_bytes(uint32_t n, uint64_t m);

// Until called again with base = nullptr, the calling thread's calls take their device
// memory from [base, base + bytes), from the start again at every call of this function,
// instead of allocating it; a call that needs more than is left returns
// TC_ERR_OUT_OF_MEMORY.  The memory must stay valid, and untouched by other work, while
// such calls run; their work is ordered on their own stream.  single_call_bytes(n, m)
// bytes suffice for one tc_count call.
void set_thread_arena(void* base, size_t bytes);

}  // namespace tc

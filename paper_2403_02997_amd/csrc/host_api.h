// Host-side orchestration shared by the C ABI (api.hip) and the server (serve.hip): no
// kernel and no launch shape is declared here.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace tc {

// Whether the single-graph path of the calling thread may run the wavefront class and
// the hub count on a second stream (default on).  A thread whose own stream is one of
// several long-lived streams that already fill the device's few hardware queues (the
// server's workers) turns it off, so that no call adds a stream beside them.
void set_thread_side_stream(bool on);

// Device bytes one tc_count call on n vertices and m stored entries allocates (its
// workspace and its workgroup items), under the current settings.
size_t single_call_bytes(uint32_t n, uint64_t m);

}  // namespace tc

// Local clustering coefficients from per-vertex triangle counts.
//
// The vertex form of the count (Section 2) gives t(v), the triangles through v; the local
// clustering coefficient (Watts and Strogatz; Section 1 names clustering coefficients
// among the uses of triangle counts) is the fraction of v's neighbour pairs that are
// adjacent:
// C(v) = t(v) / C(d(v), 2) = 2 t(v) / (d(v) (d(v) - 1)), and 0 when d(v) < 2.
//
// One thread per vertex, grid-stride; rowptr pairs and t(v) are read coalesced, C(v)
// written coalesced.  2 t(v) and d(v) (d(v) - 1) are exact in double (both below 2^53),
// so the single correctly rounded division makes C(v) a deterministic function of t(v)
// and d(v).
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "../../include/tc.h"

namespace tc {
namespace {

constexpr uint32_t kClusterThreads = 256;
constexpr uint32_t kClusterMaxBlocks = 8192;

__global__ void __launch_bounds__(kClusterThreads)
    k_local_clustering(const uint32_t* __restrict__ rowptr, const uint64_t* __restrict__ tri,
                       uint32_t n, double* __restrict__ cc) {
  const uint32_t stride = gridDim.x * kClusterThreads;
  for (uint32_t v = blockIdx.x * kClusterThreads + threadIdx.x; v < n; v += stride) {
    const uint32_t d = rowptr[v + 1] - rowptr[v];
    double c = 0.0;
    if (d >= 2) c = (2.0 * (double)tri[v]) / ((double)d * (double)(d - 1));
    cc[v] = c;
  }
}

}  // namespace
}  // namespace tc

extern "C" int tc_local_clustering(const uint32_t* rowptr, const uint64_t* tri, uint32_t n,
                                   hipStream_t stream, double* cc_out) {
  if (n >= 0x40000000u) return TC_ERR_TOO_LARGE;
  if (n == 0) return TC_OK;
  if (!rowptr || !tri || !cc_out) return TC_ERR_INVALID_ARG;
  uint32_t blocks = (n + tc::kClusterThreads - 1) / tc::kClusterThreads;
  if (blocks > tc::kClusterMaxBlocks) blocks = tc::kClusterMaxBlocks;
  tc::k_local_clustering<<<blocks, tc::kClusterThreads, 0, stream>>>(rowptr, tri, n, cc_out);
  return hipGetLastError() == hipSuccess ? TC_OK : TC_ERR_HIP;
}

// abx_query_nearest_static: the nearest query of abx_query_nearest for
// callers that cannot allocate (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).  Its scratch is the file-scope device
// array `scratch` below, one copy per GPU, created when the code object is
// loaded on that GPU and held until the process ends.  Host code never uses
// the array's name as an address: the device address of each GPU's copy is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and passed to the kernels like the caller's scratch of the plain entry
// point.  Every call on one GPU shares that GPU's copy.
#include <mutex>

#include "abx_internal.h"

static __device__ __align__(256) char scratch[ABX_STATIC_SCRATCH_BYTES];

namespace abx {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device (null: not looked up)

// the current device's copy of `scratch`
abx_status static_scratch(void **out) {
  int dev = 0;
  ABX_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return ABX_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    ABX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return ABX_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ABX_OK;
}

}  // namespace
}  // namespace abx

extern "C" abx_status abx_query_nearest_static(const abx_bvh *bvh, const float *points, int64_t m,
                                               int32_t k, int32_t sort_queries, int32_t *offsets,
                                               int32_t *indices, float *distances,
                                               abx_stream_t stream) {
  using namespace abx;
  size_t need = 0;
  ABX_TRY(abx_query_nearest_sizes(bvh, m, k, &need));
  if (need > ABX_STATIC_SCRATCH_BYTES) return ABX_ERR_CAPACITY;
  void *ptr = nullptr;
  ABX_TRY(static_scratch(&ptr));
  // no event objects either: timing stays off for these launches
  const NoEventsScope no_events;
  return abx_query_nearest(bvh, points, m, k, sort_queries, ptr, ABX_STATIC_SCRATCH_BYTES, offsets,
                           indices, distances, stream);
}

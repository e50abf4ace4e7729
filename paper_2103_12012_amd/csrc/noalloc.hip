// noalloc.hip -- sssp_solve_noalloc: sssp_solve with its workspace in a
// fixed device array of the library instead of a caller-supplied buffer, for
// callers that cannot allocate device memory at call time.
//
// The array is a file-scope __device__ variable, so every GPU the library
// runs on holds its own copy from module load until the process ends.  Its
// device address is taken once per device with hipGetSymbolAddress (the
// variable's name in host code is only a host-side stand-in, never a device
// address) and that address is what the kernels receive.  Every call on one
// GPU shares that GPU's array: calls that overlap on one GPU (different
// streams, or host threads) race on it and must be ordered by the caller.
// Nothing in the array has to start at zero: the solve's own init kernels
// clear the control block, the unit tables, the labels and the inboxes of
// every call.
#include <mutex>

#include "internal.hpp"

namespace sssp_impl {

static __device__ __align__(256) unsigned char scratch[SSSP_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_scratch[MAX_DEVICES] = {};

// Device address of this device's copy of `scratch` (taken on the first
// call on the device, with it current), or NULL on a HIP error.
void *scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}
}  // namespace

}  // namespace sssp_impl

extern "C" int sssp_solve_noalloc(const sssp_csr *g, int32_t source, const sssp_opts *o,
                                  void *dist, int32_t *pred, int32_t *pred_edge,
                                  sssp_stats *stats, void *stream) {
  // the workspace this solve needs (host-side query: nothing is enqueued)
  size_t need = 0;
  int rc = sssp_solve(g, source, o, nullptr, nullptr, nullptr, nullptr, nullptr, &need, stream);
  if (rc) return rc;
  if (need > (size_t)SSSP_NOALLOC_SCRATCH_BYTES) return SSSP_ERR_TOO_LARGE;
  void *ws = sssp_impl::scratch_ptr();
  if (!ws) return SSSP_ERR_HIP;
  size_t have = (size_t)SSSP_NOALLOC_SCRATCH_BYTES;
  return sssp_solve(g, source, o, dist, pred, pred_edge, stats, ws, &have, stream);
}

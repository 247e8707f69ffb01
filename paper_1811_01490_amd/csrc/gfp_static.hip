// gfp_fft_noalloc: the forward or inverse transform with its two work vectors
// in a file-scope device array instead of a caller workspace or an
// allocation, for callers that cannot allocate device memory (graph
// capture, serving loops, harnesses that forbid hipMalloc).
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is resolved once per device with hipGetSymbolAddress (with
// that device current) and kept in g_scratch[device]; only that pointer is
// ever handed to kernels or copies.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <mutex>

#include "../../include/gfp.h"
#include "gfp_internal.hpp"

static __device__ __align__(256) uint64_t scratch[GFP_STATIC_SCRATCH_BYTES / sizeof(uint64_t)];

namespace {

constexpr int kMaxDevices = 64;
std::atomic<void*> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// The current device's copy of `scratch` (a status code of gfp.h).
int scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return GFP_EDEVICE;
  if (dev >= kMaxDevices) return GFP_EUNSUPPORTED;
  void* p = g_scratch[dev].load(std::memory_order_acquire);
  if (!p) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    p = g_scratch[dev].load(std::memory_order_relaxed);
    if (!p) {
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GFP_EDEVICE;
      g_scratch[dev].store(p, std::memory_order_release);
    }
  }
  *out = p;
  return GFP_OK;
}

}  // namespace

extern "C" int gfp_fft_noalloc(const gfp_field* f, uint64_t n, int inverse, const uint64_t* x, uint64_t ld_x,
                               uint64_t* y, uint64_t ld_y, void* stream) {
  if (!f || !x || !y) return GFP_EINVAL;
  void* p = nullptr;
  const int rc = scratch_ptr(&p);
  if (rc != GFP_OK) return rc;
  return gfpk::transform_noalloc(f, n, inverse, x, ld_x, y, ld_y, p, GFP_STATIC_SCRATCH_BYTES, stream);
}

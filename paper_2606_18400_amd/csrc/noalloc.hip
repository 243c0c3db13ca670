// cloak_mlp_noalloc: the cloaked SwiGLU FFN (cloak_mlp) for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid allocation).  Its workspace (the hidden
// activations and the split-K partial sums) lives in one file-scope device
// array of kScratchBytes per GPU, held until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device with hipGetSymbolAddress and
// only that address is ever handed to kernels.

#include <hip/hip_runtime.h>

#include <mutex>

#include "cloak_internal.hpp"

constexpr uint64_t kScratchBytes = CLOAK_MLP_NOALLOC_MAX_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (looked up on the first
// call with that device current).
int scratch_ptr(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    cloak::set_error("cloak_mlp_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    return CLOAK_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    cloak::set_error("cloak_mlp_noalloc: device %d beyond the %d this library tracks", dev, kMaxDevices);
    return CLOAK_EINVAL;
  }
  std::lock_guard<std::mutex> g(g_lock);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      cloak::set_error("cloak_mlp_noalloc: hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return CLOAK_EHIP;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return CLOAK_OK;
}

}  // namespace

extern "C" int cloak_mlp_noalloc(const cloak_layout* L, const void* d_pool, int32_t layer, const void* d_x, int64_t M,
                                 void* d_y, void* stream) {
  cloak::clear_error();
  if (!L) {
    cloak::set_error("cloak_mlp_noalloc: null layout");
    return CLOAK_EINVAL;
  }
  if (M == 0) return cloak_mlp(L, d_pool, layer, d_x, M, d_y, nullptr, 0, stream);
  const uint64_t need = cloak_mlp_ws_bytes(L, layer, M);
  if (need == UINT64_MAX) {
    cloak::set_error("cloak_mlp_noalloc: bad layer %d or M=%lld", layer, (long long)M);
    return CLOAK_EINVAL;
  }
  if (need > kScratchBytes) {
    cloak::set_error("cloak_mlp_noalloc: M=%lld needs %llu bytes of workspace, above the static %llu; use cloak_mlp",
                     (long long)M, (unsigned long long)need, (unsigned long long)kScratchBytes);
    return CLOAK_EINVAL;
  }
  void* ws = nullptr;
  if (int rc = scratch_ptr(&ws)) return rc;
  return cloak_mlp(L, d_pool, layer, d_x, M, d_y, ws, kScratchBytes, stream);
}

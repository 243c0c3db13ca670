// Hardware-translated twin of a cloaked pool.
//
// CloakLM itself keeps kernels unmodified and lets the GPU's MMU resolve the
// shuffled placement: physical pages are mapped into the model's virtual
// range in the seeded order (arXiv 2606.18400, Section 4.2, paragraph on
// physical page remapping, built on the GPU's virtual memory management API).  This
// file builds that arrangement on MI355X for an A/B against the in-kernel
// translation of the rest of the library: every physical page of the pool is
// its own VMM allocation, mapped twice,
//   * in physical order (the pool view: cloak_load, cloak_pool_init and the
//     remap's page swaps use it exactly like a caller-owned pool), and
//   * in virtual order, virtual page v backed by physical page phi[v] (the
//     tensor view: the weight-reading kernels run untranslated on it, so the
//     MMU does the page-map lookups).
// A remap swaps page contents through the pool view, waits for the stream,
// then re-points the two virtual pages of every swapped pair.

#include <hip/hip_runtime.h>

#include <cstring>

#include "cloak.h"
#include "cloak_internal.hpp"

using namespace cloak;

namespace {

hipMemAllocationProp page_prop(int device) {
  hipMemAllocationProp prop;
  std::memset(&prop, 0, sizeof(prop));
  prop.type = hipMemAllocationTypePinned;
  prop.location.type = hipMemLocationTypeDevice;
  prop.location.id = device;
  return prop;
}

hipError_t grant(void* ptr, size_t bytes, int device) {
  hipMemAccessDesc acc;
  std::memset(&acc, 0, sizeof(acc));
  acc.location.type = hipMemLocationTypeDevice;
  acc.location.id = device;
  acc.flags = hipMemAccessFlagsProtReadWrite;
  return hipMemSetAccess(ptr, bytes, &acc, 1);
}

uint8_t* at(void* base, int64_t page, int64_t page_bytes) { return static_cast<uint8_t*>(base) + page * page_bytes; }

// Undo whatever part of the twin exists (mappings, reservations, handles).
void release(cloak_layout* L) {
  VmmState& v = L->vmm;
  const size_t bytes = size_t(L->P) * size_t(L->page_bytes);
  if (v.tensor_view) {
    for (int64_t p = 0; p < L->P; ++p) (void)hipMemUnmap(at(v.tensor_view, p, L->page_bytes), size_t(L->page_bytes));
    (void)hipMemAddressFree(v.tensor_view, bytes);
  }
  if (v.pool_view) {
    for (int64_t p = 0; p < L->P; ++p) (void)hipMemUnmap(at(v.pool_view, p, L->page_bytes), size_t(L->page_bytes));
    (void)hipMemAddressFree(v.pool_view, bytes);
  }
  for (void* h : v.handles)
    if (h) (void)hipMemRelease(static_cast<hipMemGenericAllocationHandle_t>(h));
  v = VmmState{};
}

}  // namespace

namespace cloak {

// Re-point virtual pages va -> physical b and vb -> physical a (the pair
// (a, b) has just swapped contents).  Called with the stream drained.
hipError_t vmm_repoint(cloak_layout* L, int32_t va, int32_t vb, int32_t a, int32_t b) {
  VmmState& v = L->vmm;
  const size_t B = size_t(L->page_bytes);
  const int32_t virt[2] = {va, vb};
  const int32_t phys[2] = {b, a};
  for (int i = 0; i < 2; ++i) {
    void* va_ptr = at(v.tensor_view, virt[i], L->page_bytes);
    hipError_t e = hipMemUnmap(va_ptr, B);
    if (e != hipSuccess) return e;
    e = hipMemMap(va_ptr, B, 0, static_cast<hipMemGenericAllocationHandle_t>(v.handles[size_t(phys[i])]), 0);
    if (e != hipSuccess) return e;
    e = grant(va_ptr, B, v.device);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace cloak

extern "C" int cloak_vmm_pool_create(cloak_layout* L, void** d_pool_view) {
  clear_error();
  if (!L || !d_pool_view) {
    set_error("cloak_vmm_pool_create: null argument");
    return CLOAK_EINVAL;
  }
  if (L->dev.device < 0) {
    set_error("cloak_vmm_pool_create: call cloak_layout_to_device first");
    return CLOAK_ESTATE;
  }
  if (L->native() || L->vmm.active || L->epoch.active) {
    set_error("cloak_vmm_pool_create: needs a cloaked layout without a VMM pool or a remap in progress");
    return CLOAK_ESTATE;
  }
  int dev = 0, supported = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&supported, hipDeviceAttributeVirtualMemoryManagementSupported, dev) != hipSuccess ||
      !supported) {
    set_error("cloak_vmm_pool_create: virtual memory management is not supported on this device");
    return CLOAK_ESTATE;
  }
  hipMemAllocationProp prop = page_prop(dev);
  size_t gran = 0;
  if (hipMemGetAllocationGranularity(&gran, &prop, hipMemAllocationGranularityMinimum) != hipSuccess || gran == 0 ||
      uint64_t(L->page_bytes) % gran != 0) {
    set_error("cloak_vmm_pool_create: page_bytes %lld is not a multiple of the allocation granularity %zu",
              (long long)L->page_bytes, gran);
    return CLOAK_EINVAL;
  }
  VmmState& v = L->vmm;
  v.device = dev;
  const size_t B = size_t(L->page_bytes), bytes = size_t(L->P) * B;
  hipError_t e = hipMemAddressReserve(&v.pool_view, bytes, B, nullptr, 0);
  if (e == hipSuccess) e = hipMemAddressReserve(&v.tensor_view, bytes, B, nullptr, 0);
  v.handles.assign(size_t(L->P), nullptr);
  for (int64_t p = 0; e == hipSuccess && p < L->P; ++p) {
    hipMemGenericAllocationHandle_t h{};
    e = hipMemCreate(&h, B, &prop, 0);
    if (e != hipSuccess) break;
    v.handles[size_t(p)] = h;
    e = hipMemMap(at(v.pool_view, p, L->page_bytes), B, 0, h, 0);
  }
  // virtual page v is backed by physical page phi[v]
  for (int64_t vp = 0; e == hipSuccess && vp < L->P; ++vp)
    e = hipMemMap(at(v.tensor_view, vp, L->page_bytes), B, 0,
                  static_cast<hipMemGenericAllocationHandle_t>(v.handles[size_t(L->phi[vp])]), 0);
  if (e == hipSuccess) e = grant(v.pool_view, bytes, dev);
  if (e == hipSuccess) e = grant(v.tensor_view, bytes, dev);
  if (e != hipSuccess) {
    set_error("cloak_vmm_pool_create: %s", hipGetErrorString(e));
    release(L);
    return CLOAK_EHIP;
  }
  v.active = true;
  *d_pool_view = v.pool_view;
  return CLOAK_OK;
}

extern "C" int cloak_vmm_pool_free(cloak_layout* L) {
  clear_error();
  if (!L) {
    set_error("cloak_vmm_pool_free: null layout");
    return CLOAK_EINVAL;
  }
  if (!L->vmm.active) return CLOAK_OK;
  (void)hipDeviceSynchronize();
  release(L);
  return CLOAK_OK;
}

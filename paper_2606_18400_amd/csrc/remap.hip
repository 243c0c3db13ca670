// In-place page-pair swap behind cloak_remap (CloakLM, arXiv 2606.18400,
// Section 4.2: periodic re-randomisation of page placement with no extra
// memory footprint).  The matching is drawn on the host; here every pair of
// physical pages exchanges its contents through registers, so each pool byte
// is read once and written once and no scratch page exists.
//
// A workgroup owns a 16 KiB slice of one pair (both pages at the same
// offset): each lane loads its 16 B pieces of both pages first, then stores
// them crosswise.  Pairs are disjoint, so no two lanes touch the same byte.

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace cloak {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kVecPerThread = 4;
constexpr int64_t kSlice = int64_t(kThreads) * kVecPerThread * 16;  // 16 KiB

__global__ __launch_bounds__(kThreads) void swap_pages_kernel(const SwapArgs a) {
  const int64_t page_bytes = int64_t(1) << a.log2_page;
  const int64_t slice = page_bytes < kSlice ? page_bytes : kSlice;
  const int64_t slices_per_pair = page_bytes / slice;
  const int64_t pair = int64_t(blockIdx.x) / slices_per_pair;
  const int64_t sl = int64_t(blockIdx.x) % slices_per_pair;
  if (pair >= a.npairs) return;
  const int64_t pa = a.pairs[2 * pair];
  const int64_t pb = a.pairs[2 * pair + 1];
  u32x4* A = reinterpret_cast<u32x4*>(a.pool + (pa << a.log2_page) + sl * slice);
  u32x4* B = reinterpret_cast<u32x4*>(a.pool + (pb << a.log2_page) + sl * slice);
  const int nvec = int(slice / 16);
  u32x4 va[kVecPerThread], vb[kVecPerThread];
#pragma unroll
  for (int u = 0; u < kVecPerThread; ++u) {
    const int i = threadIdx.x + u * kThreads;
    if (i < nvec) {
      va[u] = __builtin_nontemporal_load(A + i);
      vb[u] = __builtin_nontemporal_load(B + i);
    }
  }
#pragma unroll
  for (int u = 0; u < kVecPerThread; ++u) {
    const int i = threadIdx.x + u * kThreads;
    if (i < nvec) {
      __builtin_nontemporal_store(vb[u], A + i);
      __builtin_nontemporal_store(va[u], B + i);
    }
  }
}

}  // namespace

hipError_t launch_swap(const SwapArgs& a, hipStream_t s) {
  if (a.npairs <= 0) return hipSuccess;
  const int64_t page_bytes = int64_t(1) << a.log2_page;
  const int64_t slice = page_bytes < kSlice ? page_bytes : kSlice;
  const int64_t blocks = a.npairs * (page_bytes / slice);
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(swap_pages_kernel, dim3(unsigned(blocks)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace cloak

// In-place page-pair swap behind cloak_remap (CloakLM, arXiv 2606.18400,
// Section 4.2: periodic re-randomisation of page placement with no extra
// memory footprint).  The matching is drawn on the host; here every pair of
// physical pages exchanges its contents through registers, so each pool byte
// is read once and written once and no scratch page exists.
//
// A workgroup owns a 16 KiB slice of one pair (both pages at the same
// offset): each lane loads its 16 B pieces of both pages first, then stores
// them crosswise.  Pairs are disjoint, so no two lanes touch the same byte.
//
// The same file fills the free pages with decoys: weight-like values from a
// counter-based SplitMix64 stream keyed by a seed of their own (definition
// in include/cloak.h), so pages without weights do not stand out as zeros.

#include <hip/hip_runtime.h>

#include "cloak.h"
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

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// C = 2S - 786420, S the sum of the twelve 16-bit pieces of stream outputs
// 3e .. 3e+2 (output j is mix64(s0 + (j+1) * gamma)).
__device__ inline int32_t centred_sum(uint64_t s0, uint64_t e) {
  uint32_t sum = 0;
#pragma unroll
  for (int w = 0; w < 3; ++w) {
    const uint64_t r = mix64(s0 + (3 * e + uint64_t(w) + 1) * kGamma);
    const uint32_t lo = uint32_t(r), hi = uint32_t(r >> 32);
    sum += (lo & 0xffffu) + (lo >> 16) + (hi & 0xffffu) + (hi >> 16);
  }
  return 2 * int32_t(sum) - 786420;
}

// One lane writes 16 bytes: 4 f32, 8 bf16 or 16 E4M3 elements.
__global__ __launch_bounds__(kThreads) void decoy_kernel(const DecoyArgs a) {
  const int64_t page_bytes = int64_t(1) << a.log2_page;
  const int64_t slice = page_bytes < kSlice ? page_bytes : kSlice;
  const int64_t slices_per_page = page_bytes / slice;
  const int64_t i = int64_t(blockIdx.x) / slices_per_page;
  if (i >= a.nfree) return;
  const int64_t v = a.V + i;
  const int64_t byte0 = (int64_t(blockIdx.x) % slices_per_page) * slice;
  const uint64_t s0 = mix64(a.decoy_seed ^ mix64((uint64_t(7) << 32) | uint64_t(uint32_t(v))));
  const int64_t phys = int64_t(uint32_t(a.phi[v]) ^ phi_mask(a.phi_key, v));
  u32x4* dst = reinterpret_cast<u32x4*>(a.pool + (phys << a.log2_page) + byte0);
  const int nvec = int(slice / 16);
  for (int u = 0; u < kVecPerThread; ++u) {
    const int q = threadIdx.x + u * kThreads;
    if (q >= nvec) break;
    const int64_t off = byte0 + int64_t(q) * 16;
    uint32_t word[4];
    if (a.dtype == CLOAK_F32) {
      for (int k = 0; k < 4; ++k)
        word[k] = __float_as_uint(float(centred_sum(s0, uint64_t(off / 4 + k)) * 5) * 0x1p-25f);
    } else if (a.dtype == CLOAK_BF16) {
      for (int k = 0; k < 4; ++k) {
        uint32_t h[2];
        for (int j = 0; j < 2; ++j) {
          const uint32_t b = __float_as_uint(float(centred_sum(s0, uint64_t(off / 2 + 2 * k + j)) * 5) * 0x1p-25f);
          h[j] = (b + 0x7fffu + ((b >> 16) & 1u)) >> 16;   // nearest even (finite values only)
        }
        word[k] = h[0] | (h[1] << 16);
      }
    } else {
      for (int k = 0; k < 4; ++k) {
        uint32_t w = 0;
        for (int j = 0; j < 4; ++j)
          w |= e4m3_code(float(centred_sum(s0, uint64_t(off + 4 * k + j)) * 3) * 0x1p-12f) << (8 * j);
        word[k] = w;
      }
    }
    u32x4 out;
    out.x = word[0];
    out.y = word[1];
    out.z = word[2];
    out.w = word[3];
    dst[q] = out;
  }
}

// Streaming read for bandwidth calibration: every 16-byte word of the buffer
// is loaded once (non-temporal, 8 loads in flight per lane) and folded into a
// value that is stored only if it matches a constant, which keeps the loads.
__global__ __launch_bounds__(256) void stream_read_kernel(const u32x4* __restrict__ p, int64_t n, uint32_t* out) {
  constexpr int U = 8;
  uint32_t acc = 0;
  const int64_t stride = int64_t(gridDim.x) * 256 * U;
  for (int64_t base = int64_t(blockIdx.x) * 256 * U + threadIdx.x; base < n; base += stride) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + int64_t(u) * 256;
      v[u] = i < n ? __builtin_nontemporal_load(p + i) : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  if (acc == 0x9E3779B9u) out[0] = acc;
}

}  // namespace

hipError_t launch_stream_read(const void* src, int64_t bytes, uint32_t* out, hipStream_t s) {
  if (bytes <= 0) return hipSuccess;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(stream_read_kernel, dim3(unsigned(8 * (cus > 0 ? cus : 256))), dim3(256), 0, s,
                     static_cast<const u32x4*>(src), bytes / 16, out);
  return hipGetLastError();
}

hipError_t launch_decoy(const DecoyArgs& a, hipStream_t s) {
  if (a.nfree <= 0) return hipSuccess;
  const int64_t page_bytes = int64_t(1) << a.log2_page;
  const int64_t slice = page_bytes < kSlice ? page_bytes : kSlice;
  const int64_t blocks = a.nfree * (page_bytes / slice);
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(decoy_kernel, dim3(unsigned(blocks)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

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

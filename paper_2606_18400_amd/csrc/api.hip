// Device-facing C-ABI entry points of libcloak: device tables, upload and
// read-back of cloaked tensors, the cloaked linear / FFN launches and the
// in-place remap (CloakLM, arXiv 2606.18400, Sections 4.2 and 5).

#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "cloak_internal.hpp"
#include "kernels.hpp"

using namespace cloak;

#define HIP_TRY(expr, what)                                        \
  do {                                                             \
    hipError_t e_ = (expr);                                        \
    if (e_ != hipSuccess) {                                        \
      set_error("%s: %s", what, hipGetErrorString(e_));            \
      return CLOAK_EHIP;                                           \
    }                                                              \
  } while (0)

namespace {

constexpr int kRingSlots = 4;

struct Ring {
  uint8_t* host = nullptr;
  hipEvent_t ev[kRingSlots] = {};
  int64_t slot_bytes = 0;
};

// Pinned staging ring used by load/unload; cached per layout.
std::vector<std::pair<const cloak_layout*, Ring>>& rings() {
  static std::vector<std::pair<const cloak_layout*, Ring>> r;
  return r;
}

int get_ring(const cloak_layout* L, Ring** out) {
  for (auto& e : rings())
    if (e.first == L) {
      *out = &e.second;
      return CLOAK_OK;
    }
  Ring r;
  r.slot_bytes = L->page_bytes;
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&r.host), size_t(r.slot_bytes) * kRingSlots, hipHostMallocDefault),
          "hipHostMalloc(staging ring)");
  for (int i = 0; i < kRingSlots; ++i) HIP_TRY(hipEventCreateWithFlags(&r.ev[i], hipEventDisableTiming), "hipEventCreate");
  rings().emplace_back(L, r);
  *out = &rings().back().second;
  return CLOAK_OK;
}

void drop_ring(const cloak_layout* L) {
  auto& rs = rings();
  for (size_t i = 0; i < rs.size(); ++i) {
    if (rs[i].first == L) {
      for (int s = 0; s < kRingSlots; ++s)
        if (rs[i].second.ev[s]) (void)hipEventDestroy(rs[i].second.ev[s]);
      if (rs[i].second.host) (void)hipHostFree(rs[i].second.host);
      rs.erase(rs.begin() + long(i));
      return;
    }
  }
}

int check_device_state(const cloak_layout* L, const char* fn) {
  if (!L) {
    set_error("%s: null layout", fn);
    return CLOAK_EINVAL;
  }
  if (!L->dev.phi) {
    set_error("%s: cloak_layout_to_device() has not been called", fn);
    return CLOAK_ESTATE;
  }
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev != L->dev.device) {
    set_error("%s: layout lives on device %d, current device is %d", fn, L->dev.device, dev);
    return CLOAK_ESTATE;
  }
  return CLOAK_OK;
}

int check_pool(const cloak_layout* L, const void* pool, const char* fn) {
  if (!pool) {
    set_error("%s: null pool", fn);
    return CLOAK_EINVAL;
  }
  if (reinterpret_cast<uintptr_t>(pool) % 256 != 0) {
    set_error("%s: pool must be 256-byte aligned", fn);
    return CLOAK_EINVAL;
  }
  (void)L;
  return CLOAK_OK;
}

int wtype_of(int32_t dtype) { return dtype == CLOAK_F32 ? kF32 : dtype == CLOAK_BF16 ? kBF16 : kFP8; }

int mtile_for(int64_t M, int cap) {
  const int t = M <= 1 ? 1 : M <= 2 ? 2 : M <= 4 ? 4 : 8;
  return t < cap ? t : cap;
}

WSeg make_seg(const cloak_layout* L, int32_t t, bool scatter, int32_t row0, int32_t out_off) {
  const TensorInfo& ti = L->tensors[t];
  WSeg s{};
  s.vbase = ti.vbase;
  s.npages = ti.npages;
  s.out_perm = nullptr;
  if (scatter && ti.perm_layer >= 0 && is_row_permuted(ti.shape.kind))
    s.out_perm = L->dev.perms + L->ffn[ti.perm_layer].dev_off;
  s.scale = ti.shape.dtype == CLOAK_FP8_E4M3 ? L->dev.scales + ti.scale_off : nullptr;
  s.rows = int32_t(ti.shape.n_out);
  s.row0 = row0;
  s.out_off = out_off;
  return s;
}

// Runs `a` over every token block of M (each launch handles mtile tokens).
int run_gemv(const cloak_layout* L, GemvArgs a, int wtype, int64_t M, hipStream_t st, const char* fn) {
  const int mt = mtile_for(M, gemv_max_tokens(wtype, a.nchunks));
  for (int64_t m0 = 0; m0 < M; m0 += mt) {
    a.m0 = int32_t(m0);
    a.mcount = int32_t(M - m0 < mt ? M - m0 : mt);
    HIP_TRY(launch_gemv(a, wtype, mt, !L->native(), st), fn);
  }
  return CLOAK_OK;
}

bool use_gemm(int32_t dtype, int64_t K, int64_t M) {
  return dtype == CLOAK_BF16 && M >= kGemmMinTokens && K % gemm_k_step() == 0;
}

void fill_gemm(const cloak_layout* L, const void* pool, GemmArgs& g, int64_t K, int64_t M) {
  g.pool = static_cast<const uint8_t*>(pool);
  g.phi = L->dev.phi;
  g.log2_page = L->log2_page;
  g.K = int32_t(K);
  g.row_bytes = K * 2;
  g.M = int32_t(M);
  g.tiles_m = int32_t((M + gemm_tile_rows() - 1) / gemm_tile_rows());
}

void fill_common(const cloak_layout* L, const void* pool, GemvArgs& a, int64_t K, int elt) {
  a.pool = static_cast<const uint8_t*>(pool);
  a.phi = L->dev.phi;
  a.log2_page = L->log2_page;
  a.row_bytes = int32_t(K * elt);
  a.K = int32_t(K);
  a.nchunks = int32_t((K * elt + 1023) / 1024);
}

}  // namespace

extern "C" int cloak_layout_to_device(cloak_layout* L, void* stream) {
  clear_error();
  if (!L) {
    set_error("cloak_layout_to_device: null layout");
    return CLOAK_EINVAL;
  }
  if (L->dev.phi) return CLOAK_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  DeviceTables d;
  HIP_TRY(hipGetDevice(&d.device), "hipGetDevice");
  const size_t P = size_t(L->P);
  HIP_TRY(hipMalloc(&d.phi, P * 4), "hipMalloc(page map)");
  HIP_TRY(hipMalloc(&d.perms, size_t(L->n_perm > 0 ? L->n_perm : 1) * 4), "hipMalloc(permutations)");
  HIP_TRY(hipMalloc(&d.scales, size_t(L->n_scales > 0 ? L->n_scales : 1) * 4), "hipMalloc(scales)");
  HIP_TRY(hipMalloc(&d.remap_pairs, P * 4 + 4), "hipMalloc(remap pairs)");
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&d.h_stage), P * 8 + 8, hipHostMallocDefault), "hipHostMalloc");
  hipEvent_t ev;
  HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
  d.stage_event = ev;
  std::vector<int32_t> perms(size_t(L->n_perm > 0 ? L->n_perm : 1), 0);
  for (const auto& f : L->ffn) std::memcpy(perms.data() + f.dev_off, f.pi.data(), size_t(f.d_ffn) * 4);
  HIP_TRY(hipMemcpyAsync(d.phi, L->phi.data(), P * 4, hipMemcpyHostToDevice, st), "upload page map");
  HIP_TRY(hipMemcpyAsync(d.perms, perms.data(), perms.size() * 4, hipMemcpyHostToDevice, st), "upload permutations");
  HIP_TRY(hipMemsetAsync(d.scales, 0, size_t(L->n_scales > 0 ? L->n_scales : 1) * 4, st), "clear scales");
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  L->dev = d;
  return CLOAK_OK;
}

extern "C" int cloak_layout_free(cloak_layout* L) {
  clear_error();
  if (!L) return CLOAK_OK;
  drop_ring(L);
  if (L->dev.phi) {
    (void)hipFree(L->dev.phi);
    (void)hipFree(L->dev.perms);
    (void)hipFree(L->dev.scales);
    (void)hipFree(L->dev.remap_pairs);
    (void)hipHostFree(L->dev.h_stage);
    (void)hipEventDestroy(static_cast<hipEvent_t>(L->dev.stage_event));
  }
  delete L;
  return CLOAK_OK;
}

extern "C" int cloak_pool_init(const cloak_layout* L, void* d_pool, void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_pool_init")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_pool_init")) return rc;
  HIP_TRY(hipMemsetAsync(d_pool, 0, size_t(L->pool_bytes), static_cast<hipStream_t>(stream)), "hipMemsetAsync(pool)");
  return CLOAK_OK;
}

extern "C" int cloak_load(cloak_layout* L, void* d_pool, int32_t tensor, const void* h_src, const float* h_scales,
                          void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_load")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_load")) return rc;
  if (tensor < 0 || tensor >= int32_t(L->tensors.size()) || !h_src) {
    set_error("cloak_load: bad tensor index %d or null source", tensor);
    return CLOAK_EINVAL;
  }
  const TensorInfo& ti = L->tensors[tensor];
  const bool fp8 = ti.shape.dtype == CLOAK_FP8_E4M3;
  if (fp8 != (h_scales != nullptr)) {
    set_error("cloak_load: FP8 tensors need scales, other dtypes must pass NULL");
    return CLOAK_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  Ring* ring = nullptr;
  if (int rc = get_ring(L, &ring)) return rc;
  const int64_t B = L->page_bytes;
  const auto order = upload_order(L, tensor);
  for (size_t k = 0; k < order.size(); ++k) {
    const int slot = int(k % kRingSlots);
    if (k >= size_t(kRingSlots)) HIP_TRY(hipEventSynchronize(ring->ev[slot]), "hipEventSynchronize");
    uint8_t* stage = ring->host + int64_t(slot) * ring->slot_bytes;
    const int64_t v = order[k];
    stream_page(L, tensor, static_cast<const uint8_t*>(h_src), v, stage);
    uint8_t* dst = static_cast<uint8_t*>(d_pool) + int64_t(L->phi[ti.vbase + v]) * B;
    HIP_TRY(hipMemcpyAsync(dst, stage, size_t(B), hipMemcpyHostToDevice, st), "hipMemcpyAsync(page)");
    HIP_TRY(hipEventRecord(ring->ev[slot], st), "hipEventRecord");
  }
  std::vector<float> s;  // must outlive the copy below (synchronised at the end)
  if (fp8) {
    // scales follow their rows: stored row j of gate/up carries s[pi[j]]
    s.resize(size_t(ti.shape.n_out));
    const int32_t* pi = (ti.perm_layer >= 0 && is_row_permuted(ti.shape.kind)) ? L->ffn[ti.perm_layer].pi.data() : nullptr;
    for (int64_t j = 0; j < ti.shape.n_out; ++j) s[j] = h_scales[pi ? pi[j] : j];
    HIP_TRY(hipMemcpyAsync(L->dev.scales + ti.scale_off, s.data(), s.size() * 4, hipMemcpyHostToDevice, st),
            "upload scales");
  }
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  return CLOAK_OK;
}

extern "C" int cloak_unload(const cloak_layout* L, const void* d_pool, int32_t tensor, void* h_dst, void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_unload")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_unload")) return rc;
  if (tensor < 0 || tensor >= int32_t(L->tensors.size()) || !h_dst) {
    set_error("cloak_unload: bad tensor index %d or null destination", tensor);
    return CLOAK_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  Ring* ring = nullptr;
  if (int rc = get_ring(L, &ring)) return rc;
  const TensorInfo& ti = L->tensors[tensor];
  const int64_t B = L->page_bytes;
  int64_t pending[kRingSlots];
  for (int s = 0; s < kRingSlots; ++s) pending[s] = -1;
  // pages flow through the ring in order: copy k+kRingSlots is issued only
  // after page k has been copied out of its slot
  for (int64_t v = 0; v < ti.npages + kRingSlots; ++v) {
    const int slot = int(v % kRingSlots);
    uint8_t* stage = ring->host + int64_t(slot) * ring->slot_bytes;
    if (pending[slot] >= 0) {
      HIP_TRY(hipEventSynchronize(ring->ev[slot]), "hipEventSynchronize");
      unstream_page(L, tensor, stage, pending[slot], static_cast<uint8_t*>(h_dst));
      pending[slot] = -1;
    }
    if (v < ti.npages) {
      const uint8_t* src = static_cast<const uint8_t*>(d_pool) + int64_t(L->phi[ti.vbase + v]) * B;
      HIP_TRY(hipMemcpyAsync(stage, src, size_t(B), hipMemcpyDeviceToHost, st), "hipMemcpyAsync(page)");
      HIP_TRY(hipEventRecord(ring->ev[slot], st), "hipEventRecord");
      pending[slot] = v;
    }
  }
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  return CLOAK_OK;
}

extern "C" uint64_t cloak_ws_bytes(const cloak_layout* L, int32_t op, int32_t index, int64_t M) {
  if (!L || M < 0) return UINT64_MAX;
  if (op == CLOAK_OP_LINEAR) {
    if (index < 0 || index >= int32_t(L->tensors.size())) return UINT64_MAX;
    const TensorInfo& ti = L->tensors[index];
    // the prefill GEMM reads x in stored column order: a down projection's
    // activations are gathered through pi into the workspace first
    if (ti.perm_layer >= 0 && is_col_permuted(ti.shape.kind) && use_gemm(ti.shape.dtype, ti.shape.k_in, M))
      return (uint64_t(M) * uint64_t(ti.shape.k_in) * 2 + 255) / 256 * 256;
    return 0;
  }
  if (op == CLOAK_OP_MLP) {
    const FfnPerm* f = L->ffn_of_layer(index);
    if (!f || f->gate < 0 || f->up < 0 || f->down < 0) return UINT64_MAX;
    const int hb = L->tensors[f->gate].shape.dtype == CLOAK_F32 ? 4 : 2;
    const uint64_t b = uint64_t(M) * uint64_t(f->d_ffn) * uint64_t(hb);
    return (b + 255) / 256 * 256;
  }
  return UINT64_MAX;
}

extern "C" int cloak_linear_fused(const cloak_layout* L, const void* d_pool, const int32_t* tensors, int32_t n,
                                  const void* d_x, int64_t M, void* d_y, void* d_ws, uint64_t ws_bytes,
                                  void* stream) {
  clear_error();
  (void)d_ws;
  (void)ws_bytes;
  if (int rc = check_device_state(L, "cloak_linear")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_linear")) return rc;
  if (!tensors || n < 1 || n > 4 || M < 0 || M > INT32_MAX) {
    set_error("cloak_linear: need 1..4 tensors and 0 <= M < 2^31");
    return CLOAK_EINVAL;
  }
  for (int i = 0; i < n; ++i) {
    if (tensors[i] < 0 || tensors[i] >= int32_t(L->tensors.size())) {
      set_error("cloak_linear: tensor %d out of range", tensors[i]);
      return CLOAK_EINVAL;
    }
  }
  const TensorInfo& t0 = L->tensors[tensors[0]];
  const int64_t K = t0.shape.k_in;
  const int32_t dtype = t0.shape.dtype;
  const int elt = elt_bytes(dtype);
  bool any_down = false;
  int64_t total = 0;
  for (int i = 0; i < n; ++i) {
    const TensorInfo& ti = L->tensors[tensors[i]];
    if (ti.shape.k_in != K || ti.shape.dtype != dtype) {
      set_error("cloak_linear: fused tensors must share K and dtype");
      return CLOAK_ESHAPE;
    }
    any_down |= ti.perm_layer >= 0 && is_col_permuted(ti.shape.kind);
    total += ti.shape.n_out;
  }
  if (any_down && n > 1) {
    set_error("cloak_linear: a down projection (permuted K) cannot be fused with other tensors");
    return CLOAK_ESHAPE;
  }
  if ((K * elt) % 16 != 0) {
    set_error("cloak_linear: rows must be a multiple of 16 bytes (K*elt = %lld)", (long long)(K * elt));
    return CLOAK_ESHAPE;
  }
  if ((K * elt + 1023) / 1024 > 64) {
    set_error("cloak_linear: rows longer than 64 KiB are not supported");
    return CLOAK_ESHAPE;
  }
  if (total > INT32_MAX) {
    set_error("cloak_linear: too many output columns");
    return CLOAK_ESHAPE;
  }
  if (M == 0) return CLOAK_OK;
  if (!d_x || !d_y) {
    set_error("cloak_linear: null x or y");
    return CLOAK_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (use_gemm(dtype, K, M)) {
    GemmArgs g{};
    fill_gemm(L, d_pool, g, K, M);
    const void* xin = d_x;
    if (any_down) {
      const uint64_t need = cloak_ws_bytes(L, CLOAK_OP_LINEAR, tensors[0], M);
      if (!d_ws || ws_bytes < need) {
        set_error("cloak_linear: down projection at M=%lld needs a workspace of %llu bytes", (long long)M,
                  (unsigned long long)need);
        return CLOAK_EINVAL;
      }
      HIP_TRY(launch_gather_cols(static_cast<const uint16_t*>(d_x), K, L->dev.perms + L->ffn[t0.perm_layer].dev_off,
                                 static_cast<uint16_t*>(d_ws), M, K, st),
              "cloak_linear(gather)");
      xin = d_ws;
    }
    const int64_t tr = gemm_tile_rows();
    int64_t row0 = 0, out_off = 0;
    bool aligned = total % 4 == 0 && reinterpret_cast<uintptr_t>(d_y) % 8 == 0;
    for (int i = 0; i < n; ++i) {
      g.seg[i] = make_seg(L, tensors[i], true, int32_t(row0), int32_t(out_off));
      aligned = aligned && out_off % 4 == 0;
      row0 += (g.seg[i].rows + tr - 1) / tr * tr;
      out_off += g.seg[i].rows;
    }
    if (row0 > INT32_MAX) {
      set_error("cloak_linear: too many output rows");
      return CLOAK_ESHAPE;
    }
    for (int i = n; i < 4; ++i) g.seg[i] = g.seg[0], g.seg[i].row0 = INT32_MAX;
    g.nseg = n;
    g.mode = kStore;
    g.tiles_n = int32_t(row0 / tr);
    g.x = static_cast<const uint16_t*>(xin);
    g.ldx = K;
    g.y = d_y;
    g.ldy = total;
    g.vec_store = aligned ? 1 : 0;
    HIP_TRY(launch_gemm(g, !L->native(), st), "cloak_linear(gemm)");
    return CLOAK_OK;
  }
  GemvArgs a{};
  fill_common(L, d_pool, a, K, elt);
  a.nseg = n;
  // every tensor starts on a whole row group (kGemvRows launch-rows), so a
  // group never mixes tensors; out_off is the tensor's real column offset
  int64_t row0 = 0, out_off = 0;
  for (int i = 0; i < n; ++i) {
    a.seg[i] = make_seg(L, tensors[i], true, int32_t(row0), int32_t(out_off));
    row0 += (a.seg[i].rows + kGemvRows - 1) / kGemvRows * kGemvRows;
    out_off += a.seg[i].rows;
  }
  if (row0 > INT32_MAX) {
    set_error("cloak_linear: too many output rows");
    return CLOAK_ESHAPE;
  }
  for (int i = n; i < 4; ++i) a.seg[i] = a.seg[0], a.seg[i].row0 = INT32_MAX;
  a.groups = int32_t(row0 / kGemvRows);
  a.x = d_x;
  a.x_perm = any_down ? L->dev.perms + L->ffn[t0.perm_layer].dev_off : nullptr;
  a.y = d_y;
  a.ldx = K;
  a.ldy = total;
  a.mode = kStore;
  return run_gemv(L, a, wtype_of(dtype), M, st, "cloak_linear");
}

extern "C" int cloak_linear(const cloak_layout* L, const void* d_pool, int32_t tensor, const void* d_x, int64_t M,
                            void* d_y, void* d_ws, uint64_t ws_bytes, void* stream) {
  return cloak_linear_fused(L, d_pool, &tensor, 1, d_x, M, d_y, d_ws, ws_bytes, stream);
}

namespace {

// Shared checks of the FFN entry points; fills the three tensors.
int ffn_tensors(const cloak_layout* L, const void* d_pool, int32_t layer, int64_t M, const char* fn,
                const FfnPerm** out) {
  if (int rc = check_device_state(L, fn)) return rc;
  if (int rc = check_pool(L, d_pool, fn)) return rc;
  const FfnPerm* f = L->ffn_of_layer(layer);
  if (!f || f->gate < 0 || f->up < 0 || f->down < 0) {
    set_error("%s: layer %d lacks gate, up or down", fn, layer);
    return CLOAK_EINVAL;
  }
  if (M < 0 || M > INT32_MAX) {
    set_error("%s: bad M", fn);
    return CLOAK_EINVAL;
  }
  const TensorInfo& tg = L->tensors[f->gate];
  const TensorInfo& tu = L->tensors[f->up];
  const TensorInfo& td = L->tensors[f->down];
  const int32_t dtype = tg.shape.dtype;
  if (tu.shape.dtype != dtype || td.shape.dtype != dtype || tu.shape.k_in != tg.shape.k_in ||
      td.shape.n_out != tg.shape.k_in) {
    set_error("%s: gate/up/down dtypes or d_model disagree", fn);
    return CLOAK_ESHAPE;
  }
  const int elt = elt_bytes(dtype);
  const int64_t dm = tg.shape.k_in, dff = f->d_ffn;
  if ((dm * elt) % 16 != 0 || (dff * elt) % 16 != 0 || (dff * elt + 1023) / 1024 > 64 ||
      (dm * elt + 1023) / 1024 > 64) {
    set_error("%s: rows must be multiples of 16 bytes and at most 64 KiB", fn);
    return CLOAK_ESHAPE;
  }
  *out = f;
  return CLOAK_OK;
}

}  // namespace

extern "C" int cloak_swiglu(const cloak_layout* L, const void* d_pool, int32_t layer, const void* d_x, int64_t M,
                            void* d_h, void* stream) {
  clear_error();
  const FfnPerm* f = nullptr;
  if (int rc = ffn_tensors(L, d_pool, layer, M, "cloak_swiglu", &f)) return rc;
  if (M == 0) return CLOAK_OK;
  if (!d_x || !d_h) {
    set_error("cloak_swiglu: null x or h");
    return CLOAK_EINVAL;
  }
  const TensorInfo& tg = L->tensors[f->gate];
  const int32_t dtype = tg.shape.dtype;
  const int elt = elt_bytes(dtype);
  const int64_t dm = tg.shape.k_in, dff = f->d_ffn;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (use_gemm(dtype, dm, M)) {
    GemmArgs g{};
    fill_gemm(L, d_pool, g, dm, M);
    g.nseg = 2;
    g.seg[0] = make_seg(L, f->gate, false, 0, 0);
    g.seg[1] = make_seg(L, f->up, false, 0, 0);
    g.seg[2] = g.seg[0];
    g.seg[3] = g.seg[0];
    g.mode = kSwiGLU;
    g.tiles_n = int32_t((dff + gemm_tile_rows() / 2 - 1) / (gemm_tile_rows() / 2));
    g.x = static_cast<const uint16_t*>(d_x);
    g.ldx = dm;
    g.y = d_h;
    g.ldy = dff;
    g.vec_store = (dff % 4 == 0 && reinterpret_cast<uintptr_t>(d_h) % 8 == 0) ? 1 : 0;
    HIP_TRY(launch_gemm(g, !L->native(), st), "cloak_swiglu(gemm)");
    return CLOAK_OK;
  }
  // gate + up row pairs in one launch, SwiGLU epilogue -> h in permuted order
  GemvArgs a{};
  fill_common(L, d_pool, a, dm, elt);
  a.nseg = 2;
  a.seg[0] = make_seg(L, f->gate, false, 0, 0);
  a.seg[1] = make_seg(L, f->up, false, 0, 0);
  a.seg[2] = a.seg[0];
  a.seg[3] = a.seg[0];
  a.groups = int32_t((dff + kGemvRows / 2 - 1) / (kGemvRows / 2));
  a.x = d_x;
  a.x_perm = nullptr;
  a.y = d_h;
  a.ldx = dm;
  a.ldy = dff;
  a.mode = kSwiGLU;
  return run_gemv(L, a, wtype_of(dtype), M, st, "cloak_swiglu");
}

extern "C" int cloak_down(const cloak_layout* L, const void* d_pool, int32_t layer, const void* d_h, int64_t M,
                          void* d_y, void* stream) {
  clear_error();
  const FfnPerm* f = nullptr;
  if (int rc = ffn_tensors(L, d_pool, layer, M, "cloak_down", &f)) return rc;
  if (M == 0) return CLOAK_OK;
  if (!d_h || !d_y) {
    set_error("cloak_down: null h or y");
    return CLOAK_EINVAL;
  }
  const TensorInfo& tg = L->tensors[f->gate];
  const int32_t dtype = tg.shape.dtype;
  const int elt = elt_bytes(dtype);
  const int64_t dm = tg.shape.k_in, dff = f->d_ffn;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (use_gemm(dtype, dff, M)) {
    // down's stored columns are permuted exactly like h: no gather needed
    GemmArgs g{};
    fill_gemm(L, d_pool, g, dff, M);
    g.nseg = 1;
    g.seg[0] = make_seg(L, f->down, false, 0, 0);
    for (int i = 1; i < 4; ++i) g.seg[i] = g.seg[0], g.seg[i].row0 = INT32_MAX;
    g.mode = kStore;
    g.tiles_n = int32_t((dm + gemm_tile_rows() - 1) / gemm_tile_rows());
    g.x = static_cast<const uint16_t*>(d_h);
    g.ldx = dff;
    g.y = d_y;
    g.ldy = dm;
    g.vec_store = (dm % 4 == 0 && reinterpret_cast<uintptr_t>(d_y) % 8 == 0) ? 1 : 0;
    HIP_TRY(launch_gemm(g, !L->native(), st), "cloak_down(gemm)");
    return CLOAK_OK;
  }
  // down's stored columns are permuted exactly like h: no gather needed
  GemvArgs b{};
  fill_common(L, d_pool, b, dff, elt);
  b.nseg = 1;
  b.seg[0] = make_seg(L, f->down, false, 0, 0);
  for (int i = 1; i < 4; ++i) b.seg[i] = b.seg[0], b.seg[i].row0 = INT32_MAX;
  b.groups = int32_t((dm + kGemvRows - 1) / kGemvRows);
  b.x = d_h;
  b.x_perm = nullptr;
  b.y = d_y;
  b.ldx = dff;
  b.ldy = dm;
  b.mode = kStore;
  return run_gemv(L, b, wtype_of(dtype), M, st, "cloak_down");
}

extern "C" int cloak_mlp(const cloak_layout* L, const void* d_pool, int32_t layer, const void* d_x, int64_t M,
                         void* d_y, void* d_ws, uint64_t ws_bytes, void* stream) {
  clear_error();
  const FfnPerm* f = nullptr;
  if (int rc = ffn_tensors(L, d_pool, layer, M, "cloak_mlp", &f)) return rc;
  if (M == 0) return CLOAK_OK;
  const uint64_t need = cloak_ws_bytes(L, CLOAK_OP_MLP, layer, M);
  if (!d_x || !d_y || !d_ws || ws_bytes < need) {
    set_error("cloak_mlp: null x/y/workspace or workspace below %llu bytes", (unsigned long long)need);
    return CLOAK_EINVAL;
  }
  if (int rc = cloak_swiglu(L, d_pool, layer, d_x, M, d_ws, stream)) return rc;
  return cloak_down(L, d_pool, layer, d_ws, M, d_y, stream);
}

extern "C" int cloak_remap(cloak_layout* L, void* d_pool, uint64_t remap_seed, void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_remap")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_remap")) return rc;
  if (L->native()) {
    set_error("cloak_remap: native (untranslated) layouts cannot be remapped");
    return CLOAK_ESTATE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const std::vector<int32_t> tau = remap_matching(remap_seed, L->P);
  hipEvent_t ev = static_cast<hipEvent_t>(L->dev.stage_event);
  // the staging buffer may still feed the previous remap's copies
  HIP_TRY(hipEventSynchronize(ev), "hipEventSynchronize");
  int32_t* pairs = L->dev.h_stage;
  int32_t* new_phi = L->dev.h_stage + L->P + 1;
  int64_t np = 0;
  for (int64_t p = 0; p < L->P; ++p) {
    if (tau[p] > p) {
      pairs[2 * np] = int32_t(p);
      pairs[2 * np + 1] = tau[p];
      ++np;
    }
  }
  for (int64_t v = 0; v < L->P; ++v) new_phi[v] = tau[L->phi[v]];
  if (np > 0) {
    HIP_TRY(hipMemcpyAsync(L->dev.remap_pairs, pairs, size_t(np) * 8, hipMemcpyHostToDevice, st), "upload pairs");
    SwapArgs s{};
    s.pool = static_cast<uint8_t*>(d_pool);
    s.pairs = L->dev.remap_pairs;
    s.npairs = np;
    s.log2_page = L->log2_page;
    HIP_TRY(launch_swap(s, st), "swap kernel");
  }
  HIP_TRY(hipMemcpyAsync(L->dev.phi, new_phi, size_t(L->P) * 4, hipMemcpyHostToDevice, st), "upload page map");
  HIP_TRY(hipEventRecord(ev, st), "hipEventRecord");
  std::memcpy(L->phi.data(), new_phi, size_t(L->P) * 4);
  L->remaps += 1;
  return CLOAK_OK;
}

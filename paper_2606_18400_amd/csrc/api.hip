// Device-facing C-ABI entry points of libcloak: device tables, upload and
// read-back of cloaked tensors, the cloaked linear / FFN launches and the
// in-place remap (CloakLM, arXiv 2606.18400, Sections 4.2 and 5).

#include <hip/hip_runtime.h>

#include <algorithm>
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
  if (scatter) s.out_perm = L->dev_row_perm(t);
  s.scale = ti.shape.dtype == CLOAK_FP8_E4M3 ? L->dev.scales + ti.scale_off : nullptr;
  s.rows = int32_t(ti.shape.n_out);
  s.row0 = row0;
  s.out_off = out_off;
  return s;
}

// Token tile of the GEMV launches of an M-token call.
int gemv_mtile(int wtype, int nchunks, int64_t M) { return mtile_for(M, gemv_max_tokens(wtype, nchunks)); }

// Runs `a` over every token block of M (each launch handles mtile tokens).
int run_gemv(const cloak_layout* L, GemvArgs a, int wtype, int64_t M, hipStream_t st, const char* fn) {
  const int mt = gemv_mtile(wtype, a.nchunks, M);
  for (int64_t m0 = 0; m0 < M; m0 += mt) {
    a.m0 = int32_t(m0);
    a.mcount = int32_t(M - m0 < mt ? M - m0 : mt);
    HIP_TRY(launch_gemv(a, wtype, mt, L->kernel_translate(), st), fn);
  }
  return CLOAK_OK;
}

// The device copy of the current page map: plain, or (masked layouts) masked
// with the next key of the layout's key stream.  Returns the key (0: plain).
uint64_t mask_map(cloak_layout* L, int32_t* table) {
  uint64_t key = 0;
  if (L->masked_map())
    do key = L->map_keys.next(); while (key == 0);
  for (int64_t v = 0; v < L->P; ++v) table[v] = int32_t(uint32_t(L->phi[size_t(v)]) ^ phi_mask(key, v));
  return key;
}

void fill_common(const cloak_layout* L, const void* pool, GemvArgs& a, int64_t K, int elt) {
  a.pool = static_cast<const uint8_t*>(L->kernel_pool(pool));
  a.phi = L->dev.phi;
  a.phi_key = L->dev.phi_key;
  a.log2_page = L->log2_page;
  a.row_bytes = int32_t(K * elt);
  a.K = int32_t(K);
  a.nchunks = int32_t((K * elt + 1023) / 1024);
}

}  // namespace

namespace {
// Every device table of a layout; on failure whatever was allocated is freed.
void free_tables(DeviceTables& d) {
  if (d.phi) (void)hipFree(d.phi);
  if (d.perms) (void)hipFree(d.perms);
  if (d.scales) (void)hipFree(d.scales);
  if (d.remap_pairs) (void)hipFree(d.remap_pairs);
  if (d.experts) (void)hipFree(d.experts);
  if (d.h_stage) (void)hipHostFree(d.h_stage);
  if (d.stage_event) (void)hipEventDestroy(static_cast<hipEvent_t>(d.stage_event));
  d = DeviceTables{};
}

int build_tables(cloak_layout* L, DeviceTables& d, hipStream_t st) {
  HIP_TRY(hipGetDevice(&d.device), "hipGetDevice");
  const size_t P = size_t(L->P);
  HIP_TRY(hipMalloc(&d.phi, P * 4), "hipMalloc(page map)");
  HIP_TRY(hipMalloc(&d.perms, size_t(L->n_perm > 0 ? L->n_perm : 1) * 4), "hipMalloc(permutations)");
  HIP_TRY(hipMalloc(&d.scales, size_t(L->n_scales > 0 ? L->n_scales : 1) * 4), "hipMalloc(scales)");
  HIP_TRY(hipMalloc(&d.remap_pairs, P * 8 + 8), "hipMalloc(remap pairs)");
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&d.h_stage), P * 12 + 8, hipHostMallocDefault), "hipHostMalloc");
  hipEvent_t ev;
  HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
  d.stage_event = ev;
  std::vector<int32_t> perms(size_t(L->n_perm > 0 ? L->n_perm : 1), 0);
  for (const auto& pt : L->perms) std::memcpy(perms.data() + pt.dev_off, pt.p.data(), pt.p.size() * 4);
  // one MoE expert record per FFN group, ascending layer id
  std::vector<MoeExpert> ex(L->ffn.size() > 0 ? L->ffn.size() : 1);
  for (size_t i = 0; i < L->ffn_by_layer.size(); ++i) {
    const FfnPerm& f = L->ffn[size_t(L->ffn_by_layer[i])];
    MoeExpert r{};
    const int32_t ts[3] = {f.gate, f.up, f.down};
    r.ok = f.gate >= 0 && f.up >= 0 && f.down >= 0;
    for (int k = 0; k < 3; ++k) {
      r.vbase[k] = ts[k] >= 0 ? L->tensors[size_t(ts[k])].vbase : 0;
      r.npages[k] = ts[k] >= 0 ? L->tensors[size_t(ts[k])].npages : 0;
      r.scale_off[k] = ts[k] >= 0 ? int32_t(L->tensors[size_t(ts[k])].scale_off) : -1;
    }
    ex[i] = r;
  }
  HIP_TRY(hipMalloc(&d.experts, ex.size() * sizeof(MoeExpert)), "hipMalloc(expert table)");
  HIP_TRY(hipMemcpyAsync(d.experts, ex.data(), ex.size() * sizeof(MoeExpert), hipMemcpyHostToDevice, st),
          "upload expert table");
  std::vector<int32_t> table(P);
  d.phi_key = mask_map(L, table.data());
  HIP_TRY(hipMemcpyAsync(d.phi, table.data(), P * 4, hipMemcpyHostToDevice, st), "upload page map");
  HIP_TRY(hipMemcpyAsync(d.perms, perms.data(), perms.size() * 4, hipMemcpyHostToDevice, st), "upload permutations");
  HIP_TRY(hipMemsetAsync(d.scales, 0, size_t(L->n_scales > 0 ? L->n_scales : 1) * 4, st), "clear scales");
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  return CLOAK_OK;
}
}  // namespace

extern "C" int cloak_layout_to_device(cloak_layout* L, void* stream) {
  clear_error();
  if (!L) {
    set_error("cloak_layout_to_device: null layout");
    return CLOAK_EINVAL;
  }
  if (L->dev.phi) return CLOAK_OK;
  DeviceTables d;
  if (int rc = build_tables(L, d, static_cast<hipStream_t>(stream))) {
    free_tables(d);
    return rc;
  }
  L->dev = d;
  return CLOAK_OK;
}

namespace {
// Device state of a layout, released by cloak_layout_free (layout.cpp) before
// the host object goes.
void release_device(cloak_layout* L) {
  if (L->vmm.active) (void)cloak_vmm_pool_free(L);
  drop_ring(L);
  free_tables(L->dev);
}
[[maybe_unused]] const bool g_release_registered = (cloak::release_device_state = release_device, true);
}  // namespace

extern "C" int cloak_pool_init(const cloak_layout* L, void* d_pool, void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_pool_init")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_pool_init")) return rc;
  HIP_TRY(hipMemsetAsync(d_pool, 0, size_t(L->pool_bytes), static_cast<hipStream_t>(stream)), "hipMemsetAsync(pool)");
  return CLOAK_OK;
}

extern "C" int cloak_device_map_read(const cloak_layout* L, int32_t* h_out, void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_device_map_read")) return rc;
  if (!h_out) {
    set_error("cloak_device_map_read: null output");
    return CLOAK_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(h_out, L->dev.phi, size_t(L->P) * 4, hipMemcpyDeviceToHost, st), "read page map");
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  return CLOAK_OK;
}

extern "C" int cloak_pool_decoy(const cloak_layout* L, void* d_pool, uint64_t decoy_seed, void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_pool_decoy")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_pool_decoy")) return rc;
  DecoyArgs a{};
  a.pool = static_cast<uint8_t*>(d_pool);
  a.phi = L->dev.phi;
  a.phi_key = L->dev.phi_key;
  a.V = L->V;
  a.nfree = L->P - L->V;
  a.decoy_seed = decoy_seed;
  a.log2_page = L->log2_page;
  a.dtype = decoy_dtype(L);
  HIP_TRY(launch_decoy(a, static_cast<hipStream_t>(stream)), "cloak_pool_decoy");
  return CLOAK_OK;
}

extern "C" int cloak_load(cloak_layout* L, void* d_pool, int32_t tensor, const void* h_src, const float* h_scales,
                          void* stream) {
  clear_error();
  if (!L || tensor < 0 || tensor >= int32_t(L->tensors.size()) || !h_src) {
    set_error("cloak_load: null layout, bad tensor index %d or null source", tensor);
    return CLOAK_EINVAL;
  }
  // the first upload of every tensor follows sigma, so the bus never carries
  // the tensors in their architectural order (Section 4.2, Section 5)
  if (!L->loaded[size_t(tensor)] && L->sigma[size_t(L->n_loaded)] != tensor) {
    set_error("cloak_load: tensor %d uploaded out of the layout's tensor order (next first upload: tensor %d; "
              "cloak_load_all keeps that order)", tensor, L->sigma[size_t(L->n_loaded)]);
    return CLOAK_ESTATE;
  }
  if (int rc = check_device_state(L, "cloak_load")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_load")) return rc;
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
    // scales follow their rows: stored row j carries s[p[j]]
    s.resize(size_t(ti.shape.n_out));
    const int32_t* rp = L->row_perm(tensor);
    for (int64_t j = 0; j < ti.shape.n_out; ++j) s[j] = h_scales[rp ? rp[j] : j];
    HIP_TRY(hipMemcpyAsync(L->dev.scales + ti.scale_off, s.data(), s.size() * 4, hipMemcpyHostToDevice, st),
            "upload scales");
  }
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (!L->loaded[size_t(tensor)]) {
    L->loaded[size_t(tensor)] = 1;
    L->n_loaded += 1;
  }
  return CLOAK_OK;
}

extern "C" int cloak_load_all(cloak_layout* L, void* d_pool, const void* const* h_srcs, const float* const* h_scales,
                              void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_load_all")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_load_all")) return rc;
  const int64_t T = int64_t(L->tensors.size());
  if (!h_srcs) {
    set_error("cloak_load_all: null source table");
    return CLOAK_EINVAL;
  }
  // check every argument before the first page crosses the bus
  for (int64_t t = 0; t < T; ++t) {
    const bool fp8 = L->tensors[size_t(t)].shape.dtype == CLOAK_FP8_E4M3;
    const float* sc = h_scales ? h_scales[t] : nullptr;
    if (!h_srcs[t] || fp8 != (sc != nullptr)) {
      set_error("cloak_load_all: tensor %lld has no source, or scales that do not match its dtype", (long long)t);
      return CLOAK_EINVAL;
    }
  }
  for (int64_t i = 0; i < T; ++i) {
    const int32_t t = L->sigma[size_t(i)];
    if (int rc = cloak_load(L, d_pool, t, h_srcs[t], h_scales ? h_scales[t] : nullptr, stream)) return rc;
  }
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

namespace {

// Which kernel family serves a projection: the VALU GEMV below 5 tokens (and
// for f32 weights or K not a multiple of 64), the skinny split-K MFMA GEMM
// for 5..256 tokens (and, in pieces, up to 1,024), the 256x256 MFMA GEMM
// above that.
enum Path { kPathGemv, kPathSkinny, kPathGemm };

Path pick_path(int32_t dtype, int64_t K, int64_t M) {
  if ((dtype == CLOAK_BF16 || dtype == CLOAK_FP8_E4M3) && K % gemm_k_step() == 0 && M >= kGemmMinTokens)
    return M <= kSkinnyMaxTokens ? kPathSkinny : kPathGemm;
  return kPathGemv;
}

struct SplitPlan {
  int32_t ksplit, kb_per;
};

// K slices per skinny row tile: about 1024 workgroups in total (512 above
// 64 tokens, where each slice's FP32 partial sums cost more traffic), but no
// slice shorter than 8 K steps.  Tiles that take a whole CU (above 128
// tokens, and BF16 above 64 through the LDS ring): as many slices as keep
// the launch within one pass over MI355X's 256 CUs (one slice when the row
// tiles alone exceed them).
constexpr int64_t kSkinnyWideSlots = 256;
// a8: FP8 x FP8 tiles (K steps of 128 elements, LDS ring like BF16)
SplitPlan plan_split(int64_t tiles_n, int64_t K, int64_t M, int32_t dtype, bool a8) {
  const int64_t nk = K / (a8 ? gemm_k_step_a8() : gemm_k_step());
  const int64_t target = M > 64 ? 512 : 1024;
  const bool whole_cu = M > 128 || (M > 64 && (dtype == CLOAK_BF16 || a8));
  int64_t ks = whole_cu ? kSkinnyWideSlots / tiles_n : (target + tiles_n - 1) / tiles_n;
  const int64_t cap = nk / 8 > 1 ? nk / 8 : 1;
  if (ks > cap) ks = cap;
  if (ks < 1) ks = 1;
  const int64_t per = (nk + ks - 1) / ks;
  return {int32_t((nk + per - 1) / per), int32_t(per)};
}

uint64_t a256(uint64_t b) { return (b + 255) / 256 * 256; }

// One projection launch: up to 4 tensors sharing K (STORE), or a layer's
// gate/up pair with the SwiGLU epilogue.
struct Proj {
  int32_t tensors[4] = {0, 0, 0, 0};
  int n = 0;
  int mode = kStore;
  bool scatter = false;        // gate/up rows written to their logical columns
  bool gather = false;         // x gathered through pi (down via cloak_linear)
  const int32_t* x_perm = nullptr;  // that permutation on the device
  int64_t K = 0;
  int32_t dtype = CLOAK_BF16;
  int64_t rows = 0;            // sum of N (STORE) or d_ffn (SwiGLU)
};

int64_t launch_rows(const cloak_layout* L, const Proj& p, int64_t tile) {
  if (p.mode == kSwiGLU) return (p.rows + tile / 2 - 1) / (tile / 2) * tile;
  int64_t r = 0;
  for (int i = 0; i < p.n; ++i) r += (L->tensors[p.tensors[i]].shape.n_out + tile - 1) / tile * tile;
  return r;
}

// FP8 weights from kA8MinTokens tokens (the skinny direct-to-LDS tiles and
// the 256x256 GEMM): FP8 x FP8 MFMA on activations quantised per token (the
// quantisation also applies the gather of a down projection).  Below that the
// FP8 weights are widened to BF16 and meet unquantised activations.
constexpr int64_t kA8MinTokens = 65;
bool use_a8(const Proj& p, Path path, int64_t M) {
  return path != kPathGemv && M >= kA8MinTokens && p.dtype == CLOAK_FP8_E4M3 && p.K % gemm_k_step_a8() == 0;
}

uint64_t proj_ws_bytes_one(const cloak_layout* L, const Proj& p, int64_t M) {
  const Path path = pick_path(p.dtype, p.K, M);
  const bool a8 = use_a8(p, path, M);
  uint64_t b = 0;
  if (a8)
    b += a256(uint64_t(M) * uint64_t(p.K)) + a256(uint64_t(M) * 4);
  else if (p.gather && path != kPathGemv)
    b += a256(uint64_t(M) * uint64_t(p.K) * 2);
  if (path == kPathSkinny) {
    const int64_t lr = launch_rows(L, p, skinny_tile_rows(M));
    const SplitPlan sp = plan_split(lr / skinny_tile_rows(M), p.K, M, p.dtype, a8);
    b += a256(uint64_t(sp.ksplit) * uint64_t(M) * uint64_t(lr) * 4);
  }
  return b;
}

int run_proj_one(const cloak_layout* L, const void* pool, const Proj& p, const void* x, int64_t ldx, int64_t M,
                 void* y, int64_t ldy, void* ws, uint64_t ws_bytes, hipStream_t st, const char* fn) {
  const uint64_t need = proj_ws_bytes_one(L, p, M);
  if (need > 0 && (!ws || ws_bytes < need)) {
    set_error("%s: M=%lld needs a workspace of %llu bytes (cloak_ws_bytes)", fn, (long long)M,
              (unsigned long long)need);
    return CLOAK_EINVAL;
  }
  const int elt = elt_bytes(p.dtype);
  const Path path = pick_path(p.dtype, p.K, M);
  if (path == kPathGemv) {
    GemvArgs a{};
    fill_common(L, pool, a, p.K, elt);
    const int64_t kGemvRows = gemv_rows(a.nchunks, gemv_mtile(wtype_of(p.dtype), a.nchunks, M));
    if (p.mode == kSwiGLU) {
      a.nseg = 2;
      a.seg[0] = make_seg(L, p.tensors[0], false, 0, 0);
      a.seg[1] = make_seg(L, p.tensors[1], false, 0, 0);
      a.seg[2] = a.seg[0];
      a.seg[3] = a.seg[0];
      a.groups = int32_t((p.rows + kGemvRows / 2 - 1) / (kGemvRows / 2));
    } else {
      // every tensor starts on a whole row group, so a group never mixes tensors
      int64_t row0 = 0, out_off = 0;
      for (int i = 0; i < p.n; ++i) {
        a.seg[i] = make_seg(L, p.tensors[i], p.scatter, int32_t(row0), int32_t(out_off));
        row0 += (a.seg[i].rows + kGemvRows - 1) / kGemvRows * kGemvRows;
        out_off += a.seg[i].rows;
      }
      for (int i = p.n; i < 4; ++i) a.seg[i] = a.seg[0], a.seg[i].row0 = INT32_MAX;
      a.nseg = p.n;
      a.groups = int32_t(row0 / kGemvRows);
    }
    a.x = x;
    a.x_perm = p.x_perm;
    a.y = y;
    a.ldx = ldx;
    a.ldy = ldy;
    a.mode = p.mode;
    const int xelt = p.dtype == CLOAK_F32 ? 4 : 2;
    a.x_vec = !p.x_perm && reinterpret_cast<uintptr_t>(x) % 16 == 0 && (ldx * xelt) % 16 == 0 ? 1 : 0;
    return run_gemv(L, a, wtype_of(p.dtype), M, st, fn);
  }
  // MFMA paths read x in the tensors' stored column order
  uint8_t* wsb = static_cast<uint8_t*>(ws);
  const void* xin = x;
  const bool a8 = use_a8(p, path, M);
  float* sx = nullptr;
  if (a8) {
    uint8_t* q = wsb;
    sx = reinterpret_cast<float*>(wsb + a256(uint64_t(M) * uint64_t(p.K)));
    HIP_TRY(launch_quant_rows(static_cast<const uint16_t*>(x), ldx, p.gather ? p.x_perm : nullptr, q, sx, M, p.K,
                              st),
            fn);
    xin = q;
    ldx = p.K;
    wsb += a256(uint64_t(M) * uint64_t(p.K)) + a256(uint64_t(M) * 4);
  } else if (p.gather) {
    HIP_TRY(launch_gather_cols(static_cast<const uint16_t*>(x), ldx, p.x_perm, reinterpret_cast<uint16_t*>(wsb), M,
                               p.K, st),
            fn);
    xin = wsb;
    ldx = p.K;
    wsb += a256(uint64_t(M) * uint64_t(p.K) * 2);
  }
  const int64_t tile = path == kPathSkinny ? skinny_tile_rows(M) : gemm_tile_rows();
  SkinnyArgs g{};
  g.pool = static_cast<const uint8_t*>(L->kernel_pool(pool));
  g.phi = L->dev.phi;
  g.phi_key = L->dev.phi_key;
  g.log2_page = L->log2_page;
  g.K = int32_t(p.K);
  g.row_bytes = p.K * elt;
  g.f8 = p.dtype == CLOAK_FP8_E4M3 ? 1 : 0;
  g.a8 = a8 ? 1 : 0;
  g.sx = sx;
  g.M = int32_t(M);
  g.mode = p.mode;
  g.x = static_cast<const uint16_t*>(xin);
  g.ldx = ldx;
  g.y = y;
  g.ldy = ldy;
  bool aligned = ldy % 4 == 0 && reinterpret_cast<uintptr_t>(y) % 8 == 0;
  if (p.mode == kSwiGLU) {
    g.nseg = 2;
    g.seg[0] = make_seg(L, p.tensors[0], false, 0, 0);
    g.seg[1] = make_seg(L, p.tensors[1], false, 0, 0);
    g.seg[2] = g.seg[0];
    g.seg[3] = g.seg[0];
  } else {
    int64_t row0 = 0, out_off = 0;
    for (int i = 0; i < p.n; ++i) {
      g.seg[i] = make_seg(L, p.tensors[i], p.scatter, int32_t(row0), int32_t(out_off));
      aligned = aligned && out_off % 4 == 0;
      row0 += (g.seg[i].rows + tile - 1) / tile * tile;
      out_off += g.seg[i].rows;
    }
    for (int i = p.n; i < 4; ++i) g.seg[i] = g.seg[0], g.seg[i].row0 = INT32_MAX;
    g.nseg = p.n;
  }
  const int64_t lr = launch_rows(L, p, tile);
  if (lr > INT32_MAX) {
    set_error("%s: too many output rows", fn);
    return CLOAK_ESHAPE;
  }
  g.tiles_n = int32_t(lr / tile);
  g.tiles_m = int32_t((M + gemm_tile_rows() - 1) / gemm_tile_rows());
  g.vec_store = aligned ? 1 : 0;
  if (path == kPathSkinny) {
    const SplitPlan sp = plan_split(g.tiles_n, p.K, M, p.dtype, a8);
    g.part = reinterpret_cast<float*>(wsb);
    g.ldp = lr;
    g.ksplit = sp.ksplit;
    g.kblocks_per_split = sp.kb_per;
    g.tile_rows = int32_t(tile);
    HIP_TRY(launch_skinny(g, L->kernel_translate(), st), fn);
  } else {
    GemmArgs ga{};
    std::memcpy(&ga, &g, sizeof(GemmArgs));
    HIP_TRY(launch_gemm(ga, L->kernel_translate(), st), fn);
  }
  return CLOAK_OK;
}

// 257..1024 tokens run as ceil(M / 256) near-equal calls of the skinny
// split-K path: a 256 x 256 tile GEMM has too few tiles there to fill the
// CUs (the 4096-row projections at 512 tokens: 32 workgroups), and one
// skinny call per at most 256 tokens, each reading the weights once, is
// faster up to 1,024 tokens (measured on the 4096/14336 layer: 276 TFLOP/s
// at 512 tokens and 482 at 1,024 through the GEMM, 515 per 256-token skinny
// call).  Chunks are 129..256 tokens, so FP8 weights meet quantised
// activations in every chunk, as they would in the GEMM.
constexpr int64_t kChunkTokens = 256, kChunkedMaxTokens = 1024;
bool chunked(const Proj& p, int64_t M) {
  return M > kChunkTokens && M <= kChunkedMaxTokens && pick_path(p.dtype, p.K, M) == kPathGemm;
}
int64_t n_chunks(int64_t M) { return (M + kChunkTokens - 1) / kChunkTokens; }

uint64_t proj_ws_bytes(const cloak_layout* L, const Proj& p, int64_t M) {
  if (!chunked(p, M)) return proj_ws_bytes_one(L, p, M);
  // the workspace serves each chunk in turn (sizes M / n and M / n + 1)
  const int64_t n = n_chunks(M), base = M / n;
  const uint64_t a = proj_ws_bytes_one(L, p, base), b = proj_ws_bytes_one(L, p, base + 1);
  return a > b ? a : b;
}

int run_proj(const cloak_layout* L, const void* pool, const Proj& p, const void* x, int64_t ldx, int64_t M, void* y,
             int64_t ldy, void* ws, uint64_t ws_bytes, hipStream_t st, const char* fn) {
  if (!chunked(p, M)) return run_proj_one(L, pool, p, x, ldx, M, y, ldy, ws, ws_bytes, st, fn);
  const uint64_t need = proj_ws_bytes(L, p, M);
  if (!ws || ws_bytes < need) {
    set_error("%s: M=%lld needs a workspace of %llu bytes (cloak_ws_bytes)", fn, (long long)M,
              (unsigned long long)need);
    return CLOAK_EINVAL;
  }
  // MFMA paths take bf16 activations and write bf16 results; chunks run in
  // stream order, so they share the workspace
  const int64_t n = n_chunks(M), base = M / n, rem = M % n;
  for (int64_t c = 0, m0 = 0; c < n; ++c) {
    const int64_t mc = base + (c < rem ? 1 : 0);
    const void* xc = static_cast<const uint16_t*>(x) + m0 * ldx;
    void* yc = static_cast<uint16_t*>(y) + m0 * ldy;
    if (int rc = run_proj_one(L, pool, p, xc, ldx, mc, yc, ldy, ws, ws_bytes, st, fn)) return rc;
    m0 += mc;
  }
  return CLOAK_OK;
}

int linear_proj(const cloak_layout* L, const int32_t* tensors, int32_t n, Proj& p, const char* fn) {
  if (!tensors || n < 1 || n > 4) {
    set_error("%s: need 1..4 tensors", fn);
    return CLOAK_EINVAL;
  }
  for (int i = 0; i < n; ++i) {
    if (tensors[i] < 0 || tensors[i] >= int32_t(L->tensors.size())) {
      set_error("%s: tensor %d out of range", fn, tensors[i]);
      return CLOAK_EINVAL;
    }
  }
  const TensorInfo& t0 = L->tensors[tensors[0]];
  p.K = t0.shape.k_in;
  p.dtype = t0.shape.dtype;
  bool any_down = false;
  for (int i = 0; i < n; ++i) {
    const TensorInfo& ti = L->tensors[tensors[i]];
    if (ti.shape.k_in != p.K || ti.shape.dtype != p.dtype) {
      set_error("%s: fused tensors must share K and dtype", fn);
      return CLOAK_ESHAPE;
    }
    any_down |= ti.col_perm >= 0;
    p.rows += ti.shape.n_out;
    p.tensors[i] = tensors[i];
  }
  p.n = n;
  p.mode = kStore;
  p.scatter = true;
  if (any_down && n > 1) {
    set_error("%s: a tensor with permuted columns (down, head-permuted o) cannot be fused with others", fn);
    return CLOAK_ESHAPE;
  }
  p.gather = any_down;
  p.x_perm = any_down ? L->dev_col_perm(tensors[0]) : nullptr;
  const int elt = elt_bytes(p.dtype);
  if ((p.K * elt) % 16 != 0 || (p.K * elt + 1023) / 1024 > 64) {
    set_error("%s: rows must be a multiple of 16 bytes and at most 64 KiB (K*elt = %lld)", fn,
              (long long)(p.K * elt));
    return CLOAK_ESHAPE;
  }
  if (p.rows > INT32_MAX) {
    set_error("%s: too many output columns", fn);
    return CLOAK_ESHAPE;
  }
  return CLOAK_OK;
}

// Gate/up (SwiGLU) or down projection of one layer.
int ffn_proj(const cloak_layout* L, int32_t layer, bool swiglu, Proj& p, int64_t& dm, int64_t& dff, const char* fn) {
  const FfnPerm* f = L->ffn_of_layer(layer);
  if (!f || f->gate < 0 || f->up < 0 || f->down < 0) {
    set_error("%s: layer %d lacks gate, up or down", fn, layer);
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
  dm = tg.shape.k_in;
  dff = f->d_ffn;
  if ((dm * elt) % 16 != 0 || (dff * elt) % 16 != 0 || (dff * elt + 1023) / 1024 > 64 ||
      (dm * elt + 1023) / 1024 > 64) {
    set_error("%s: rows must be multiples of 16 bytes and at most 64 KiB", fn);
    return CLOAK_ESHAPE;
  }
  p.dtype = dtype;
  if (swiglu) {
    p.tensors[0] = f->gate;
    p.tensors[1] = f->up;
    p.n = 2;
    p.mode = kSwiGLU;
    p.K = dm;
    p.rows = dff;
  } else {
    // down's stored columns carry the same permutation as h: no gather
    p.tensors[0] = f->down;
    p.n = 1;
    p.mode = kStore;
    p.K = dff;
    p.rows = dm;
  }
  return CLOAK_OK;
}

}  // namespace

namespace cloak {
uint64_t linear_fused_ws_bytes(const cloak_layout* L, const int32_t* tensors, int32_t n, int64_t M) {
  Proj p;
  if (!L || M < 0 || linear_proj(L, tensors, n, p, "cloak_ws_bytes")) return UINT64_MAX;
  return proj_ws_bytes(L, p, M);
}
}  // namespace cloak

extern "C" uint64_t cloak_linear_fused_ws_bytes(const cloak_layout* L, const int32_t* tensors, int32_t n,
                                                int64_t M) {
  return linear_fused_ws_bytes(L, tensors, n, M);
}

extern "C" uint64_t cloak_mlp_ws_bytes(const cloak_layout* L, int32_t layer, int64_t M) {
  return cloak_ws_bytes(L, CLOAK_OP_MLP, layer, M);
}

extern "C" uint64_t cloak_ws_bytes(const cloak_layout* L, int32_t op, int32_t index, int64_t M) {
  if (!L || M < 0) return UINT64_MAX;
  if (op == CLOAK_OP_LINEAR) return linear_fused_ws_bytes(L, &index, 1, M);
  Proj p;
  int64_t dm = 0, dff = 0;
  if (op == CLOAK_OP_SWIGLU || op == CLOAK_OP_DOWN) {
    if (ffn_proj(L, index, op == CLOAK_OP_SWIGLU, p, dm, dff, "cloak_ws_bytes")) return UINT64_MAX;
    return proj_ws_bytes(L, p, M);
  }
  if (op == CLOAK_OP_MLP) {
    Proj d;
    if (ffn_proj(L, index, true, p, dm, dff, "cloak_ws_bytes") || ffn_proj(L, index, false, d, dm, dff, "cloak_ws_bytes"))
      return UINT64_MAX;
    const int hb = p.dtype == CLOAK_F32 ? 4 : 2;
    const uint64_t a = proj_ws_bytes(L, p, M), b = proj_ws_bytes(L, d, M);
    return a256(uint64_t(M) * uint64_t(dff) * uint64_t(hb)) + (a > b ? a : b);
  }
  return UINT64_MAX;
}

extern "C" int cloak_linear_fused(const cloak_layout* L, const void* d_pool, const int32_t* tensors, int32_t n,
                                  const void* d_x, int64_t M, void* d_y, void* d_ws, uint64_t ws_bytes,
                                  void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_linear")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_linear")) return rc;
  if (M < 0 || M > INT32_MAX) {
    set_error("cloak_linear: bad M");
    return CLOAK_EINVAL;
  }
  Proj p;
  if (int rc = linear_proj(L, tensors, n, p, "cloak_linear")) return rc;
  if (M == 0) return CLOAK_OK;
  if (!d_x || !d_y) {
    set_error("cloak_linear: null x or y");
    return CLOAK_EINVAL;
  }
  return run_proj(L, d_pool, p, d_x, p.K, M, d_y, p.rows, d_ws, ws_bytes, static_cast<hipStream_t>(stream),
                  "cloak_linear");
}

// Both sides in stored order: permuted rows are not scattered, permuted
// columns not gathered.  The decoder step keeps attention and the FFN in that
// order, where the permutations cancel between consecutive projections.
extern "C" int cloak_linear_stored(const cloak_layout* L, const void* d_pool, const int32_t* tensors, int32_t n,
                                   const void* d_x, int64_t M, void* d_y, void* d_ws, uint64_t ws_bytes,
                                   void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_linear_stored")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_linear_stored")) return rc;
  if (M < 0 || M > INT32_MAX) {
    set_error("cloak_linear_stored: bad M");
    return CLOAK_EINVAL;
  }
  Proj p;
  if (int rc = linear_proj(L, tensors, n, p, "cloak_linear_stored")) return rc;
  p.scatter = false;
  p.gather = false;
  p.x_perm = nullptr;
  if (M == 0) return CLOAK_OK;
  if (!d_x || !d_y) {
    set_error("cloak_linear_stored: null x or y");
    return CLOAK_EINVAL;
  }
  return run_proj(L, d_pool, p, d_x, p.K, M, d_y, p.rows, d_ws, ws_bytes, static_cast<hipStream_t>(stream),
                  "cloak_linear_stored");
}

extern "C" int cloak_linear(const cloak_layout* L, const void* d_pool, int32_t tensor, const void* d_x, int64_t M,
                            void* d_y, void* d_ws, uint64_t ws_bytes, void* stream) {
  return cloak_linear_fused(L, d_pool, &tensor, 1, d_x, M, d_y, d_ws, ws_bytes, stream);
}

namespace {
int ffn_call(const cloak_layout* L, const void* d_pool, int32_t layer, bool swiglu, const void* d_in, int64_t M,
             void* d_out, void* d_ws, uint64_t ws_bytes, void* stream, const char* fn) {
  clear_error();
  if (int rc = check_device_state(L, fn)) return rc;
  if (int rc = check_pool(L, d_pool, fn)) return rc;
  if (M < 0 || M > INT32_MAX) {
    set_error("%s: bad M", fn);
    return CLOAK_EINVAL;
  }
  Proj p;
  int64_t dm = 0, dff = 0;
  if (int rc = ffn_proj(L, layer, swiglu, p, dm, dff, fn)) return rc;
  if (M == 0) return CLOAK_OK;
  if (!d_in || !d_out) {
    set_error("%s: null input or output", fn);
    return CLOAK_EINVAL;
  }
  const int64_t ldx = swiglu ? dm : dff, ldy = swiglu ? dff : dm;
  return run_proj(L, d_pool, p, d_in, ldx, M, d_out, ldy, d_ws, ws_bytes, static_cast<hipStream_t>(stream), fn);
}
}  // namespace

extern "C" int cloak_swiglu(const cloak_layout* L, const void* d_pool, int32_t layer, const void* d_x, int64_t M,
                            void* d_h, void* d_ws, uint64_t ws_bytes, void* stream) {
  return ffn_call(L, d_pool, layer, true, d_x, M, d_h, d_ws, ws_bytes, stream, "cloak_swiglu");
}

extern "C" int cloak_down(const cloak_layout* L, const void* d_pool, int32_t layer, const void* d_h, int64_t M,
                          void* d_y, void* d_ws, uint64_t ws_bytes, void* stream) {
  return ffn_call(L, d_pool, layer, false, d_h, M, d_y, d_ws, ws_bytes, stream, "cloak_down");
}

extern "C" int cloak_mlp(const cloak_layout* L, const void* d_pool, int32_t layer, const void* d_x, int64_t M,
                         void* d_y, void* d_ws, uint64_t ws_bytes, void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_mlp")) return rc;
  Proj p;
  int64_t dm = 0, dff = 0;
  if (int rc = ffn_proj(L, layer, true, p, dm, dff, "cloak_mlp")) return rc;
  if (M < 0 || M > INT32_MAX) {
    set_error("cloak_mlp: bad M");
    return CLOAK_EINVAL;
  }
  if (M == 0) return CLOAK_OK;
  const uint64_t need = cloak_ws_bytes(L, CLOAK_OP_MLP, layer, M);
  if (!d_x || !d_y || !d_ws || ws_bytes < need) {
    set_error("cloak_mlp: null x/y/workspace or workspace below %llu bytes", (unsigned long long)need);
    return CLOAK_EINVAL;
  }
  const int hb = p.dtype == CLOAK_F32 ? 4 : 2;
  const uint64_t hbytes = a256(uint64_t(M) * uint64_t(dff) * uint64_t(hb));
  uint8_t* scratch = static_cast<uint8_t*>(d_ws) + hbytes;
  if (int rc = cloak_swiglu(L, d_pool, layer, d_x, M, d_ws, scratch, ws_bytes - hbytes, stream)) return rc;
  return cloak_down(L, d_pool, layer, d_ws, M, d_y, scratch, ws_bytes - hbytes, stream);
}

namespace {
// The experts of a MoE call: FFN groups of layers first .. first+E-1, which
// sit at consecutive positions of the ascending-layer table.  Returns the
// position of the first, or -1 (error set).
int64_t moe_experts(const cloak_layout* L, int32_t first, int32_t E, int32_t& dtype, int64_t& dm, int64_t& dff,
                    const char* fn) {
  if (E < 1 || E > 1024) {
    set_error("%s: n_experts must be 1..1024", fn);
    return -1;
  }
  int64_t pos = -1;
  for (size_t i = 0; i < L->ffn_by_layer.size(); ++i)
    if (L->ffn[size_t(L->ffn_by_layer[i])].layer == first) pos = int64_t(i);
  if (pos < 0 || pos + E > int64_t(L->ffn_by_layer.size())) {
    set_error("%s: layers %d..%d are not all FFN groups", fn, first, first + E - 1);
    return -1;
  }
  for (int32_t e = 0; e < E; ++e) {
    const FfnPerm& f = L->ffn[size_t(L->ffn_by_layer[size_t(pos + e)])];
    if (f.layer != first + e || f.gate < 0 || f.up < 0 || f.down < 0) {
      set_error("%s: expert %d (layer %d) lacks gate, up or down", fn, e, first + e);
      return -1;
    }
    const cloak_shape& g = L->tensors[size_t(f.gate)].shape;
    const cloak_shape& u = L->tensors[size_t(f.up)].shape;
    const cloak_shape& d = L->tensors[size_t(f.down)].shape;
    if (e == 0) {
      dtype = g.dtype;
      dm = g.k_in;
      dff = f.d_ffn;
    }
    if (g.dtype != dtype || u.dtype != dtype || d.dtype != dtype || g.k_in != dm || u.k_in != dm ||
        d.n_out != dm || f.d_ffn != dff) {
      set_error("%s: experts must share dtype, d_model and d_ffn", fn);
      return -1;
    }
  }
  if (dtype != CLOAK_BF16 && dtype != CLOAK_FP8_E4M3) {
    set_error("%s: experts must be BF16 or FP8 E4M3", fn);
    return -1;
  }
  const int elt = elt_bytes(dtype);
  if ((dm * elt) % 16 != 0 || (dff * elt) % 16 != 0 || dm % 8 != 0 || dff % 8 != 0 || dm > INT32_MAX ||
      dff > INT32_MAX) {
    set_error("%s: d_model and d_ffn rows must be multiples of 16 bytes", fn);
    return -1;
  }
  return pos;
}

constexpr int64_t kMoeMaxPairs = 4096;

// ints of the routing workspace for n pairs over E experts: counts and runs,
// the sorted pairs, and the MFMA path's token-tile list
uint64_t moe_route_ints(uint64_t n, uint64_t E) { return 1 + 3 * E + n + 1 + 2 * uint64_t(moe_max_tiles(int64_t(n), int64_t(E))); }
}  // namespace

extern "C" uint64_t cloak_moe_ws_bytes(const cloak_layout* L, int32_t first_layer, int32_t n_experts, int32_t top_k,
                                       int64_t M) {
  if (!L || M < 0 || top_k < 1) return UINT64_MAX;
  int32_t dt = 0;
  int64_t dm = 0, dff = 0;
  if (moe_experts(L, first_layer, n_experts, dt, dm, dff, "cloak_moe_ws_bytes") < 0) return UINT64_MAX;
  if (top_k > kMoeMaxPairs) return UINT64_MAX;
  // calls above kMoeMaxPairs pairs run in token chunks that reuse one chunk's workspace
  const int64_t chunk = kMoeMaxPairs / top_k;
  const uint64_t n = uint64_t(M < chunk ? M : chunk) * uint64_t(top_k);
  return a256(moe_route_ints(n, uint64_t(n_experts)) * 4) + a256(n * uint64_t(dff) * 2) + a256(n * uint64_t(dm) * 4);
}

extern "C" int cloak_moe(const cloak_layout* L, const void* d_pool, int32_t first_layer, int32_t n_experts,
                         int32_t top_k, const void* d_x, int64_t M, const int32_t* d_ids, const float* d_weights,
                         void* d_y, void* d_ws, uint64_t ws_bytes, void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_moe")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_moe")) return rc;
  int32_t dt = 0;
  int64_t dm = 0, dff = 0;
  const int64_t pos = moe_experts(L, first_layer, n_experts, dt, dm, dff, "cloak_moe");
  if (pos < 0) return CLOAK_EINVAL;
  if (top_k < 1 || top_k > kMoeMaxPairs || M < 0 || M > INT32_MAX) {
    set_error("cloak_moe: need 1 <= top_k <= %lld and 0 <= M", (long long)kMoeMaxPairs);
    return CLOAK_EINVAL;
  }
  if (M == 0) return CLOAK_OK;
  const uint64_t need = cloak_moe_ws_bytes(L, first_layer, n_experts, top_k, M);
  if (!d_x || !d_ids || !d_weights || !d_y || !d_ws || ws_bytes < need) {
    set_error("cloak_moe: null buffer or workspace below %llu bytes", (unsigned long long)need);
    return CLOAK_EINVAL;
  }
  if (reinterpret_cast<uintptr_t>(d_x) % 16 != 0 || reinterpret_cast<uintptr_t>(d_y) % 8 != 0 ||
      reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) {
    set_error("cloak_moe: x must be 16-byte, y 8-byte and the workspace 256-byte aligned");
    return CLOAK_EINVAL;
  }
  // the workspace holds one chunk: its regions are sized for the largest chunk's pairs
  const int64_t chunk = kMoeMaxPairs / top_k;
  const uint64_t n = uint64_t(M < chunk ? M : chunk) * uint64_t(top_k);
  uint8_t* w = static_cast<uint8_t*>(d_ws);
  MoeArgs a{};
  a.pool = static_cast<const uint8_t*>(L->kernel_pool(d_pool));
  a.phi = L->dev.phi;
  a.phi_key = L->dev.phi_key;
  a.log2_page = L->log2_page;
  a.wtype = dt == CLOAK_FP8_E4M3 ? kFP8 : kBF16;
  a.experts = static_cast<const MoeExpert*>(L->dev.experts) + pos;
  a.scales = L->dev.scales;
  a.E = n_experts;
  a.topk = top_k;
  a.d_model = int32_t(dm);
  a.d_ffn = int32_t(dff);
  a.route = reinterpret_cast<int32_t*>(w);
  w += a256(moe_route_ints(n, uint64_t(n_experts)) * 4);
  a.h = reinterpret_cast<uint16_t*>(w);
  w += a256(n * uint64_t(dff) * 2);
  a.yp = reinterpret_cast<float*>(w);
  // token chunks of at most kMoeMaxPairs pairs, in order, on one workspace
  for (int64_t m0 = 0; m0 < M; m0 += chunk) {
    const int64_t mc = M - m0 < chunk ? M - m0 : chunk;
    a.M = int32_t(mc);
    a.x = static_cast<const uint16_t*>(d_x) + m0 * dm;
    a.ids = d_ids + m0 * top_k;
    a.wts = d_weights + m0 * top_k;
    a.y = static_cast<uint16_t*>(d_y) + m0 * dm;
    HIP_TRY(launch_moe(a, L->kernel_translate(), static_cast<hipStream_t>(stream)), "cloak_moe");
  }
  return CLOAK_OK;
}

extern "C" int cloak_stream_read(const void* d_src, uint64_t bytes, uint32_t* d_out, void* stream) {
  clear_error();
  if (!d_src || !d_out || bytes % 16 != 0 || reinterpret_cast<uintptr_t>(d_src) % 16 != 0 || bytes > uint64_t(INT64_MAX)) {
    set_error("cloak_stream_read: need a 16-byte aligned buffer of a multiple of 16 bytes and an output word");
    return CLOAK_EINVAL;
  }
  HIP_TRY(launch_stream_read(d_src, int64_t(bytes), d_out, static_cast<hipStream_t>(stream)), "cloak_stream_read");
  return CLOAK_OK;
}

extern "C" int cloak_quantize_fp8(const void* d_x, int64_t M, int64_t K, int64_t ldx, void* d_q, void* d_s,
                                  void* stream) {
  using namespace cloak;
  if (M < 0 || M > INT32_MAX || K < 1 || ldx < K) {
    set_error("cloak_quantize_fp8: bad sizes M=%lld K=%lld ldx=%lld", (long long)M, (long long)K, (long long)ldx);
    return CLOAK_EINVAL;
  }
  if (M == 0) return CLOAK_OK;
  if (!d_x || !d_q || !d_s) {
    set_error("cloak_quantize_fp8: null buffer");
    return CLOAK_EINVAL;
  }
  HIP_TRY(launch_quant_rows(static_cast<const uint16_t*>(d_x), ldx, nullptr, static_cast<uint8_t*>(d_q),
                            static_cast<float*>(d_s), M, K, static_cast<hipStream_t>(stream)),
          "cloak_quantize_fp8");
  return CLOAK_OK;
}

extern "C" int cloak_remap_step(cloak_layout* L, void* d_pool, int64_t max_pairs, int64_t* remaining, void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_remap_step")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_remap_step")) return rc;
  RemapEpoch& e = L->epoch;
  if (!e.active) {
    set_error("cloak_remap_step: no remap in progress (cloak_remap_begin)");
    return CLOAK_ESTATE;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t left = e.npairs() - e.next;
  // a bounded slice stops at the end of its pass; max_pairs <= 0 runs every
  // remaining pair, one launch per pass (pairs of the two passes share pages)
  const int64_t n = max_pairs <= 0 ? left : std::min(max_pairs, e.launchable());
  hipEvent_t ev = static_cast<hipEvent_t>(L->dev.stage_event);
  // the staging buffer may still feed earlier asynchronous copies
  HIP_TRY(hipEventSynchronize(ev), "hipEventSynchronize");
  int32_t* pairs = L->dev.h_stage;
  int32_t* new_phi = L->dev.h_stage + 2 * L->P;
  if (!e.uploaded) {
    // the whole pair list once per epoch; later slices index into it
    std::memcpy(pairs, e.pairs.data(), e.pairs.size() * 4);
    if (!e.pairs.empty())
      HIP_TRY(hipMemcpyAsync(L->dev.remap_pairs, pairs, e.pairs.size() * 4, hipMemcpyHostToDevice, st),
              "upload pairs");
    e.uploaded = true;
  }
  int64_t done = 0;
  do {  // once with nothing to swap: that closes the epoch
    const int64_t seg = std::min(n - done, e.launchable());
    if (seg > 0) {
      SwapArgs sa{};
      sa.pool = static_cast<uint8_t*>(d_pool);
      sa.pairs = L->dev.remap_pairs + 2 * e.next;
      sa.npairs = seg;
      sa.log2_page = L->log2_page;
      HIP_TRY(launch_swap(sa, st), "swap kernel");
    }
    // with a VMM pool the kernels read the tensor view: once the swaps are
    // done, re-point the two virtual pages of every swapped pair
    std::vector<int32_t> moved;
    if (L->vmm.active && seg > 0) {
      moved.reserve(size_t(4 * seg));
      for (int64_t i = e.next; i < e.next + seg; ++i) {
        const int32_t a = e.pairs[2 * i], b = e.pairs[2 * i + 1];
        moved.insert(moved.end(), {e.where[a], e.where[b], a, b});
      }
    }
    remap_epoch_advance(L, seg);
    if (!moved.empty()) {
      HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
      for (size_t i = 0; i < moved.size(); i += 4)
        HIP_TRY(vmm_repoint(L, moved[i], moved[i + 1], moved[i + 2], moved[i + 3]), "remap of the tensor view");
    }
    done += seg;
  } while (done < n);
  // the device map follows in stream order, so the next kernel sees the
  // pages where they now are
  L->dev.phi_key = mask_map(L, new_phi);
  HIP_TRY(hipMemcpyAsync(L->dev.phi, new_phi, size_t(L->P) * 4, hipMemcpyHostToDevice, st), "upload page map");
  HIP_TRY(hipEventRecord(ev, st), "hipEventRecord");
  if (remaining) *remaining = left - n;
  return CLOAK_OK;
}

extern "C" int cloak_remap(cloak_layout* L, void* d_pool, uint64_t remap_seed, void* stream) {
  clear_error();
  if (int rc = check_device_state(L, "cloak_remap")) return rc;
  if (int rc = check_pool(L, d_pool, "cloak_remap")) return rc;
  if (int rc = cloak_remap_begin(L, remap_seed)) return rc;
  return cloak_remap_step(L, d_pool, 0, nullptr, stream);
}

// Native decoder-step driver for the serving loop: one C call enqueues every
// kernel of a step (embedding through argmax), so the host pays one call per
// step instead of ~10 per layer.  The projections are the cloaked entry
// points (cloak_linear_fused / cloak_linear / cloak_swiglu / cloak_down),
// which pick the GEMV or the MFMA GEMM by token count.  Like the FFN's hidden
// units, attention runs on the heads in their stored (permuted) order: q/k/v
// results are not scattered and o reads the attention output as stored.

#include <hip/hip_runtime.h>

#include <cmath>
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

struct cloak_model {
  const cloak_layout* L = nullptr;
  const void* pool = nullptr;
  cloak_model_config cfg{};
  const uint16_t* gains = nullptr;
  uint16_t* kv = nullptr;
  std::vector<int32_t> t;  // per layer: q k v o gate up down
  int32_t embed = -1, head = -1;
  // Projection scratch is not monotone in the token count (the split-K
  // kernels need FP32 partial sums, the larger GEMM none), so the workspace
  // reserves the largest need over every count up to the step's: prefix
  // maxima over token counts (layers) and logit-row counts (head), grown on
  // demand.
  std::vector<uint64_t> sc_tok{0}, sc_head{0};
};

namespace {

constexpr int kPerLayer = 7;
const int32_t kKinds[kPerLayer] = {CLOAK_Q, CLOAK_K, CLOAK_V, CLOAK_O, CLOAK_GATE, CLOAK_UP, CLOAK_DOWN};

uint64_t align256(uint64_t b) { return (b + 255) / 256 * 256; }

struct WsPlan {
  uint64_t r, h, qkv, attn, o, f, y, hsel, logits, part_o, part_ml, scratch, scratch_bytes, total;
};

uint64_t umax(uint64_t a, uint64_t b) { return a > b ? a : b; }

// Largest projection scratch over every token count 1..n (head: logit rows).
uint64_t scratch_bound(const cloak_model* cm, int64_t n, bool head) {
  cloak_model* m = const_cast<cloak_model*>(cm);
  std::vector<uint64_t>& v = head ? m->sc_head : m->sc_tok;
  const int32_t* t = m->t.data();
  while (int64_t(v.size()) <= n) {
    const int64_t k = int64_t(v.size());
    uint64_t need;
    if (head) {
      need = linear_fused_ws_bytes(m->L, &m->head, 1, k);
    } else {
      need = linear_fused_ws_bytes(m->L, t, 3, k);
      need = umax(need, linear_fused_ws_bytes(m->L, t + 3, 1, k));
      need = umax(need, cloak_ws_bytes(m->L, CLOAK_OP_SWIGLU, 0, k));
      need = umax(need, cloak_ws_bytes(m->L, CLOAK_OP_DOWN, 0, k));
    }
    v.push_back(umax(v.back(), need));
  }
  return v[n > 0 ? n : 0];
}

WsPlan plan_ws(const cloak_model* m, int64_t T, int64_t R, int64_t tiles, int64_t splits) {
  const cloak_model_config& c = m->cfg;
  const int64_t D = c.d_model, KVD = int64_t(c.n_kv_heads) * c.head_dim;
  WsPlan p{};
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = off;
    off += align256(bytes);
    return at;
  };
  p.r = take(uint64_t(T) * D * 2);
  p.h = take(uint64_t(T) * D * 2);
  p.qkv = take(uint64_t(T) * (D + 2 * KVD) * 2);
  p.attn = take(uint64_t(T) * D * 2);
  p.o = take(uint64_t(T) * D * 2);
  p.f = take(uint64_t(T) * c.d_ffn * 2);
  p.y = take(uint64_t(T) * D * 2);
  p.hsel = take(uint64_t(R > 0 ? R : 1) * D * 2);
  p.logits = take(uint64_t(R > 0 ? R : 1) * c.vocab * 2);
  p.part_o = take(uint64_t(tiles) * splits * c.n_heads * 16 * 128 * 4);
  p.part_ml = take(uint64_t(tiles) * splits * c.n_heads * 16 * 2 * 4);
  // scratch of the projections (split-K partial sums, quantised
  // activations); all layers share shapes
  p.scratch_bytes = align256(umax(scratch_bound(m, T, false), scratch_bound(m, R, true)));
  p.scratch = take(p.scratch_bytes);
  p.total = off;
  return p;
}

}  // namespace

extern "C" int cloak_model_create(const cloak_layout* L, const void* d_pool, const cloak_model_config* cfg,
                                  const void* d_gains, void* d_kv, cloak_model** out) {
  clear_error();
  if (!L || !d_pool || !cfg || !d_kv || !out) {
    set_error("cloak_model_create: null argument");
    return CLOAK_EINVAL;
  }
  *out = nullptr;
  const cloak_model_config& c = *cfg;
  if (c.n_layers <= 0 || c.d_model <= 0 || c.n_heads <= 0 || c.n_kv_heads <= 0 || c.head_dim != 128 ||
      c.n_heads % c.n_kv_heads != 0 || c.n_heads / c.n_kv_heads > 8 || c.n_heads * c.head_dim != c.d_model ||
      c.d_ffn <= 0 || c.vocab <= 0 || c.block_size <= 0 || c.num_blocks <= 0 || !(c.norm_eps > 0.f) ||
      !(c.rope_theta > 0.f)) {
    set_error("cloak_model_create: unsupported config (head_dim must be 128, n_heads*128 == d_model, "
              "n_heads/n_kv_heads in 1..8)");
    return CLOAK_EINVAL;
  }
  if (reinterpret_cast<uintptr_t>(d_pool) % 256 != 0) {
    set_error("cloak_model_create: pool must be 256-byte aligned");
    return CLOAK_EINVAL;
  }
  if (!L->dev.phi) {
    set_error("cloak_model_create: layout has no device tables");
    return CLOAK_ESTATE;
  }
  auto m = new (std::nothrow) cloak_model();
  if (!m) {
    set_error("cloak_model_create: out of host memory");
    return CLOAK_ENOMEM;
  }
  m->L = L;
  m->pool = d_pool;
  m->cfg = c;
  m->gains = static_cast<const uint16_t*>(d_gains);
  m->kv = static_cast<uint16_t*>(d_kv);
  const int64_t D = c.d_model, KVD = int64_t(c.n_kv_heads) * c.head_dim, F = c.d_ffn;
  const int64_t want_n[kPerLayer] = {D, KVD, KVD, D, F, F, D};
  const int64_t want_k[kPerLayer] = {D, D, D, D, D, D, F};
  for (int l = 0; l < c.n_layers; ++l) {
    for (int i = 0; i < kPerLayer; ++i) {
      const int t = L->find_tensor(l, kKinds[i]);
      if (t < 0 || L->tensors[t].shape.n_out != want_n[i] || L->tensors[t].shape.k_in != want_k[i] ||
          L->tensors[t].shape.dtype != CLOAK_BF16) {
        set_error("cloak_model_create: layer %d kind %d missing or not a BF16 [%lld][%lld] tensor", l, kKinds[i],
                  (long long)want_n[i], (long long)want_k[i]);
        delete m;
        return CLOAK_ESHAPE;
      }
      m->t.push_back(t);
    }
    const AttnPerm* ap = L->attn_of_layer(l);
    if (ap && ap->head_dim != c.head_dim) {
      set_error("cloak_model_create: layer %d is head-permuted with head_dim %lld, the model uses %d", l,
                (long long)ap->head_dim, c.head_dim);
      delete m;
      return CLOAK_ESHAPE;
    }
  }
  m->embed = L->find_tensor(-1, CLOAK_EMBED);
  m->head = L->find_tensor(-1, CLOAK_HEAD);
  for (int t : {m->embed, m->head}) {
    if (t < 0 || L->tensors[t].shape.n_out != c.vocab || L->tensors[t].shape.k_in != D ||
        L->tensors[t].shape.dtype != CLOAK_BF16) {
      set_error("cloak_model_create: embed/head must be BF16 [vocab][d_model] tensors of layer -1");
      delete m;
      return CLOAK_ESHAPE;
    }
  }
  *out = m;
  return CLOAK_OK;
}

extern "C" int cloak_model_free(cloak_model* m) {
  delete m;
  return CLOAK_OK;
}

extern "C" uint64_t cloak_model_ws_bytes(const cloak_model* m, int64_t max_tokens, int64_t max_logits,
                                         int64_t max_tiles, int64_t max_splits) {
  if (!m || max_tokens < 0 || max_logits < 0 || max_tiles < 0 || max_splits < 0) return UINT64_MAX;
  return plan_ws(m, max_tokens, max_logits, max_tiles, max_splits).total;
}

extern "C" int cloak_model_step(cloak_model* m, const cloak_step* s, void* d_ws, uint64_t ws_bytes, void* stream) {
  clear_error();
  if (!m || !s || !d_ws) {
    set_error("cloak_model_step: null argument");
    return CLOAK_EINVAL;
  }
  const cloak_model_config& c = m->cfg;
  const int64_t T = s->n_tokens, R = s->n_logits;
  if (T <= 0 || s->n_seqs <= 0 || R < 0 || R > T || s->max_blocks <= 0 || s->n_tiles <= 0 || s->n_splits <= 0 ||
      s->split_keys <= 0 || s->n_single < 0 || s->n_single > s->n_tiles || !s->d_tokens || !s->d_positions || !s->d_tok_seq || !s->d_block_table ||
      !s->d_tile_seq || !s->d_tile_tok0 || !s->d_tile_ntok || (R > 0 && (!s->d_logit_rows || !s->d_out_tokens))) {
    set_error("cloak_model_step: bad batch description");
    return CLOAK_EINVAL;
  }
  const WsPlan p = plan_ws(m, T, R, s->n_tiles, s->n_splits);
  if (ws_bytes < p.total) {
    set_error("cloak_model_step: workspace of %llu bytes, step needs %llu", (unsigned long long)ws_bytes,
              (unsigned long long)p.total);
    return CLOAK_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const cloak_layout* L = m->L;
  auto* base = static_cast<uint8_t*>(d_ws);
  auto bf = [&](uint64_t off) { return reinterpret_cast<uint16_t*>(base + off); };
  uint16_t *r = bf(p.r), *h = bf(p.h), *qkv = bf(p.qkv), *attn = bf(p.attn), *o = bf(p.o), *f = bf(p.f),
           *y = bf(p.y), *hsel = bf(p.hsel);
  uint16_t* logits = s->d_out_logits ? static_cast<uint16_t*>(s->d_out_logits) : bf(p.logits);
  void* scratch = base + p.scratch;
  const uint64_t sb = p.scratch_bytes;
  const int64_t D = c.d_model, KVD = int64_t(c.n_kv_heads) * c.head_dim;
  const int64_t layer_kv = int64_t(c.num_blocks) * c.n_kv_heads * c.block_size * c.head_dim;

  // embedding rows, read through the page map
  {
    const TensorInfo& te = L->tensors[m->embed];
    EmbedArgs e{};
    e.pool = static_cast<const uint8_t*>(L->kernel_pool(m->pool));
    e.phi = L->dev.phi;
    e.phi_key = L->dev.phi_key;
    e.log2_page = L->log2_page;
    e.translate = L->kernel_translate() ? 1 : 0;
    e.vbase = te.vbase;
    e.vocab = c.vocab;
    e.row_bytes = int32_t(D * 2);
    e.ids = s->d_tokens;
    e.T = int32_t(T);
    e.out = r;
    HIP_TRY(launch_embed(e, st), "cloak_model_step(embed)");
  }
  for (int l = 0; l < c.n_layers; ++l) {
    const int32_t* t = &m->t[size_t(l) * kPerLayer];
    NormArgs na{};
    na.x = r;
    na.add = l == 0 ? nullptr : y;
    na.r_out = l == 0 ? nullptr : r;
    na.gain = m->gains ? m->gains + int64_t(2 * l) * D : nullptr;
    na.h = h;
    na.rows = nullptr;
    na.D = int32_t(D);
    na.eps = c.norm_eps;
    HIP_TRY(launch_rmsnorm(na, int(T), st), "cloak_model_step(norm)");
    if (int rc = cloak_linear_stored(L, m->pool, t, 3, h, T, qkv, scratch, sb, stream)) return rc;
    uint16_t* kc = m->kv + int64_t(2 * l) * layer_kv;
    uint16_t* vc = kc + layer_kv;
    RopeArgs ra{};
    ra.qkv = qkv;
    ra.ldqkv = D + 2 * KVD;
    ra.positions = s->d_positions;
    ra.tok_seq = s->d_tok_seq;
    ra.block_table = s->d_block_table;
    ra.max_blocks = s->max_blocks;
    ra.bs = c.block_size;
    ra.n_heads = c.n_heads;
    ra.n_kv = c.n_kv_heads;
    ra.hd = c.head_dim;
    ra.theta = c.rope_theta;
    ra.num_blocks = c.num_blocks;
    ra.kc = kc;
    ra.vc = vc;
    HIP_TRY(launch_rope_kv(ra, int(T), st), "cloak_model_step(rope)");
    AttnArgs aa{};
    aa.q = qkv;
    aa.ldq = D + 2 * KVD;
    aa.kc = kc;
    aa.vc = vc;
    aa.block_table = s->d_block_table;
    aa.max_blocks = s->max_blocks;
    aa.bs = c.block_size;
    aa.num_blocks = c.num_blocks;
    aa.tile_seq = s->d_tile_seq;
    aa.tile_tok0 = s->d_tile_tok0;
    aa.tile_ntok = s->d_tile_ntok;
    aa.positions = s->d_positions;
    aa.n_tiles = s->n_tiles;
    aa.n_single = s->n_single;
    aa.n_splits = s->n_splits;
    aa.split_keys = s->split_keys;
    aa.n_heads = c.n_heads;
    aa.n_kv = c.n_kv_heads;
    aa.scale = 1.0f / std::sqrt(float(c.head_dim));
    aa.part_o = reinterpret_cast<float*>(base + p.part_o);
    aa.part_ml = reinterpret_cast<float*>(base + p.part_ml);
    aa.out = attn;
    aa.ldo = D;
    HIP_TRY(launch_attention(aa, st), "cloak_model_step(attention)");
    if (int rc = cloak_linear_stored(L, m->pool, t + 3, 1, attn, T, o, scratch, sb, stream)) return rc;
    NormArgs nb = na;
    nb.add = o;
    nb.r_out = r;
    nb.gain = m->gains ? m->gains + int64_t(2 * l + 1) * D : nullptr;
    HIP_TRY(launch_rmsnorm(nb, int(T), st), "cloak_model_step(norm)");
    if (int rc = cloak_swiglu(L, m->pool, l, h, T, f, scratch, sb, stream)) return rc;
    if (int rc = cloak_down(L, m->pool, l, f, T, y, scratch, sb, stream)) return rc;
  }
  if (R == 0) return CLOAK_OK;
  NormArgs nf{};
  nf.x = r;
  nf.add = y;
  nf.r_out = nullptr;
  nf.gain = m->gains ? m->gains + int64_t(2 * c.n_layers) * D : nullptr;
  nf.h = hsel;
  nf.rows = s->d_logit_rows;
  nf.D = int32_t(D);
  nf.eps = c.norm_eps;
  HIP_TRY(launch_rmsnorm(nf, int(R), st), "cloak_model_step(final norm)");
  if (int rc = cloak_linear(L, m->pool, m->head, hsel, R, logits, scratch, sb, stream)) return rc;
  HIP_TRY(launch_argmax(logits, R, c.vocab, s->d_out_tokens, st), "cloak_model_step(argmax)");
  return CLOAK_OK;
}

// Layout core of libcloak: seeded draws, the layout descriptor, host-side
// page streams and the remap matching.  Pure host C++; the definitions it
// implements are written out in include/cloak.h (CloakLM, arXiv 2606.18400:
// inter-layer order Section 4.2 / Table 1a, page placement Section 4.2 /
// Table 1b, seeding before transfer Section 5).

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "cloak_internal.hpp"

namespace cloak {

static thread_local std::string g_error;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
}
void clear_error() { g_error.clear(); }
const char* last_error() { return g_error.c_str(); }

// SplitMix64: Weyl state advanced by the golden-ratio increment, output
// through the variant-13 finaliser (Steele, Lea, Flood, OOPSLA 2014).
uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t SplitMix64::next() {
  state += 0x9E3779B97F4A7C15ull;
  return mix64(state);
}

SplitMix64 substream(uint64_t seed, uint32_t tag, uint32_t idx) {
  SplitMix64 g;
  g.state = mix64(seed ^ mix64((uint64_t(tag) << 32) | uint64_t(idx)));
  return g;
}

// Uniform draw on [0, n): the 2^64 mod n smallest outputs are rejected so the
// remaining range is a whole number of copies of [0, n).
Stream stream(uint64_t seed, uint32_t tag, uint32_t idx, bool csprng) {
  Stream g;
  g.sha = csprng;
  if (csprng)
    g.ctr = sha256_substream(seed, tag, idx);
  else
    g.sm = substream(seed, tag, idx);
  return g;
}

uint64_t bounded(Stream& g, uint64_t n) {
  const uint64_t reject_below = (0 - n) % n;  // == 2^64 mod n
  for (;;) {
    uint64_t r = g.next();
    if (r >= reject_below) return r % n;
  }
}

// Durstenfeld's in-place Fisher-Yates walk from the top slot down.
std::vector<int32_t> fisher_yates(int64_t n, Stream g) { return fisher_yates_from(n, g); }

std::vector<int32_t> fisher_yates_from(int64_t n, Stream& g) {
  std::vector<int32_t> a(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) a[i] = static_cast<int32_t>(i);
  for (int64_t i = n - 1; i >= 1; --i) {
    int64_t j = static_cast<int64_t>(bounded(g, static_cast<uint64_t>(i + 1)));
    std::swap(a[i], a[j]);
  }
  return a;
}

std::vector<int32_t> upload_order(const cloak_layout* L, int32_t t) {
  const int64_t n = L->tensors[t].npages;
  if (L->identity()) {
    std::vector<int32_t> a(n);
    for (int64_t i = 0; i < n; ++i) a[i] = int32_t(i);
    return a;
  }
  return fisher_yates(n, stream(L->seed, kTagUpload, uint32_t(t), L->csprng()));
}

std::vector<int32_t> remap_matching(uint64_t remap_seed, int64_t P, bool csprng) {
  std::vector<int32_t> s = fisher_yates(P, stream(remap_seed, kTagRemap, 0, csprng));
  std::vector<int32_t> tau(P);
  for (int64_t p = 0; p < P; ++p) tau[p] = int32_t(p);
  for (int64_t i = 0; 2 * i + 1 < P; ++i) {
    tau[s[2 * i]] = s[2 * i + 1];
    tau[s[2 * i + 1]] = s[2 * i];
  }
  return tau;
}

std::vector<int32_t> remap_uniform_draw(uint64_t remap_seed, int64_t P, bool csprng) {
  return fisher_yates(P, stream(remap_seed, kTagRemap, 1, csprng));
}

// A cycle c_0 -> c_1 -> ... -> c_{k-1} -> c_0 of rho (c_0 its smallest page)
// shifts contents by one place.  That shift is the reflection i -> -i
// (mod k) followed by the reflection i -> 1 - i, and each reflection is a
// set of disjoint transpositions: pass 1 pairs c_i with c_{k-i}, pass 2
// pairs c_0 with c_1 and c_i with c_{k+1-i}.  Together they use k - 1 swaps.
void remap_uniform_passes(const std::vector<int32_t>& rho, std::vector<int32_t>& pass1, std::vector<int32_t>& pass2) {
  const int64_t P = int64_t(rho.size());
  std::vector<std::pair<int32_t, int32_t>> one, two;
  std::vector<char> seen(size_t(P), 0);
  std::vector<int32_t> c;
  for (int64_t start = 0; start < P; ++start) {
    if (seen[size_t(start)]) continue;
    c.clear();
    for (int32_t q = int32_t(start); !seen[size_t(q)]; q = rho[size_t(q)]) {
      seen[size_t(q)] = 1;
      c.push_back(q);
    }
    const int64_t k = int64_t(c.size());
    auto lohi = [](int32_t a, int32_t b) { return a < b ? std::make_pair(a, b) : std::make_pair(b, a); };
    for (int64_t i = 1; 2 * i < k; ++i) one.push_back(lohi(c[size_t(i)], c[size_t(k - i)]));
    if (k > 1) two.push_back(lohi(c[0], c[1]));
    for (int64_t i = 2; 2 * i < k + 1; ++i) two.push_back(lohi(c[size_t(i)], c[size_t(k + 1 - i)]));
  }
  std::sort(one.begin(), one.end());
  std::sort(two.begin(), two.end());
  pass1.clear();
  pass2.clear();
  for (const auto& q : one) pass1.insert(pass1.end(), {q.first, q.second});
  for (const auto& q : two) pass2.insert(pass2.end(), {q.first, q.second});
}

bool remap_epoch_begin(cloak_layout* L, uint64_t remap_seed) {
  RemapEpoch& e = L->epoch;
  if (e.active) return false;
  e.pairs.clear();
  if (L->uniform_remap()) {
    std::vector<int32_t> two;
    remap_uniform_passes(remap_uniform_draw(remap_seed, L->P, L->csprng()), e.pairs, two);
    e.pass_end = e.npairs();
    e.pairs.insert(e.pairs.end(), two.begin(), two.end());
  } else {
    const std::vector<int32_t> tau = remap_matching(remap_seed, L->P, L->csprng());
    for (int64_t p = 0; p < L->P; ++p)
      if (tau[p] > p) {
        e.pairs.push_back(int32_t(p));
        e.pairs.push_back(tau[p]);
      }
    e.pass_end = e.npairs();
  }
  e.where.assign(size_t(L->P), 0);
  for (int64_t v = 0; v < L->P; ++v) e.where[size_t(L->phi[v])] = int32_t(v);
  e.next = 0;
  e.uploaded = false;
  e.active = true;
  return true;
}

void remap_epoch_advance(cloak_layout* L, int64_t n) {
  RemapEpoch& e = L->epoch;
  for (int64_t i = e.next; i < e.next + n; ++i) {
    const int32_t a = e.pairs[2 * i], b = e.pairs[2 * i + 1];
    const int32_t va = e.where[a], vb = e.where[b];
    L->phi[va] = b;
    L->phi[vb] = a;
    e.where[a] = vb;
    e.where[b] = va;
  }
  e.next += n;
  if (e.next >= e.npairs()) {
    e.active = false;
    L->remaps += 1;
  }
}

double contiguity(const cloak_layout* L) {
  int64_t hits = 0, total = 0;
  for (const auto& ti : L->tensors) {
    for (int64_t i = 0; i + 1 < ti.npages; ++i) {
      ++total;
      hits += (L->phi[ti.vbase + i + 1] == L->phi[ti.vbase + i] + 1);
    }
  }
  return total ? double(hits) / double(total) : 1.0;
}

// d[e - e0] = srow[pi[e]] for e in [e0, e1), elements of `elt` bytes.
static void gather_elements(uint8_t* d, const uint8_t* srow, const int32_t* pi, int64_t e0, int64_t e1, int elt) {
  if (elt == 2) {
    auto* dd = reinterpret_cast<uint16_t*>(d);
    for (int64_t e = e0; e < e1; ++e) std::memcpy(dd + (e - e0), srow + int64_t(pi[e]) * 2, 2);
  } else if (elt == 4) {
    auto* dd = reinterpret_cast<uint32_t*>(d);
    for (int64_t e = e0; e < e1; ++e) std::memcpy(dd + (e - e0), srow + int64_t(pi[e]) * 4, 4);
  } else {
    for (int64_t e = e0; e < e1; ++e) d[e - e0] = srow[pi[e]];
  }
}

// Bytes [page*B, page*B + B) of tensor t's shuffled stream, built from the
// logical array `src`; bytes past the tensor are zero.
void stream_page(const cloak_layout* L, int32_t t, const uint8_t* src, int64_t page, uint8_t* dst) {
  const TensorInfo& ti = L->tensors[t];
  const int64_t B = L->page_bytes;
  const int64_t begin = page * B;
  const int64_t end = std::min(begin + B, ti.bytes);
  std::memset(dst, 0, size_t(B));
  if (begin >= end) return;
  const int64_t rb = ti.row_bytes;
  const int elt = elt_bytes(ti.shape.dtype);
  const int32_t* rp = L->row_perm(t);
  const int32_t* cp = L->col_perm(t);
  int64_t o = begin;
  while (o < end) {
    const int64_t row = o / rb;
    const int64_t col = o % rb;
    const int64_t seg = std::min(end - o, rb - col);
    // stored row `row` is logical row rp[row]; its element e is logical element cp[e]
    const uint8_t* srow = src + int64_t(rp ? rp[row] : row) * rb;
    if (cp) {
      gather_elements(dst + (o - begin), srow, cp, col / elt, (col + seg) / elt, elt);
    } else {
      std::memcpy(dst + (o - begin), srow + col, size_t(seg));
    }
    o += seg;
  }
}

// Inverse of stream_page: scatter one page of the stream back into the
// logical array `dst`.
void unstream_page(const cloak_layout* L, int32_t t, const uint8_t* pagebuf, int64_t page, uint8_t* dst) {
  const TensorInfo& ti = L->tensors[t];
  const int64_t B = L->page_bytes;
  const int64_t begin = page * B;
  const int64_t end = std::min(begin + B, ti.bytes);
  if (begin >= end) return;
  const int64_t rb = ti.row_bytes;
  const int elt = elt_bytes(ti.shape.dtype);
  const int32_t* rp = L->row_perm(t);
  const int32_t* cp = L->col_perm(t);
  int64_t o = begin;
  while (o < end) {
    const int64_t row = o / rb;
    const int64_t col = o % rb;
    const int64_t seg = std::min(end - o, rb - col);
    uint8_t* drow = dst + int64_t(rp ? rp[row] : row) * rb;
    const uint8_t* sp = pagebuf + (o - begin);
    if (cp) {
      const int64_t e0 = col / elt, e1 = (col + seg) / elt;
      for (int64_t e = e0; e < e1; ++e) std::memcpy(drow + int64_t(cp[e]) * elt, sp + (e - e0) * elt, size_t(elt));
    } else {
      std::memcpy(drow + col, sp, size_t(seg));
    }
    o += seg;
  }
}

}  // namespace cloak

int cloak_layout::find_tensor(int32_t layer, int32_t kind) const {
  for (size_t t = 0; t < tensors.size(); ++t)
    if (tensors[t].shape.layer == layer && tensors[t].shape.kind == kind) return int(t);
  return -1;
}

const cloak::FfnPerm* cloak_layout::ffn_of_layer(int32_t layer) const {
  for (const auto& f : ffn)
    if (f.layer == layer) return &f;
  return nullptr;
}

const cloak::AttnPerm* cloak_layout::attn_of_layer(int32_t layer) const {
  for (const auto& a : attn)
    if (a.layer == layer) return &a;
  return nullptr;
}

using namespace cloak;

extern "C" const char* cloak_last_error(void) { return cloak::last_error(); }

namespace cloak {
void (*release_device_state)(cloak_layout*) = nullptr;
}

extern "C" int cloak_layout_free(cloak_layout* L) {
  clear_error();
  if (!L) return CLOAK_OK;
  if (release_device_state) release_device_state(L);
  delete L;
  return CLOAK_OK;
}

extern "C" int cloak_layout_build(uint64_t seed, const cloak_shape* shapes, int32_t n_shapes,
                                  uint64_t page_bytes, uint64_t pool_bytes, uint32_t flags,
                                  cloak_layout** out) {
  clear_error();
  if (!out || (!shapes && n_shapes > 0) || n_shapes < 0) {
    set_error("cloak_layout_build: null argument or negative count");
    return CLOAK_EINVAL;
  }
  *out = nullptr;
  if (page_bytes < 1024 || (page_bytes & (page_bytes - 1)) != 0) {
    set_error("cloak_layout_build: page_bytes must be a power of two >= 1024 (got %llu)",
              (unsigned long long)page_bytes);
    return CLOAK_EINVAL;
  }
  if (pool_bytes == 0 || pool_bytes % page_bytes != 0) {
    set_error("cloak_layout_build: pool_bytes must be a positive multiple of page_bytes");
    return CLOAK_EINVAL;
  }
  if ((flags & ~(CLOAK_IDENTITY | CLOAK_NATIVE | CLOAK_CSPRNG | CLOAK_MASKED_MAP | CLOAK_REMAP_UNIFORM)) != 0 ||
      ((flags & CLOAK_NATIVE) && !(flags & CLOAK_IDENTITY))) {
    set_error("cloak_layout_build: bad flags 0x%x (CLOAK_NATIVE needs CLOAK_IDENTITY)", flags);
    return CLOAK_EINVAL;
  }
  const int64_t P = int64_t(pool_bytes / page_bytes);
  if (P > INT32_MAX) {
    set_error("cloak_layout_build: too many pages");
    return CLOAK_EINVAL;
  }
  auto L = new (std::nothrow) cloak_layout();
  if (!L) {
    set_error("cloak_layout_build: out of host memory");
    return CLOAK_ENOMEM;
  }
  L->seed = seed;
  L->flags = flags;
  L->map_keys = sha256_substream(seed, kTagMapKey, 0);
  L->page_bytes = int64_t(page_bytes);
  while ((int64_t(1) << L->log2_page) < L->page_bytes) ++L->log2_page;
  L->pool_bytes = int64_t(pool_bytes);
  L->P = P;
  const bool ident = (flags & CLOAK_IDENTITY) != 0;

  // Validate shapes and collect the FFN groups and head-permuted layers.
  L->tensors.resize(n_shapes);
  for (int32_t t = 0; t < n_shapes; ++t) {
    const cloak_shape& s = shapes[t];
    if (s.kind < CLOAK_Q || s.kind > CLOAK_HEAD || s.dtype < CLOAK_F32 || s.dtype > CLOAK_FP8_E4M3 ||
        s.n_out <= 0 || s.k_in <= 0 || s.n_out > INT32_MAX || s.k_in > INT32_MAX || s.head_dim < 0 ||
        (s.head_dim > 0 && !is_attn(s.kind))) {
      set_error("cloak_layout_build: tensor %d has a bad kind/dtype/size/head_dim", t);
      delete L;
      return CLOAK_EINVAL;
    }
    for (int32_t u = 0; u < t; ++u) {
      if (shapes[u].layer == s.layer && shapes[u].kind == s.kind) {
        set_error("cloak_layout_build: tensors %d and %d are both (layer %d, kind %d)", u, t, s.layer, s.kind);
        delete L;
        return CLOAK_ESHAPE;
      }
    }
    TensorInfo& ti = L->tensors[t];
    ti.shape = s;
    ti.row_bytes = s.k_in * elt_bytes(s.dtype);
    ti.bytes = s.n_out * ti.row_bytes;
    ti.npages = (ti.bytes + L->page_bytes - 1) / L->page_bytes;
    if (is_ffn_row(s.kind) || is_ffn_col(s.kind)) {
      const int64_t h = is_ffn_row(s.kind) ? s.n_out : s.k_in;
      int idx = -1;
      for (size_t f = 0; f < L->ffn.size(); ++f)
        if (L->ffn[f].layer == s.layer) idx = int(f);
      if (idx < 0) {
        FfnPerm fp;
        fp.layer = s.layer;
        fp.d_ffn = h;
        L->ffn.push_back(fp);
        idx = int(L->ffn.size()) - 1;
      } else if (L->ffn[idx].d_ffn != h) {
        set_error("cloak_layout_build: layer %d hidden sizes disagree (%lld vs %lld)", s.layer,
                  (long long)L->ffn[idx].d_ffn, (long long)h);
        delete L;
        return CLOAK_ESHAPE;
      }
      if (s.kind == CLOAK_GATE) L->ffn[idx].gate = t;
      if (s.kind == CLOAK_UP) L->ffn[idx].up = t;
      if (s.kind == CLOAK_DOWN) L->ffn[idx].down = t;
    }
    if (s.head_dim > 0) {
      int idx = -1;
      for (size_t a = 0; a < L->attn.size(); ++a)
        if (L->attn[a].layer == s.layer) idx = int(a);
      if (idx < 0) {
        AttnPerm ap;
        ap.layer = s.layer;
        ap.head_dim = s.head_dim;
        L->attn.push_back(ap);
        idx = int(L->attn.size()) - 1;
      }
      AttnPerm& ap = L->attn[idx];
      (s.kind == CLOAK_Q ? ap.q : s.kind == CLOAK_K ? ap.k : s.kind == CLOAK_V ? ap.v : ap.o) = t;
    }
    if (s.dtype == CLOAK_FP8_E4M3) {
      ti.scale_off = L->n_scales;
      L->n_scales += s.n_out;
    }
  }
  // A head-permuted layer needs all four attention tensors, with whole heads.
  for (AttnPerm& a : L->attn) {
    const int32_t idx[4] = {a.q, a.k, a.v, a.o};
    bool ok = a.layer >= 0;
    for (int i = 0; i < 4 && ok; ++i) {
      if (idx[i] >= 0) continue;
      // a q/k/v/o of this layer without the head size counts as missing
      ok = false;
    }
    if (ok) {
      const cloak_shape &q = shapes[a.q], &k = shapes[a.k], &v = shapes[a.v], &o = shapes[a.o];
      const int64_t hd = a.head_dim;
      ok = q.head_dim == hd && k.head_dim == hd && v.head_dim == hd && o.head_dim == hd && q.n_out % hd == 0 &&
           k.n_out % hd == 0 && v.n_out == k.n_out && o.k_in == q.n_out && q.k_in == k.k_in && k.k_in == v.k_in &&
           (q.n_out / hd) % (k.n_out / hd) == 0;
      if (ok) {
        a.n_kv = k.n_out / hd;
        a.group = q.n_out / hd / a.n_kv;
      }
    }
    if (!ok) {
      set_error("cloak_layout_build: layer %d: q, k, v and o must all carry one head_dim, form whole heads "
                "(Hq a multiple of Hkv, o's K = q's N) and have layer >= 0", a.layer);
      delete L;
      return CLOAK_ESHAPE;
    }
  }

  // Inter-layer shuffle: tensor order in the virtual page stream.
  if (ident) {
    L->sigma.resize(n_shapes);
    for (int32_t i = 0; i < n_shapes; ++i) L->sigma[i] = i;
  } else {
    L->sigma = fisher_yates(n_shapes, stream(seed, kTagTensorOrder, 0, L->csprng()));
  }
  auto iota = [](int64_t n) {
    std::vector<int32_t> a(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) a[size_t(i)] = int32_t(i);
    return a;
  };
  auto add_table = [&](std::vector<int32_t> p) {
    PermTable pt;
    pt.p = std::move(p);
    pt.dev_off = L->n_perm;
    L->n_perm += int64_t(pt.p.size());
    L->perms.push_back(std::move(pt));
    return int32_t(L->perms.size()) - 1;
  };
  // Intra-layer shuffle: hidden-neuron permutation of each FFN.
  for (auto& f : L->ffn) {
    f.table = add_table(ident ? iota(f.d_ffn) : fisher_yates(f.d_ffn, stream(seed, kTagHiddenPerm, uint32_t(f.layer), L->csprng())));
    for (int32_t t : {f.gate, f.up})
      if (t >= 0) L->tensors[t].row_perm = f.table;
    if (f.down >= 0) L->tensors[f.down].col_perm = f.table;
  }
  L->ffn_by_layer.resize(L->ffn.size());
  for (size_t f = 0; f < L->ffn.size(); ++f) L->ffn_by_layer[f] = int32_t(f);
  std::sort(L->ffn_by_layer.begin(), L->ffn_by_layer.end(),
            [&](int32_t a, int32_t b) { return L->ffn[size_t(a)].layer < L->ffn[size_t(b)].layer; });
  // Attention heads: kv groups, query heads inside a group, value dimensions.
  for (auto& a : L->attn) {
    const int64_t hd = a.head_dim, G = a.group, nkv = a.n_kv;
    if (ident) {
      a.rho = iota(nkv);
      a.theta.clear();
      for (int64_t c = 0; c < nkv; ++c) {
        auto t = iota(G);
        a.theta.insert(a.theta.end(), t.begin(), t.end());
      }
      a.chi = iota(hd);
    } else {
      Stream g = stream(seed, kTagHeadPerm, uint32_t(a.layer), L->csprng());
      a.rho = fisher_yates_from(nkv, g);
      a.theta.clear();
      for (int64_t c = 0; c < nkv; ++c) {
        auto t = fisher_yates_from(G, g);
        a.theta.insert(a.theta.end(), t.begin(), t.end());
      }
      a.chi = fisher_yates_from(hd, g);
    }
    std::vector<int32_t> q, k, v, o;
    for (int64_t c = 0; c < nkv; ++c) {
      for (int64_t i = 0; i < G; ++i) {
        const int64_t h = int64_t(a.rho[c]) * G + a.theta[size_t(c * G + i)];
        for (int64_t d = 0; d < hd; ++d) {
          q.push_back(int32_t(h * hd + d));
          o.push_back(int32_t(h * hd + a.chi[size_t(d)]));
        }
      }
      for (int64_t d = 0; d < hd; ++d) {
        k.push_back(int32_t(int64_t(a.rho[c]) * hd + d));
        v.push_back(int32_t(int64_t(a.rho[c]) * hd + a.chi[size_t(d)]));
      }
    }
    L->tensors[a.q].row_perm = add_table(std::move(q));
    L->tensors[a.k].row_perm = add_table(std::move(k));
    L->tensors[a.v].row_perm = add_table(std::move(v));
    L->tensors[a.o].col_perm = add_table(std::move(o));
  }
  // Virtual pages, tensors in sigma order.
  int64_t cursor = 0;
  for (int32_t i = 0; i < n_shapes; ++i) {
    TensorInfo& ti = L->tensors[L->sigma[i]];
    ti.vbase = cursor;
    cursor += ti.npages;
  }
  L->V = cursor;
  if (L->V > P) {
    set_error("cloak_layout_build: tensors need %lld pages, pool has %lld", (long long)L->V, (long long)P);
    delete L;
    return CLOAK_ENOMEM;
  }
  // Physical placement over the whole pool.
  if (ident) {
    L->phi.resize(P);
    for (int64_t p = 0; p < P; ++p) L->phi[p] = int32_t(p);
  } else {
    L->phi = fisher_yates(P, stream(seed, kTagPageMap, 0, L->csprng()));
  }
  L->loaded.assign(size_t(n_shapes), 0);
  *out = L;
  return CLOAK_OK;
}

extern "C" int cloak_query(const cloak_layout* L, int32_t what, int64_t index, void* out, uint64_t out_bytes) {
  clear_error();
  if (!L || !out) {
    set_error("cloak_query: null argument");
    return CLOAK_EINVAL;
  }
  auto need = [&](uint64_t n) {
    if (out_bytes < n) {
      set_error("cloak_query: buffer of %llu bytes, need %llu", (unsigned long long)out_bytes,
                (unsigned long long)n);
      return false;
    }
    return true;
  };
  const int64_t T = int64_t(L->tensors.size());
  switch (what) {
    case CLOAK_QUERY_REMAP_PENDING: {
      if (!need(8)) return CLOAK_EINVAL;
      *static_cast<int64_t*>(out) = L->epoch.active ? L->epoch.npairs() - L->epoch.next : 0;
      return CLOAK_OK;
    }
    case CLOAK_QUERY_P:
    case CLOAK_QUERY_V:
    case CLOAK_QUERY_T:
    case CLOAK_QUERY_PAGE_BYTES:
    case CLOAK_QUERY_REMAPS: {
      if (!need(8)) return CLOAK_EINVAL;
      int64_t v = what == CLOAK_QUERY_P ? L->P : what == CLOAK_QUERY_V ? L->V : what == CLOAK_QUERY_T ? T
                : what == CLOAK_QUERY_PAGE_BYTES ? L->page_bytes : L->remaps;
      std::memcpy(out, &v, 8);
      return CLOAK_OK;
    }
    case CLOAK_QUERY_PHI:
      if (!need(uint64_t(L->P) * 4)) return CLOAK_EINVAL;
      std::memcpy(out, L->phi.data(), size_t(L->P) * 4);
      return CLOAK_OK;
    case CLOAK_QUERY_SIGMA:
      if (!need(uint64_t(T) * 4)) return CLOAK_EINVAL;
      std::memcpy(out, L->sigma.data(), size_t(T) * 4);
      return CLOAK_OK;
    case CLOAK_QUERY_PI: {
      const FfnPerm* f = L->ffn_of_layer(int32_t(index));
      if (!f) {
        set_error("cloak_query: layer %lld has no FFN tensors", (long long)index);
        return CLOAK_EINVAL;
      }
      if (!need(uint64_t(f->d_ffn) * 4)) return CLOAK_EINVAL;
      std::memcpy(out, L->perms[size_t(f->table)].p.data(), size_t(f->d_ffn) * 4);
      return CLOAK_OK;
    }
    case CLOAK_QUERY_MAP_KEY: {
      if (!need(8)) return CLOAK_EINVAL;
      std::memcpy(out, &L->dev.phi_key, 8);
      return CLOAK_OK;
    }
    case CLOAK_QUERY_SHAPE: {
      if (index < 0 || index >= T) {
        set_error("cloak_query: tensor %lld out of range", (long long)index);
        return CLOAK_EINVAL;
      }
      if (!need(32)) return CLOAK_EINVAL;
      const cloak_shape& sh = L->tensors[size_t(index)].shape;
      const int64_t v[4] = {sh.n_out, sh.k_in, sh.dtype, sh.head_dim};
      std::memcpy(out, v, 32);
      return CLOAK_OK;
    }
    case CLOAK_QUERY_ROW_PERM:
    case CLOAK_QUERY_COL_PERM: {
      if (index < 0 || index >= T) {
        set_error("cloak_query: tensor %lld out of range", (long long)index);
        return CLOAK_EINVAL;
      }
      const bool rows = what == CLOAK_QUERY_ROW_PERM;
      const TensorInfo& ti = L->tensors[size_t(index)];
      const int64_t n = rows ? ti.shape.n_out : ti.shape.k_in;
      if (!need(uint64_t(n) * 4)) return CLOAK_EINVAL;
      const int32_t i = rows ? ti.row_perm : ti.col_perm;
      int32_t* o = static_cast<int32_t*>(out);
      for (int64_t j = 0; j < n; ++j) o[j] = i >= 0 ? L->perms[size_t(i)].p[size_t(j)] : int32_t(j);
      return CLOAK_OK;
    }
    case CLOAK_QUERY_VBASE:
    case CLOAK_QUERY_NPAGES: {
      if (!need(uint64_t(T) * 8)) return CLOAK_EINVAL;
      int64_t* o = static_cast<int64_t*>(out);
      for (int64_t t = 0; t < T; ++t) o[t] = what == CLOAK_QUERY_VBASE ? L->tensors[t].vbase : L->tensors[t].npages;
      return CLOAK_OK;
    }
    case CLOAK_QUERY_CONTIGUITY: {
      if (!need(8)) return CLOAK_EINVAL;
      double c = contiguity(L);
      std::memcpy(out, &c, 8);
      return CLOAK_OK;
    }
    case CLOAK_QUERY_UPLOAD_ORDER: {
      if (index < 0 || index >= T) {
        set_error("cloak_query: tensor %lld out of range", (long long)index);
        return CLOAK_EINVAL;
      }
      auto ord = upload_order(L, int32_t(index));
      if (!need(uint64_t(ord.size()) * 4)) return CLOAK_EINVAL;
      std::memcpy(out, ord.data(), ord.size() * 4);
      return CLOAK_OK;
    }
    case CLOAK_QUERY_DFFN: {
      if (!need(8)) return CLOAK_EINVAL;
      const FfnPerm* f = L->ffn_of_layer(int32_t(index));
      int64_t v = f ? f->d_ffn : 0;
      std::memcpy(out, &v, 8);
      return CLOAK_OK;
    }
    case CLOAK_QUERY_TENSOR: {
      if (!need(8)) return CLOAK_EINVAL;
      int64_t v = L->find_tensor(int32_t(index >> 8), int32_t(index & 255));
      std::memcpy(out, &v, 8);
      return CLOAK_OK;
    }
    default:
      set_error("cloak_query: unknown selector %d", what);
      return CLOAK_EINVAL;
  }
}

extern "C" int cloak_pack_host(const cloak_layout* L, int32_t tensor, const void* h_src, void* h_pool,
                               uint64_t h_pool_bytes) {
  clear_error();
  if (!L || !h_src || !h_pool) {
    set_error("cloak_pack_host: null argument");
    return CLOAK_EINVAL;
  }
  if (tensor < 0 || tensor >= int32_t(L->tensors.size())) {
    set_error("cloak_pack_host: tensor %d out of range", tensor);
    return CLOAK_EINVAL;
  }
  if (h_pool_bytes < uint64_t(L->pool_bytes)) {
    set_error("cloak_pack_host: pool image of %llu bytes, layout needs %lld", (unsigned long long)h_pool_bytes,
              (long long)L->pool_bytes);
    return CLOAK_EINVAL;
  }
  const TensorInfo& ti = L->tensors[tensor];
  auto* pool = static_cast<uint8_t*>(h_pool);
  for (int64_t i = 0; i < ti.npages; ++i) {
    stream_page(L, tensor, static_cast<const uint8_t*>(h_src), i, pool + int64_t(L->phi[ti.vbase + i]) * L->page_bytes);
  }
  return CLOAK_OK;
}

namespace cloak {

int decoy_dtype(const cloak_layout* L) {
  int64_t total[3] = {0, 0, 0};  // indexed by cloak_dtype
  for (const auto& ti : L->tensors) total[ti.shape.dtype] += ti.bytes;
  if (total[0] + total[1] + total[2] == 0) return CLOAK_BF16;
  int best = CLOAK_FP8_E4M3;  // ties: fp8, then bf16, then f32
  for (int d : {CLOAK_BF16, CLOAK_F32})
    if (total[d] > total[best]) best = d;
  return best;
}

namespace {

// Nearest-even bf16 of a finite binary32 value.
uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return uint16_t((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// OCP E4M3FN code of a finite binary32 value: nearest, ties to the even code,
// saturating at 448.  Magnitudes are compared against the code values
// directly: code c (c < 0x7F) has value (8 + c % 8) * 2^(c / 8 - 10) for
// c >= 8 and c * 2^-9 below.
uint8_t e4m3_rne(float f) {
  const double a = std::fabs(double(f));
  const uint8_t sign = std::signbit(f) ? 0x80 : 0;
  auto value = [](int c) { return c < 8 ? std::ldexp(double(c), -9) : std::ldexp(double(8 + c % 8), c / 8 - 10); };
  if (a >= 448.0) return sign | 0x7E;
  int lo = 0, hi = 0x7E;  // largest code with value <= a, by bisection
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (value(mid) <= a) lo = mid; else hi = mid - 1;
  }
  int code = lo;
  if (lo < 0x7E) {
    const double dl = a - value(lo), dh = value(lo + 1) - a;
    if (dh < dl || (dh == dl && ((lo + 1) % 2 == 0))) code = lo + 1;
  }
  return sign | uint8_t(code);
}

int32_t centred_sum(const SplitMix64& g0, int64_t e) {
  SplitMix64 g = g0;
  g.state += uint64_t(3 * e) * 0x9E3779B97F4A7C15ull;  // skip outputs 0 .. 3e-1
  uint32_t sum = 0;
  for (int w = 0; w < 3; ++w) {
    const uint64_t r = g.next();
    for (int i = 0; i < 4; ++i) sum += uint32_t((r >> (16 * i)) & 0xffffu);
  }
  return 2 * int32_t(sum) - 786420;
}

}  // namespace

void decoy_page(uint64_t decoy_seed, int64_t v, int64_t page_bytes, int dtype, uint8_t* dst) {
  const SplitMix64 g0 = substream(decoy_seed, kTagDecoy, uint32_t(v));
  const int elt = elt_bytes(dtype);
  const int64_t n = page_bytes / elt;
  for (int64_t e = 0; e < n; ++e) {
    const int32_t c = centred_sum(g0, e);
    if (dtype == CLOAK_FP8_E4M3) {
      dst[e] = e4m3_rne(std::ldexp(float(c * 3), -12));
    } else {
      const float f = std::ldexp(float(c * 5), -25);
      if (dtype == CLOAK_F32) {
        std::memcpy(dst + 4 * e, &f, 4);
      } else {
        const uint16_t h = bf16_rne(f);
        std::memcpy(dst + 2 * e, &h, 2);
      }
    }
  }
}

}  // namespace cloak

extern "C" int cloak_pool_decoy_host(const cloak_layout* L, void* h_pool, uint64_t h_pool_bytes,
                                     uint64_t decoy_seed) {
  clear_error();
  if (!L || !h_pool) {
    set_error("cloak_pool_decoy_host: null argument");
    return CLOAK_EINVAL;
  }
  if (h_pool_bytes < uint64_t(L->pool_bytes)) {
    set_error("cloak_pool_decoy_host: pool image of %llu bytes, layout needs %lld", (unsigned long long)h_pool_bytes,
              (long long)L->pool_bytes);
    return CLOAK_EINVAL;
  }
  const int dt = decoy_dtype(L);
  auto* pool = static_cast<uint8_t*>(h_pool);
  for (int64_t v = L->V; v < L->P; ++v)
    decoy_page(decoy_seed, v, L->page_bytes, dt, pool + int64_t(L->phi[v]) * L->page_bytes);
  return CLOAK_OK;
}

extern "C" int cloak_remap_begin(cloak_layout* L, uint64_t remap_seed) {
  clear_error();
  if (!L) {
    set_error("cloak_remap_begin: null layout");
    return CLOAK_EINVAL;
  }
  if (L->native()) {
    set_error("cloak_remap_begin: native (untranslated) layouts cannot be remapped");
    return CLOAK_ESTATE;
  }
  if (!remap_epoch_begin(L, remap_seed)) {
    set_error("cloak_remap_begin: a remap is in progress (finish it with cloak_remap_step)");
    return CLOAK_ESTATE;
  }
  return CLOAK_OK;
}

namespace {
// Swap pairs [e.next, e.next + n) of the active epoch in a host pool image.
void swap_pairs_host(cloak_layout* L, uint8_t* pool, int64_t n) {
  const RemapEpoch& e = L->epoch;
  std::vector<uint8_t> tmp(size_t(L->page_bytes));
  for (int64_t i = e.next; i < e.next + n; ++i) {
    uint8_t* a = pool + int64_t(e.pairs[2 * i]) * L->page_bytes;
    uint8_t* b = pool + int64_t(e.pairs[2 * i + 1]) * L->page_bytes;
    std::memcpy(tmp.data(), a, size_t(L->page_bytes));
    std::memcpy(a, b, size_t(L->page_bytes));
    std::memcpy(b, tmp.data(), size_t(L->page_bytes));
  }
}
}  // namespace

extern "C" int cloak_remap_step_host(cloak_layout* L, void* h_pool, uint64_t h_pool_bytes, int64_t max_pairs,
                                     int64_t* remaining) {
  clear_error();
  if (!L || !h_pool) {
    set_error("cloak_remap_step_host: null argument");
    return CLOAK_EINVAL;
  }
  if (!L->epoch.active) {
    set_error("cloak_remap_step_host: no remap in progress (cloak_remap_begin)");
    return CLOAK_ESTATE;
  }
  if (h_pool_bytes < uint64_t(L->pool_bytes)) {
    set_error("cloak_remap_step_host: pool image too small");
    return CLOAK_EINVAL;
  }
  RemapEpoch& e = L->epoch;
  const int64_t left = e.npairs() - e.next;
  // a bounded slice stops at the end of its pass; max_pairs <= 0 runs both
  const int64_t n = max_pairs <= 0 ? left : std::min(max_pairs, e.launchable());
  swap_pairs_host(L, static_cast<uint8_t*>(h_pool), n);
  remap_epoch_advance(L, n);
  if (remaining) *remaining = left - n;
  return CLOAK_OK;
}

extern "C" int cloak_remap_host(cloak_layout* L, void* h_pool, uint64_t h_pool_bytes, uint64_t remap_seed) {
  clear_error();
  if (!L || !h_pool) {
    set_error("cloak_remap_host: null argument");
    return CLOAK_EINVAL;
  }
  if (L->native()) {
    set_error("cloak_remap_host: native (untranslated) layouts cannot be remapped");
    return CLOAK_ESTATE;
  }
  if (h_pool_bytes < uint64_t(L->pool_bytes)) {
    set_error("cloak_remap_host: pool image too small");
    return CLOAK_EINVAL;
  }
  if (L->epoch.active) {
    set_error("cloak_remap_host: a remap is in progress (finish it with cloak_remap_step_host)");
    return CLOAK_ESTATE;
  }
  remap_epoch_begin(L, remap_seed);
  const int64_t n = L->epoch.npairs() - L->epoch.next;
  swap_pairs_host(L, static_cast<uint8_t*>(h_pool), n);
  remap_epoch_advance(L, n);
  return CLOAK_OK;
}

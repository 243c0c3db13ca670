// Kernels of the decoder step that the serving loop runs around the cloaked
// projections: embedding rows read through the page map, residual add +
// RMSNorm, rotary embedding with the write into the paged KV cache, causal
// GQA attention over the paged cache (BF16 MFMA, online softmax, context
// split across workgroups), the split combine and greedy argmax.
//
// KV cache of one layer: K and V each [num_blocks][n_kv][block_size][head_dim]
// bf16, so the keys of one head inside a block are contiguous.  The engine
// keeps it on the device and does not cloak it (the paper cloaks weights).

#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.hpp"

namespace cloak {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// ------------------------------------------------------------------ embedding
__global__ __launch_bounds__(256) void embed_kernel(const EmbedArgs a) {
  const int t = blockIdx.x;
  int id = a.ids[t];
  id = id < 0 ? 0 : (id >= a.vocab ? a.vocab - 1 : id);   // ids are validated on the host
  const int64_t page_mask = (int64_t(1) << a.log2_page) - 1;
  uint8_t* out = reinterpret_cast<uint8_t*>(a.out) + int64_t(t) * a.row_bytes;
  for (int p = threadIdx.x; p < a.row_bytes / 16; p += blockDim.x) {
    const int64_t o = int64_t(id) * a.row_bytes + int64_t(p) * 16;
    const int64_t v = a.vbase + (o >> a.log2_page);
    const int64_t phys = a.translate ? int64_t(uint32_t(a.phi[v]) ^ phi_mask(a.phi_key, v)) : v;
    const u32x4 w = *reinterpret_cast<const u32x4*>(a.pool + (phys << a.log2_page) + (o & page_mask));
    *reinterpret_cast<u32x4*>(out + int64_t(p) * 16) = w;
  }
}

// ------------------------------------------------------------------ RMSNorm
// row i of the output uses source row rows[i] (or i): r = x + add, rounded
// to bf16 (and stored to r_out when given); h = r / sqrt(mean(r^2) + eps) * g.
// Rows of D % 8 == 0 and D <= 8 * 256 * kNormChunks: each thread keeps its
// 16-byte chunks of the row in registers (one read of x and add).
constexpr int kNormChunks = 4;

__device__ inline float block_sum256(float v, float* red) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float tot = 0.f;
  for (int w = 0; w < int(blockDim.x >> 6); ++w) tot += red[w];
  return tot;
}

__global__ __launch_bounds__(256) void rmsnorm_vec_kernel(const NormArgs a) {
  const int i = blockIdx.x;
  const int src = a.rows ? a.rows[i] : i;
  const int nch = a.D / 8;
  const u32x4* x = reinterpret_cast<const u32x4*>(a.x + int64_t(src) * a.D);
  const u32x4* add = a.add ? reinterpret_cast<const u32x4*>(a.add + int64_t(src) * a.D) : nullptr;
  __shared__ float red[8];
  float r[kNormChunks][8];
  float ss = 0.f;
#pragma unroll
  for (int j = 0; j < kNormChunks; ++j) {
    const int c = threadIdx.x + j * 256;
    if (c >= nch) break;
    const u32x4 xv = x[c];
    u32x4 av = {0u, 0u, 0u, 0u};
    if (add) av = add[c];
    const uint32_t xw[4] = {xv.x, xv.y, xv.z, xv.w}, aw[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float v = bf2f(uint16_t(xw[e / 2] >> (16 * (e & 1))));
      if (add) v = bf2f(f2bf(v + bf2f(uint16_t(aw[e / 2] >> (16 * (e & 1))))));
      r[j][e] = v;
      ss += v * v;
    }
  }
  const float inv = rsqrtf(block_sum256(ss, red) / float(a.D) + a.eps);
  u32x4* r_out = a.r_out ? reinterpret_cast<u32x4*>(a.r_out + int64_t(src) * a.D) : nullptr;
  u32x4* h = reinterpret_cast<u32x4*>(a.h + int64_t(i) * a.D);
  const u32x4* gain = a.gain ? reinterpret_cast<const u32x4*>(a.gain) : nullptr;
#pragma unroll
  for (int j = 0; j < kNormChunks; ++j) {
    const int c = threadIdx.x + j * 256;
    if (c >= nch) break;
    u32x4 gv = {0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u};   // bf16 ones
    if (gain) gv = gain[c];
    const uint32_t gw[4] = {gv.x, gv.y, gv.z, gv.w};
    uint32_t ho[4], ro[4];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      const float g0 = bf2f(uint16_t(gw[e / 2])), g1 = bf2f(uint16_t(gw[e / 2] >> 16));
      ho[e / 2] = uint32_t(f2bf(r[j][e] * inv * g0)) | (uint32_t(f2bf(r[j][e + 1] * inv * g1)) << 16);
      ro[e / 2] = uint32_t(f2bf(r[j][e])) | (uint32_t(f2bf(r[j][e + 1])) << 16);
    }
    h[c] = u32x4{ho[0], ho[1], ho[2], ho[3]};
    if (r_out) r_out[c] = u32x4{ro[0], ro[1], ro[2], ro[3]};
  }
}

__global__ __launch_bounds__(256) void rmsnorm_kernel(const NormArgs a) {
  const int i = blockIdx.x;
  const int src = a.rows ? a.rows[i] : i;
  const uint16_t* x = a.x + int64_t(src) * a.D;
  const uint16_t* add = a.add ? a.add + int64_t(src) * a.D : nullptr;
  __shared__ float red[8];
  float ss = 0.f;
  for (int d = threadIdx.x; d < a.D; d += blockDim.x) {
    float r = bf2f(x[d]);
    if (add) r = bf2f(f2bf(r + bf2f(add[d])));
    ss += r * r;
  }
  for (int off = 32; off >= 1; off >>= 1) ss += __shfl_xor(ss, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
  __syncthreads();
  float tot = 0.f;
  for (int w = 0; w < int(blockDim.x >> 6); ++w) tot += red[w];
  const float inv = rsqrtf(tot / float(a.D) + a.eps);
  uint16_t* r_out = a.r_out ? a.r_out + int64_t(src) * a.D : nullptr;
  uint16_t* h = a.h + int64_t(i) * a.D;
  for (int d = threadIdx.x; d < a.D; d += blockDim.x) {
    float r = bf2f(x[d]);
    if (add) r = bf2f(f2bf(r + bf2f(add[d])));
    if (r_out) r_out[d] = f2bf(r);
    const float g = a.gain ? bf2f(a.gain[d]) : 1.f;
    h[d] = f2bf(r * inv * g);
  }
}

// ------------------------------------------------------------------ RoPE + KV write
// Rotate-half convention: pair (i, i + d/2) turns by pos * theta^(-2i/d).
// Angles are formed in double so long positions keep their accuracy.
constexpr int kMaxHalf = 64;   // head_dim 128
__global__ __launch_bounds__(256) void rope_kv_kernel(const RopeArgs a) {
  const int t = blockIdx.x;
  const int pos = a.positions[t];
  const int seq = a.tok_seq[t];
  const int half = a.hd / 2;
  // table entries are produced by the engine; clamp so a bad entry cannot
  // address memory outside this layer's cache
  const int bidx = min(pos / a.bs, a.max_blocks - 1);
  const int block = int(min(max(int64_t(a.block_table[int64_t(seq) * a.max_blocks + bidx]), int64_t(0)),
                            a.num_blocks - 1));
  const int off = pos % a.bs;
  uint16_t* row = a.qkv + int64_t(t) * a.ldqkv;
  // every head turns pair i by the same angle: half cosines and sines per token
  __shared__ float cs[2][kMaxHalf];
  for (int i = threadIdx.x; i < half; i += blockDim.x) {
    const double ang = double(pos) * pow(double(a.theta), -2.0 * double(i) / double(a.hd));
    cs[0][i] = float(cos(ang));
    cs[1][i] = float(sin(ang));
  }
  __syncthreads();
  // 8 pairs (16 bytes of each half) per item: rotations of q and k heads,
  // then 16-byte copies of the v heads into the cache
  const int per_head = half / 8;
  const int nrot = (a.n_heads + a.n_kv) * per_head, ncopy = a.n_kv * (a.hd / 8);
  for (int it = threadIdx.x; it < nrot + ncopy; it += blockDim.x) {
    if (it < nrot) {
      const int head = it / per_head, i0 = (it % per_head) * 8;
      const uint16_t* src = row + head * a.hd;
      const u32x4 lo = *reinterpret_cast<const u32x4*>(src + i0);
      const u32x4 hi = *reinterpret_cast<const u32x4*>(src + i0 + half);
      const uint32_t lw[4] = {lo.x, lo.y, lo.z, lo.w}, hw[4] = {hi.x, hi.y, hi.z, hi.w};
      uint32_t y1[4], y2[4];
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        uint16_t r1[2], r2[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const float c = cs[0][i0 + e + u], sn = cs[1][i0 + e + u];
          const float x1 = bf2f(uint16_t(lw[e / 2] >> (16 * u))), x2 = bf2f(uint16_t(hw[e / 2] >> (16 * u)));
          r1[u] = f2bf(x1 * c - x2 * sn);
          r2[u] = f2bf(x2 * c + x1 * sn);
        }
        y1[e / 2] = uint32_t(r1[0]) | (uint32_t(r1[1]) << 16);
        y2[e / 2] = uint32_t(r2[0]) | (uint32_t(r2[1]) << 16);
      }
      uint16_t* dst = head < a.n_heads
                          ? row + head * a.hd
                          : a.kc + ((int64_t(block) * a.n_kv + (head - a.n_heads)) * a.bs + off) * a.hd;
      *reinterpret_cast<u32x4*>(dst + i0) = u32x4{y1[0], y1[1], y1[2], y1[3]};
      *reinterpret_cast<u32x4*>(dst + i0 + half) = u32x4{y2[0], y2[1], y2[2], y2[3]};
    } else {
      const int j = it - nrot;
      const int head = j / (a.hd / 8), i0 = (j % (a.hd / 8)) * 8;
      const uint16_t* src = row + (a.n_heads + a.n_kv + head) * a.hd;
      uint16_t* vd = a.vc + ((int64_t(block) * a.n_kv + head) * a.bs + off) * a.hd;
      *reinterpret_cast<u32x4*>(vd + i0) = *reinterpret_cast<const u32x4*>(src + i0);
    }
  }
}

// ------------------------------------------------------------------ attention
// One workgroup: a tile of up to 16 consecutive new tokens of one sequence,
// one KV head, one slice of the context.  Wave w serves query head
// kv*group + w.  Per 64-key block the keys go to LDS as K[key][dim] and the
// values transposed as Vt[dim][key]; scores are computed transposed,
// S^T = K . Q^T (A = keys, B = the wave's 16 query tokens), so every lane
// holds 16 scores of ONE token: the online-softmax row statistics need only
// two cross-lane steps, and P^T can be fed to the P.V product (O^T = V^T . P^T)
// straight from registers by choosing the MFMA k-slot -> key mapping to match
// the score layout.
constexpr int kHD = 128;
constexpr int kKB = 64;   // keys per block

__device__ inline int kswz(int key, int chunk) { return key * (kHD * 2) + ((chunk ^ (key & 15)) << 4); }
// V^T rows (one per dim): the 16-byte slot of a key chunk is XORed with the
// dim's low bits and with dim / 8, so that the 16 lanes of a staging write
// (dims 8c + e for c = 0..15) land on 8 different slots instead of one bank
__device__ inline int vswz(int dim, int chunk) {
  return dim * (kKB * 2) + ((chunk ^ (dim & 7) ^ ((dim >> 3) & 7)) << 4);
}

// One block per (tile, kv head, key slice), one wave per query head of the
// group.  The next 64 keys are fetched into registers while the current 64
// are multiplied out of LDS.
template <int GROUP>
__global__ __launch_bounds__(64 * GROUP) void attention_kernel(const AttnArgs a) {
  constexpr int NT = 64 * GROUP;
  constexpr int NPT = (kKB * 16 + NT - 1) / NT;   // 16-byte K (and V) chunks per thread
  __shared__ __attribute__((aligned(16))) uint8_t kl[kKB * kHD * 2];
  __shared__ __attribute__((aligned(16))) uint8_t vl[kKB * kHD * 2];
  constexpr int group = GROUP;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;

  int b = blockIdx.x;
  const int sp = b % a.n_splits;
  b /= a.n_splits;
  const int kvh = b % a.n_kv;
  const int tile = a.tile0 + b / a.n_kv;
  const int seq = a.tile_seq[tile];
  const int tok0 = a.tile_tok0[tile];
  const int ntok = a.tile_ntok[tile];
  const int p0 = a.positions[tok0];
  const int maxpos = a.positions[tok0 + ntok - 1];
  const int k_lo = sp * a.split_keys;
  // slices past the tile's last position hold no key; the combine stops
  // before them
  if (k_lo > maxpos) return;
  int k_hi = k_lo + a.split_keys;
  if (k_hi > maxpos + 1) k_hi = maxpos + 1;
  const int qh = kvh * group + w;

  // the wave's query fragments (B operand of S^T = K Q^T): token col, dims s*32 + 8g
  bf16x8_t qf[4];
  {
    const bool ok = col < ntok;
    const uint16_t* qrow = a.q + int64_t(tok0 + (ok ? col : 0)) * a.ldq + qh * kHD;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      u32x4 v = ok ? *reinterpret_cast<const u32x4*>(qrow + s * 32 + g * 8) : u32x4{0u, 0u, 0u, 0u};
      qf[s] = __builtin_bit_cast(bf16x8_t, v);
    }
  }
  f32x4 o[8];
#pragma unroll
  for (int d = 0; d < 8; ++d) o[d] = f32x4{0.f, 0.f, 0.f, 0.f};
  float m_run = -INFINITY, l_run = 0.f;
  const int my_pos = p0 + col;
  const bool col_ok = col < ntok;

  // K and V chunks of keys kb0 .. kb0+63 (zeros past the slice)
  u32x4 kr[NPT], vr[NPT];
  auto fetch = [&](int kb0) {
#pragma unroll
    for (int n = 0; n < NPT; ++n) {
      const int i = int(threadIdx.x) + n * NT;
      const int key = i >> 4, ch = i & 15;
      const int kp = kb0 + key;
      kr[n] = u32x4{0u, 0u, 0u, 0u};
      vr[n] = u32x4{0u, 0u, 0u, 0u};
      if (i < kKB * 16 && kp < k_hi) {
        const int bidx = min(kp / a.bs, a.max_blocks - 1);
        const int blk = int(min(max(int64_t(a.block_table[int64_t(seq) * a.max_blocks + bidx]), int64_t(0)),
                                a.num_blocks - 1));
        const int64_t off = ((int64_t(blk) * a.n_kv + kvh) * a.bs + kp % a.bs) * kHD + ch * 8;
        kr[n] = *reinterpret_cast<const u32x4*>(a.kc + off);
        vr[n] = *reinterpret_cast<const u32x4*>(a.vc + off);
      }
    }
  };
  if (k_lo < k_hi) fetch(k_lo);

  for (int kb0 = k_lo; kb0 < k_hi; kb0 += kKB) {
    // stage K and V^T of this block
#pragma unroll
    for (int n = 0; n < NPT; ++n) {
      const int i = int(threadIdx.x) + n * NT;
      if (i >= kKB * 16) break;
      const int key = i >> 4, ch = i & 15;
      *reinterpret_cast<u32x4*>(kl + kswz(key, ch)) = kr[n];
      const uint16_t* ve = reinterpret_cast<const uint16_t*>(&vr[n]);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int dim = ch * 8 + e;
        *reinterpret_cast<uint16_t*>(vl + vswz(dim, key >> 3) + (key & 7) * 2) = ve[e];
      }
    }
    __syncthreads();
    if (kb0 + kKB < k_hi) fetch(kb0 + kKB);

    // S^T blocks: lane holds keys kb0 + 16*j + 4g + r of token col
    f32x4 st[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      st[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bf16x8_t kf = *reinterpret_cast<const bf16x8_t*>(kl + kswz(j * 16 + col, s * 4 + g));
        st[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kf, qf[s], st[j], 0, 0, 0);
      }
    }
    float bmax = -INFINITY;
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int kp = kb0 + 16 * j + 4 * g + r;
        const bool keep = col_ok && kp < k_hi && kp <= my_pos;
        st[j][r] = keep ? st[j][r] * a.scale : -INFINITY;
        bmax = fmaxf(bmax, st[j][r]);
      }
    bmax = fmaxf(bmax, __shfl_xor(bmax, 16));
    bmax = fmaxf(bmax, __shfl_xor(bmax, 32));
    const float m_new = fmaxf(m_run, bmax);
    const float alpha = (m_run == -INFINITY) ? (m_new == -INFINITY ? 1.f : 0.f) : __expf(m_run - m_new);
    float psum = 0.f;
    uint16_t pb[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float p = st[j][r] == -INFINITY ? 0.f : __expf(st[j][r] - m_new);
        psum += p;
        pb[j][r] = f2bf(p);
      }
    psum += __shfl_xor(psum, 16);
    psum += __shfl_xor(psum, 32);
    l_run = l_run * alpha + psum;
    m_run = m_new;
#pragma unroll
    for (int d = 0; d < 8; ++d) o[d] *= alpha;

    // O^T += V^T . P^T over two 32-key steps; k-slot 8g+e <-> key
    // 32h + 4g + e (e < 4) or 32h + 16 + 4g + (e - 4)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      u32x4 pv;
      pv.x = uint32_t(pb[2 * h][0]) | (uint32_t(pb[2 * h][1]) << 16);
      pv.y = uint32_t(pb[2 * h][2]) | (uint32_t(pb[2 * h][3]) << 16);
      pv.z = uint32_t(pb[2 * h + 1][0]) | (uint32_t(pb[2 * h + 1][1]) << 16);
      pv.w = uint32_t(pb[2 * h + 1][2]) | (uint32_t(pb[2 * h + 1][3]) << 16);
      const bf16x8_t pf = __builtin_bit_cast(bf16x8_t, pv);
      const int c0 = (32 * h + 4 * g) >> 3, c1 = (32 * h + 16 + 4 * g) >> 3;
      const int within = (g & 1) * 8;
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const int dim = d * 16 + col;
        const uint2 lo = *reinterpret_cast<const uint2*>(vl + vswz(dim, c0) + within);
        const uint2 hi = *reinterpret_cast<const uint2*>(vl + vswz(dim, c1) + within);
        const u32x4 vv = {lo.x, lo.y, hi.x, hi.y};
        o[d] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, vv), pf, o[d], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // partial result of this slice: O^T lane holds dims 16d + 4g + r of token col
  if (col_ok) {
    const int64_t slot = ((int64_t(tile) * a.n_kv + kvh) * a.n_splits + sp) * group + w;
    float* po = a.part_o + (slot * 16 + col) * kHD;
#pragma unroll
    for (int d = 0; d < 8; ++d) *reinterpret_cast<f32x4*>(po + d * 16 + 4 * g) = o[d];
    if (g == 0) {
      a.part_ml[(slot * 16 + col) * 2] = m_run;
      a.part_ml[(slot * 16 + col) * 2 + 1] = l_run;
    }
  }
}

// ------------------------------------------------------------------ single-token attention
// A decode token has one query row per head, too few to fill a matrix-core
// tile, so the GROUP query heads that share a KV head share one:
// S^T = K Q^T runs on MFMA with those heads as columns and K read straight
// from the cache in the operand layout (key c, dims 32s + 8g).  P.V runs on
// the vector ALUs as packed bf16 dot products over pairs of keys.  Each
// 16-lane row g of a wave keeps its own online-softmax state over keys
// 4g..4g+3 of every 16-key run; rows and waves merge through LDS at the end.
// One block of four waves per (tile, KV head, key slice); wave w takes the
// runs w, w + 4, ... of the slice.  A run lies in one KV block: block_size
// and split_keys are multiples of 16 (checked by the launcher).
template <int H, int GROUP>
__device__ inline void pv_heads(float (&o)[GROUP][8], float alpha, uint32_t p01, uint32_t p23,
                                const uint32_t (&v01)[8], const uint32_t (&v23)[8]) {
  if constexpr (H < GROUP) {
    // lane H of the row holds head H's alpha and packed probabilities
    const float al = __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, alpha), 0x150 + H,
                                                                        0xF, 0xF, false));
    const bf16x2_t q01 = __builtin_bit_cast(bf16x2_t, __builtin_amdgcn_mov_dpp(int(p01), 0x150 + H, 0xF, 0xF, false));
    const bf16x2_t q23 = __builtin_bit_cast(bf16x2_t, __builtin_amdgcn_mov_dpp(int(p23), 0x150 + H, 0xF, 0xF, false));
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float t = __builtin_amdgcn_fdot2_f32_bf16(q01, __builtin_bit_cast(bf16x2_t, v01[e]), o[H][e] * al, false);
      o[H][e] = __builtin_amdgcn_fdot2_f32_bf16(q23, __builtin_bit_cast(bf16x2_t, v23[e]), t, false);
    }
    pv_heads<H + 1, GROUP>(o, alpha, p01, p23, v01, v23);
  }
}

__device__ inline uint32_t pack_bf16x2(float lo, float hi) {
  return uint32_t(__builtin_bit_cast(uint16_t, __bf16(lo))) | (uint32_t(__builtin_bit_cast(uint16_t, __bf16(hi))) << 16);
}

template <int GROUP>
__global__ __launch_bounds__(256) void attention_single_kernel(const AttnArgs a) {
  __shared__ __attribute__((aligned(16))) float so[4][4][GROUP][kHD];   // wave, row, head: unnormalised o
  __shared__ float sml[4][4][GROUP][2];                                   // wave, row, head: m, l
  int b = blockIdx.x;
  const int sp = b % a.n_splits;
  b /= a.n_splits;
  const int kvh = b % a.n_kv;
  const int tile = b / a.n_kv;
  const int seq = a.tile_seq[tile], tok0 = a.tile_tok0[tile], ntok = a.tile_ntok[tile];
  const int k_lo = sp * a.split_keys;
  if (k_lo > a.positions[tok0 + ntok - 1]) return;
  // wave-uniform, so that the block-table lookups are scalar loads
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  const int32_t* table = a.block_table + int64_t(seq) * a.max_blocks;
  const int64_t blk_elems = int64_t(a.n_kv) * a.bs * kHD;

  for (int tcol = 0; tcol < ntok; ++tcol) {
    const int tok = tok0 + tcol;
    const int hi = min(k_lo + a.split_keys, a.positions[tok] + 1);   // keys [k_lo, hi)
    bf16x8_t qf[4];   // column c = query head kvh*GROUP + c, dims 32s + 8g
    {
      const bool ok = c < GROUP;
      const uint16_t* qrow = a.q + int64_t(tok) * a.ldq + (kvh * GROUP + (ok ? c : 0)) * kHD;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const u32x4 v = ok ? *reinterpret_cast<const u32x4*>(qrow + s * 32 + g * 8) : u32x4{0u, 0u, 0u, 0u};
        qf[s] = __builtin_bit_cast(bf16x8_t, v);
      }
    }
    // K of a run in the operand layout; V rows 4g + j, dims 8c .. 8c+7
    auto fetch = [&](int run, u32x4 (&kq)[4], u32x4 (&vq)[4]) {
      const int kp0 = k_lo + 16 * run;
      const int bidx = __builtin_amdgcn_readfirstlane(min(kp0 / a.bs, a.max_blocks - 1));
      // the block table is read through the constant address space: a
      // scalar load, which leaves the vector loads of the run in flight
      const int32_t e = ((const int32_t __attribute__((address_space(4)))*)table)[bidx];
      const int64_t blk = min(max(int64_t(e), int64_t(0)), a.num_blocks - 1);
      const int64_t base = blk * blk_elems + (int64_t(kvh) * a.bs + kp0 % a.bs) * kHD;
      const uint16_t* kb = a.kc + base;
      const uint16_t* vb = a.vc + base;
      // keys past hi read the run's first key instead (scores masked, p = 0),
      // so the loads need no branch and stay in flight together
      const int rk = kp0 + c < hi ? c : 0;
#pragma unroll
      for (int s = 0; s < 4; ++s) kq[s] = *reinterpret_cast<const u32x4*>(kb + rk * kHD + s * 32 + g * 8);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int rv = kp0 + 4 * g + j < hi ? 4 * g + j : 0;
        vq[j] = *reinterpret_cast<const u32x4*>(vb + rv * kHD + c * 8);
      }
    };
    float m = -INFINITY, l = 0.f;   // the row's state for head c
    float o[GROUP][8];
#pragma unroll
    for (int h = 0; h < GROUP; ++h)
#pragma unroll
      for (int e = 0; e < 8; ++e) o[h][e] = 0.f;
    // one 16-key run: scores on MFMA, online softmax per row, P.V on VALU
    auto step = [&](const u32x4 (&kq)[4], const u32x4 (&vq)[4], int run) {
      f32x4 st = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 4; ++s)
        st = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, kq[s]), qf[s], st, 0, 0, 0);
      // st[j]: key k_lo + 16 run + 4g + j, head c
      const int kp0 = k_lo + 16 * run;
      float bm = -INFINITY;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        st[j] = kp0 + 4 * g + j < hi ? st[j] * a.scale : -INFINITY;
        bm = fmaxf(bm, st[j]);
      }
      const float m_new = fmaxf(m, bm);
      const float alpha = m_new == -INFINITY ? 1.f : __expf(m - m_new);
      float p[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) p[j] = st[j] == -INFINITY ? 0.f : __expf(st[j] - m_new);
      l = l * alpha + ((p[0] + p[1]) + (p[2] + p[3]));
      m = m_new;
      const uint32_t p01 = pack_bf16x2(p[0], p[1]), p23 = pack_bf16x2(p[2], p[3]);
      // pairs of keys per dim: lo half key j, hi half key j + 1
      uint32_t v01[8], v23[8];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        v01[2 * d] = __builtin_amdgcn_perm(vq[1][d], vq[0][d], 0x05040100u);
        v01[2 * d + 1] = __builtin_amdgcn_perm(vq[1][d], vq[0][d], 0x07060302u);
        v23[2 * d] = __builtin_amdgcn_perm(vq[3][d], vq[2][d], 0x05040100u);
        v23[2 * d + 1] = __builtin_amdgcn_perm(vq[3][d], vq[2][d], 0x07060302u);
      }
      pv_heads<0, GROUP>(o, alpha, p01, p23, v01, v23);
    };
    // two register sets in turn: the next run's loads are in flight while
    // the current run is computed
    // (the last run fetches itself again rather than branch around a fetch,
    // which would make the first set wait for the second)
    u32x4 ka[4], va[4], kb[4], vb[4];
    int run = w;
    if (k_lo + 16 * run < hi) {
      fetch(run, ka, va);
      for (;;) {
        bool more = k_lo + 16 * (run + 4) < hi;
        fetch(more ? run + 4 : run, kb, vb);
        __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the math
        step(ka, va, run);
        if (!more) break;
        run += 4;
        more = k_lo + 16 * (run + 4) < hi;
        fetch(more ? run + 4 : run, ka, va);
        __builtin_amdgcn_sched_barrier(0);
        step(kb, vb, run);
        if (!more) break;
        run += 4;
      }
    }
    // merge the 16 row states of each head
    if (c < GROUP) {
      sml[w][g][c][0] = m;
      sml[w][g][c][1] = l;
    }
#pragma unroll
    for (int h = 0; h < GROUP; ++h) {
      *reinterpret_cast<f32x4*>(&so[w][g][h][8 * c]) = f32x4{o[h][0], o[h][1], o[h][2], o[h][3]};
      *reinterpret_cast<f32x4*>(&so[w][g][h][8 * c + 4]) = f32x4{o[h][4], o[h][5], o[h][6], o[h][7]};
    }
    __syncthreads();
    for (int h = w; h < GROUP; h += 4) {
      float M = -INFINITY;
#pragma unroll
      for (int i = 0; i < 16; ++i) M = fmaxf(M, sml[i >> 2][i & 3][h][0]);
      float L = 0.f, ax = 0.f, ay = 0.f;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const float mi = sml[i >> 2][i & 3][h][0];
        if (mi == -INFINITY) continue;
        const float e = __expf(mi - M);
        L += sml[i >> 2][i & 3][h][1] * e;
        const float2 v = *reinterpret_cast<const float2*>(&so[i >> 2][i & 3][h][2 * lane]);
        ax += v.x * e;
        ay += v.y * e;
      }
      const int64_t slot = ((int64_t(tile) * a.n_kv + kvh) * a.n_splits + sp) * GROUP + h;
      *reinterpret_cast<float2*>(a.part_o + (slot * 16 + tcol) * kHD + 2 * lane) = float2{ax, ay};
      if (lane == 0) {
        a.part_ml[(slot * 16 + tcol) * 2] = M;
        a.part_ml[(slot * 16 + tcol) * 2 + 1] = L;
      }
    }
    __syncthreads();
  }
}

// out[token][head*128 + d] from the partials of the slices that reach the
// tile: one wave per (tile, query head), two dims per lane
__global__ __launch_bounds__(256) void attn_combine_kernel(const AttnArgs a) {
  const int item = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * 4 + int(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (item >= a.n_tiles * a.n_heads) return;
  const int group = a.n_heads / a.n_kv;
  const int qh = item % a.n_heads, tile = item / a.n_heads;
  const int kvh = qh / group, w = qh % group;
  const int ntok = a.tile_ntok[tile], tok0 = a.tile_tok0[tile];
  // slices that start past the tile's last position were never written
  const int nsp = min(a.n_splits, a.positions[tok0 + ntok - 1] / a.split_keys + 1);
  const int64_t slot0 = (int64_t(tile) * a.n_kv + kvh) * a.n_splits * group + w;
  for (int tcol = 0; tcol < ntok; ++tcol) {
    auto ml = [&](int sp) { return a.part_ml + ((slot0 + int64_t(sp) * group) * 16 + tcol) * 2; };
    float M = -INFINITY;
    for (int sp = lane; sp < nsp; sp += 64) M = fmaxf(M, ml(sp)[0]);
    for (int off = 32; off >= 1; off >>= 1) M = fmaxf(M, __shfl_xor(M, off));
    // lane k holds the weight of slice base + k; the partial rows are then
    // read with no load waiting on another
    float L = 0.f, ax = 0.f, ay = 0.f;
    for (int base = 0; base < nsp; base += 64) {
      float e = 0.f;
      if (base + lane < nsp) {
        const float mi = ml(base + lane)[0];
        if (mi != -INFINITY) {
          e = __expf(mi - M);
          L += ml(base + lane)[1] * e;
        }
      }
      const int cnt = min(64, nsp - base);
      auto row = [&](int k) {
        return *reinterpret_cast<const float2*>(a.part_o + ((slot0 + int64_t(base + k) * group) * 16 + tcol) * kHD +
                                                2 * lane);
      };
      auto weight = [&](int k) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, e), k));
      };
      int k = 0;
      for (; k + 4 <= cnt; k += 4) {
        const float2 v0 = row(k), v1 = row(k + 1), v2 = row(k + 2), v3 = row(k + 3);
        const float e0 = weight(k), e1 = weight(k + 1), e2 = weight(k + 2), e3 = weight(k + 3);
        ax += v0.x * e0 + v1.x * e1 + v2.x * e2 + v3.x * e3;
        ay += v0.y * e0 + v1.y * e1 + v2.y * e2 + v3.y * e3;
      }
      for (; k < cnt; ++k) {
        const float2 v = row(k);
        const float ek = weight(k);
        ax += v.x * ek;
        ay += v.y * ek;
      }
    }
    for (int off = 32; off >= 1; off >>= 1) L += __shfl_xor(L, off);
    const float inv = L > 0.f ? 1.f / L : 0.f;
    const uint32_t pk = uint32_t(f2bf(ax * inv)) | (uint32_t(f2bf(ay * inv)) << 16);
    *reinterpret_cast<uint32_t*>(a.out + int64_t(tok0 + tcol) * a.ldo + qh * kHD + 2 * lane) = pk;
  }
}

// ------------------------------------------------------------------ argmax
// Greedy token: the largest logit of the row, the smallest index among equal
// ones.  Rows whose start is 16-byte aligned are read 8 logits per load.
constexpr int kArgmaxThreads = 1024;
__global__ __launch_bounds__(kArgmaxThreads) void argmax_kernel(const uint16_t* __restrict__ logits, int64_t V,
                                                                int32_t* __restrict__ out) {
  const uint16_t* row = logits + int64_t(blockIdx.x) * V;
  float best = -INFINITY;
  int64_t bi = 0;
  auto take = [&](float v, int64_t i) {
    if (v > best || (v == best && i < bi)) {
      best = v;
      bi = i;
    }
  };
  int64_t head = 0;
  if ((reinterpret_cast<uintptr_t>(row) & 15) == 0) {
    head = V / 8 * 8;
    const u32x4* r8 = reinterpret_cast<const u32x4*>(row);
    for (int64_t c = threadIdx.x; c < V / 8; c += blockDim.x) {
      const u32x4 w = r8[c];
      const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int e = 0; e < 8; ++e) take(bf2f(uint16_t(ww[e / 2] >> (16 * (e & 1)))), c * 8 + e);
    }
  }
  for (int64_t i = head + threadIdx.x; i < V; i += blockDim.x) take(bf2f(row[i]), i);
  __shared__ float sv[kArgmaxThreads];
  __shared__ int64_t si[kArgmaxThreads];
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) {
      const float ov = sv[threadIdx.x + s];
      const int64_t oi = si[threadIdx.x + s];
      if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
        sv[threadIdx.x] = ov;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = int32_t(si[0]);
}

}  // namespace

hipError_t launch_embed(const EmbedArgs& a, hipStream_t s) {
  if (a.T <= 0) return hipSuccess;
  hipLaunchKernelGGL(embed_kernel, dim3(a.T), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rmsnorm(const NormArgs& a, int rows, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const bool vec = a.D % 8 == 0 && a.D <= 8 * 256 * kNormChunks && reinterpret_cast<uintptr_t>(a.x) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(a.h) % 16 == 0 && (!a.add || reinterpret_cast<uintptr_t>(a.add) % 16 == 0) &&
                   (!a.r_out || reinterpret_cast<uintptr_t>(a.r_out) % 16 == 0) &&
                   (!a.gain || reinterpret_cast<uintptr_t>(a.gain) % 16 == 0);
  if (vec)
    hipLaunchKernelGGL(rmsnorm_vec_kernel, dim3(rows), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(rmsnorm_kernel, dim3(rows), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rope_kv(const RopeArgs& a, int T, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  // 16-byte items: half a head a multiple of 8 elements, rows 16-byte aligned
  if (a.hd / 2 > kMaxHalf || a.hd % 16 != 0 || a.ldqkv % 8 != 0 || reinterpret_cast<uintptr_t>(a.qkv) % 16 != 0 ||
      reinterpret_cast<uintptr_t>(a.kc) % 16 != 0 || reinterpret_cast<uintptr_t>(a.vc) % 16 != 0)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(rope_kv_kernel, dim3(T), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int G>
hipError_t launch_attention_g(const AttnArgs& a, int n_single, hipStream_t s) {
  if constexpr ((G & (G - 1)) != 0) n_single = 0;
  else if (n_single > 0) {
    const int64_t blocks = int64_t(n_single) * a.n_kv * a.n_splits;
    hipLaunchKernelGGL(attention_single_kernel<G>, dim3(unsigned(blocks)), dim3(256), 0, s, a);
    if (hipError_t e = hipGetLastError()) return e;
  }
  if (a.n_tiles > n_single) {
    AttnArgs m = a;
    m.tile0 = n_single;
    const int64_t blocks = int64_t(a.n_tiles - n_single) * a.n_kv * a.n_splits;
    hipLaunchKernelGGL(attention_kernel<G>, dim3(unsigned(blocks)), dim3(64 * G), 0, s, m);
    if (hipError_t e = hipGetLastError()) return e;
  }
  return hipSuccess;
}

hipError_t launch_attention(const AttnArgs& a, hipStream_t s) {
  if (a.n_tiles <= 0) return hipSuccess;
  const int group = a.n_heads / a.n_kv;
  // the single-token path takes group sizes 1, 2, 4 and 8, and 16-key runs
  // that stay inside one KV block
  const bool single_ok = (group & (group - 1)) == 0 && a.bs % 16 == 0 && a.split_keys % 16 == 0;
  const int n_single = single_ok ? min(max(a.n_single, 0), a.n_tiles) : 0;
  hipError_t e;
  switch (group) {
    case 1: e = launch_attention_g<1>(a, n_single, s); break;
    case 2: e = launch_attention_g<2>(a, n_single, s); break;
    case 3: e = launch_attention_g<3>(a, 0, s); break;
    case 4: e = launch_attention_g<4>(a, n_single, s); break;
    case 5: e = launch_attention_g<5>(a, 0, s); break;
    case 6: e = launch_attention_g<6>(a, 0, s); break;
    case 7: e = launch_attention_g<7>(a, 0, s); break;
    case 8: e = launch_attention_g<8>(a, n_single, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  const int64_t waves = int64_t(a.n_tiles) * a.n_heads;
  hipLaunchKernelGGL(attn_combine_kernel, dim3(unsigned((waves + 3) / 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_argmax(const uint16_t* logits, int64_t rows, int64_t V, int32_t* out, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(argmax_kernel, dim3(unsigned(rows)), dim3(kArgmaxThreads), 0, s, logits, V, out);
  return hipGetLastError();
}

}  // namespace cloak

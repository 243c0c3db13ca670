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
  const int nq = a.n_heads * half, nk = a.n_kv * half;
  for (int it = threadIdx.x; it < nq + 2 * nk; it += blockDim.x) {
    if (it < nq + nk) {
      const bool is_q = it < nq;
      const int j = is_q ? it : it - nq;
      const int head = j / half, i = j % half;
      const double ang = double(pos) * pow(double(a.theta), -2.0 * double(i) / double(a.hd));
      const float c = float(cos(ang)), s = float(sin(ang));
      uint16_t* base = row + (is_q ? head * a.hd : (a.n_heads + head) * a.hd);
      const float x1 = bf2f(base[i]), x2 = bf2f(base[i + half]);
      const uint16_t y1 = f2bf(x1 * c - x2 * s), y2 = f2bf(x2 * c + x1 * s);
      if (is_q) {
        base[i] = y1;
        base[i + half] = y2;
      } else {
        uint16_t* kd = a.kc + ((int64_t(block) * a.n_kv + head) * a.bs + off) * a.hd;
        kd[i] = y1;
        kd[i + half] = y2;
      }
    } else {
      const int j = it - nq - nk;   // v: plain copy, two elements per item
      const int head = j / half, i = j % half;
      const uint16_t* src = row + (a.n_heads + a.n_kv + head) * a.hd;
      uint16_t* vd = a.vc + ((int64_t(block) * a.n_kv + head) * a.bs + off) * a.hd;
      vd[2 * i] = src[2 * i];
      vd[2 * i + 1] = src[2 * i + 1];
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
__device__ inline int vswz(int dim, int chunk) { return dim * (kKB * 2) + ((chunk ^ (dim & 7)) << 4); }

__global__ __launch_bounds__(512) void attention_kernel(const AttnArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t kl[kKB * kHD * 2];
  __shared__ __attribute__((aligned(16))) uint8_t vl[kKB * kHD * 2];
  const int nthreads = blockDim.x;
  const int group = nthreads >> 6;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;

  int b = blockIdx.x;
  const int sp = b % a.n_splits;
  b /= a.n_splits;
  const int kvh = b % a.n_kv;
  const int tile = b / a.n_kv;
  const int seq = a.tile_seq[tile];
  const int tok0 = a.tile_tok0[tile];
  const int ntok = a.tile_ntok[tile];
  const int p0 = a.positions[tok0];
  const int maxpos = a.positions[tok0 + ntok - 1];
  const int k_lo = sp * a.split_keys;
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

  for (int kb0 = k_lo; kb0 < k_hi; kb0 += kKB) {
    // stage K and V^T of keys kb0 .. kb0+63 (zeros past the slice)
    for (int i = threadIdx.x; i < kKB * 16; i += nthreads) {
      const int key = i >> 4, ch = i & 15;
      const int kp = kb0 + key;
      u32x4 kv = {0u, 0u, 0u, 0u}, vv = {0u, 0u, 0u, 0u};
      if (kp < k_hi) {
        const int bidx = min(kp / a.bs, a.max_blocks - 1);
        const int blk = int(min(max(int64_t(a.block_table[int64_t(seq) * a.max_blocks + bidx]), int64_t(0)),
                                a.num_blocks - 1));
        const int64_t off = ((int64_t(blk) * a.n_kv + kvh) * a.bs + kp % a.bs) * kHD + ch * 8;
        kv = *reinterpret_cast<const u32x4*>(a.kc + off);
        vv = *reinterpret_cast<const u32x4*>(a.vc + off);
      }
      *reinterpret_cast<u32x4*>(kl + kswz(key, ch)) = kv;
      const uint16_t* ve = reinterpret_cast<const uint16_t*>(&vv);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int dim = ch * 8 + e;
        *reinterpret_cast<uint16_t*>(vl + vswz(dim, key >> 3) + (key & 7) * 2) = ve[e];
      }
    }
    __syncthreads();

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

// out[token][head*128 + d] from the context slices of its tile
__global__ __launch_bounds__(128) void attn_combine_kernel(const AttnArgs a) {
  const int group = a.n_heads / a.n_kv;
  int b = blockIdx.x;
  const int tcol = b % 16;
  b /= 16;
  const int qh = b % a.n_heads;
  const int tile = b / a.n_heads;
  if (tcol >= a.tile_ntok[tile]) return;
  const int kvh = qh / group, w = qh % group;
  const int d = threadIdx.x;
  float M = -INFINITY;
  for (int sp = 0; sp < a.n_splits; ++sp) {
    const int64_t slot = ((int64_t(tile) * a.n_kv + kvh) * a.n_splits + sp) * group + w;
    M = fmaxf(M, a.part_ml[(slot * 16 + tcol) * 2]);
  }
  float L = 0.f, acc = 0.f;
  for (int sp = 0; sp < a.n_splits; ++sp) {
    const int64_t slot = ((int64_t(tile) * a.n_kv + kvh) * a.n_splits + sp) * group + w;
    const float m = a.part_ml[(slot * 16 + tcol) * 2];
    if (m == -INFINITY) continue;
    const float e = __expf(m - M);
    L += a.part_ml[(slot * 16 + tcol) * 2 + 1] * e;
    acc += a.part_o[(slot * 16 + tcol) * kHD + d] * e;
  }
  const int tok = a.tile_tok0[tile] + tcol;
  a.out[int64_t(tok) * a.ldo + qh * kHD + d] = f2bf(L > 0.f ? acc / L : 0.f);
}

// ------------------------------------------------------------------ argmax
__global__ __launch_bounds__(256) void argmax_kernel(const uint16_t* __restrict__ logits, int64_t V,
                                                     int32_t* __restrict__ out) {
  const uint16_t* row = logits + int64_t(blockIdx.x) * V;
  float best = -INFINITY;
  int64_t bi = 0;
  for (int64_t i = threadIdx.x; i < V; i += blockDim.x) {
    const float v = bf2f(row[i]);
    if (v > best) {
      best = v;
      bi = i;
    }
  }
  __shared__ float sv[256];
  __shared__ int64_t si[256];
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
  hipLaunchKernelGGL(rmsnorm_kernel, dim3(rows), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rope_kv(const RopeArgs& a, int T, hipStream_t s) {
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(rope_kv_kernel, dim3(T), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_attention(const AttnArgs& a, hipStream_t s) {
  if (a.n_tiles <= 0) return hipSuccess;
  const int group = a.n_heads / a.n_kv;
  const int64_t blocks = int64_t(a.n_tiles) * a.n_kv * a.n_splits;
  hipLaunchKernelGGL(attention_kernel, dim3(unsigned(blocks)), dim3(64 * group), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(attn_combine_kernel, dim3(unsigned(int64_t(a.n_tiles) * a.n_heads * 16)), dim3(kHD), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_argmax(const uint16_t* logits, int64_t rows, int64_t V, int32_t* out, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(argmax_kernel, dim3(unsigned(rows)), dim3(256), 0, s, logits, V, out);
  return hipGetLastError();
}

}  // namespace cloak

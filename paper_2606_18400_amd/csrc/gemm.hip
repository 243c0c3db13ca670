// Prefill GEMM over cloaked weights: Y[M][N] = X[M][K] . W^T with W's rows
// read from page-scattered storage (CloakLM, arXiv 2606.18400, Section 4.2),
// BF16 MFMA (v_mfma_f32_16x16x32_bf16) with FP32 accumulation on gfx950.
//
// Tiling: a workgroup of 8 waves computes a 256 (tokens) x 256 (weight rows)
// tile, K in steps of 64.  Waves form a 2 x 4 grid; each owns 128 tokens x 64
// rows = 8 x 4 MFMA blocks of 16 x 16 (128 FP32 accumulators per lane).
// Both operands are K-contiguous, so each lane loads 16 B (8 bf16) pieces of
// rows of X and of W; tiles go global -> registers -> LDS (double buffered,
// 16-byte chunks XOR-swizzled by row so the MFMA fragment reads of 16
// consecutive rows spread over the banks) -> MFMA fragments.
//
// Page translation: every thread always loads the same 4 weight rows of the
// tile, so it keeps each row's current virtual page and its physical base in
// registers and reads the page map again only when the row's stream crosses
// into the next page (never for rows that fit in a page, e.g. 8 KiB rows in
// 2 MiB pages).  A 128-byte row segment never straddles a page: rows and
// page sizes are multiples of 128 B.
//
// Output: lane l of an MFMA block holds D[4*(l/16)+r][l%16], i.e. four
// consecutive weight rows (output columns) of one token, written as one 8 B
// store.  SwiGLU mode: the tile's 256 rows are 128 gate rows and the same 128
// up rows, and each wave's four row blocks are two gate blocks and the two
// matching up blocks, so silu(g)*u is formed in registers.

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace cloak {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 256, BN = 256, BK = 64;
constexpr int WAVES_M = 2, WAVES_N = 4;
constexpr int NTHREADS = 64 * WAVES_M * WAVES_N;
constexpr int WM = BM / WAVES_M;  // 128 tokens per wave
constexpr int WN = BN / WAVES_N;  // 64 weight rows per wave
constexpr int MB = WM / 16;       // 8 token blocks
constexpr int NB = WN / 16;       // 4 row blocks
constexpr int ROWB = BK * 2;      // 128 bytes per tile row in LDS
constexpr int TILE_BYTES = BM * ROWB;  // 32 KiB per operand tile
constexpr int LOADS = BM * (ROWB / 16) / NTHREADS;  // 16 B loads per thread per operand per K step (4)

__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// byte offset in a tile of (row, 16-byte chunk): chunks XOR-swizzled by row
__device__ inline int swz(int row, int chunk) { return row * ROWB + ((chunk ^ (row & 7)) << 4); }

struct RowRef {
  const uint8_t* pool;
  int64_t vbase;    // first virtual page of the row's tensor
  int64_t rowoff;   // byte offset of the row in the tensor's stream
  int64_t cvp;      // cached virtual page (relative to vbase), -1 = none
  int64_t cbase;    // physical byte offset of that page in the pool
  bool ok;
};

template <bool TR>
__device__ inline const uint8_t* row_addr(const int32_t* phi, int log2_page, RowRef& r, int64_t koff) {
  const int64_t o = r.rowoff + koff;
  const int64_t vp = o >> log2_page;
  if (vp != r.cvp) {
    r.cvp = vp;
    const int64_t v = r.vbase + vp;
    r.cbase = (TR ? int64_t(phi[v]) : v) << log2_page;
  }
  return r.pool + r.cbase + (o & ((int64_t(1) << log2_page) - 1));
}

template <int EPI>
__device__ inline bool tile_row(const GemmArgs& a, int tile_n, int tr, int& seg, int& n) {
  if (EPI == kSwiGLU) {
    seg = tr < BN / 2 ? 0 : 1;
    n = tile_n * (BN / 2) + (tr % (BN / 2));
    return n < a.seg[0].rows;
  }
  const int row = tile_n * BN + tr;
  seg = 0;
#pragma unroll
  for (int i = 1; i < 4; ++i)
    if (i < a.nseg && row >= a.seg[i].row0) seg = i;
  n = row - a.seg[seg].row0;
  return n < a.seg[seg].rows;
}

template <bool TR, int EPI>
__global__ __launch_bounds__(NTHREADS, 1) void gemm_kernel(const GemmArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  // buffer b: X tile at smem + 2b*TILE_BYTES, W tile right after it
  auto lds_x = [&](int buf) { return smem + buf * 2 * TILE_BYTES; };
  auto lds_w = [&](int buf) { return smem + buf * 2 * TILE_BYTES + TILE_BYTES; };

  // XCD-aware tile order: consecutive workgroup ids go to different XCDs, so
  // give each XCD a contiguous run of tiles; inside a run, tokens vary
  // fastest and the run's weight tiles stay in that XCD's L2.
  const int ntiles = a.tiles_m * a.tiles_n;
  const int b = blockIdx.x;
  const int per_xcd = (ntiles + 7) / 8;
  const int xcd = b % 8, slot = b / 8;
  const int t_id = xcd * per_xcd + slot;
  if (t_id >= ntiles) return;
  const int tile_m = t_id % a.tiles_m;
  const int tile_n = t_id / a.tiles_m;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;

  // this thread's load slots: rows (tid >> 3) + 64 i, 16 B chunk (tid & 7)
  const int ch = tid & 7;
  const uint16_t* xrow[LOADS];
  bool xok[LOADS];
  RowRef wr[LOADS];
#pragma unroll
  for (int i = 0; i < LOADS; ++i) {
    const int tr = (tid >> 3) + 64 * i;
    const int m = tile_m * BM + tr;
    xok[i] = m < a.M;
    xrow[i] = a.x + int64_t(xok[i] ? m : 0) * a.ldx + ch * 8;
    int seg, n;
    wr[i].ok = tile_row<EPI>(a, tile_n, tr, seg, n);
    wr[i].pool = a.pool;
    wr[i].vbase = a.seg[seg].vbase;
    wr[i].rowoff = int64_t(wr[i].ok ? n : 0) * a.row_bytes + ch * 16;
    wr[i].cvp = -1;
    wr[i].cbase = 0;
  }

  u32x4 gx[LOADS], gw[LOADS];
  auto gload = [&](int kb) {
    const int64_t koff = int64_t(kb) * ROWB;
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      gx[i] = xok[i] ? *reinterpret_cast<const u32x4*>(xrow[i] + kb * BK) : u32x4{0u, 0u, 0u, 0u};
      gw[i] = wr[i].ok ? __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(row_addr<TR>(a.phi, a.log2_page, wr[i], koff)))
                       : u32x4{0u, 0u, 0u, 0u};
    }
  };
  auto swrite = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      const int tr = (tid >> 3) + 64 * i;
      *reinterpret_cast<u32x4*>(lds_x(buf) + swz(tr, ch)) = gx[i];
      *reinterpret_cast<u32x4*>(lds_w(buf) + swz(tr, ch)) = gw[i];
    }
  };

  f32x4 acc[NB][MB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < MB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // tile rows of this wave's row blocks
  int wrow[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    if (EPI == kSwiGLU) {
      // two gate blocks, then the two up blocks of the same hidden units
      wrow[nb] = (nb < NB / 2 ? 0 : BN / 2) + wn * (WN / 2) + (nb % (NB / 2)) * 16;
    } else {
      wrow[nb] = wn * WN + nb * 16;
    }
  }

  const int nk = a.K / BK;
  gload(0);
  swrite(0);
  __syncthreads();
  for (int kb = 0; kb < nk; ++kb) {
    const int buf = kb & 1;
    if (kb + 1 < nk) gload(kb + 1);
#pragma unroll
    for (int s = 0; s < BK / 32; ++s) {
      const int chunk = s * 4 + (lane >> 4);
      bf16x8_t fa[NB], fb[MB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int r = wrow[nb] + (lane & 15);
        fa[nb] = *reinterpret_cast<const bf16x8_t*>(lds_w(buf) + swz(r, chunk));
      }
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int r = wm * WM + mb * 16 + (lane & 15);
        fb[mb] = *reinterpret_cast<const bf16x8_t*>(lds_x(buf) + swz(r, chunk));
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
          acc[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[nb], fb[mb], acc[nb][mb], 0, 0, 0);
    }
    if (kb + 1 < nk) swrite(buf ^ 1);
    __syncthreads();
  }

  // ---------------------------------------------------------------- epilogue
  const int r4 = 4 * (lane >> 4);
  const int tok = lane & 15;
  if constexpr (EPI == kStore) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int tr0 = wrow[nb] + r4;  // first of this lane's 4 tile rows
      int seg, n0;
      const bool ok0 = tile_row<EPI>(a, tile_n, tr0, seg, n0);
      if (!ok0) continue;
      const int rows = a.seg[seg].rows;
      const int32_t* perm = a.seg[seg].out_perm;
      const float* scale = a.seg[seg].scale;
      const int out_off = a.seg[seg].out_off;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int m = tile_m * BM + wm * WM + mb * 16 + tok;
        if (m >= a.M) continue;
        uint16_t* yrow = static_cast<uint16_t*>(a.y) + int64_t(m) * a.ldy + out_off;
        float v[4] = {acc[nb][mb][0], acc[nb][mb][1], acc[nb][mb][2], acc[nb][mb][3]};
        if (!perm && a.vec_store && n0 + 3 < rows) {
          uint32_t lo, hi;
          float s0 = scale ? scale[n0] : 1.f, s1 = scale ? scale[n0 + 1] : 1.f;
          float s2 = scale ? scale[n0 + 2] : 1.f, s3 = scale ? scale[n0 + 3] : 1.f;
          lo = uint32_t(f32_to_bf16_rne(v[0] * s0)) | (uint32_t(f32_to_bf16_rne(v[1] * s1)) << 16);
          hi = uint32_t(f32_to_bf16_rne(v[2] * s2)) | (uint32_t(f32_to_bf16_rne(v[3] * s3)) << 16);
          *reinterpret_cast<uint2*>(yrow + n0) = make_uint2(lo, hi);
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int n = n0 + r;
            if (n < rows) yrow[perm ? perm[n] : n] = f32_to_bf16_rne(v[r] * (scale ? scale[n] : 1.f));
          }
        }
      }
    }
  } else {
    const float* sg = a.seg[0].scale;
    const float* su = a.seg[1].scale;
    const int dff = a.seg[0].rows;
#pragma unroll
    for (int nb = 0; nb < NB / 2; ++nb) {
      const int j0 = tile_n * (BN / 2) + wn * (WN / 2) + nb * 16 + r4;
      if (j0 >= dff) continue;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const int m = tile_m * BM + wm * WM + mb * 16 + tok;
        if (m >= a.M) continue;
        uint16_t* hrow = static_cast<uint16_t*>(a.y) + int64_t(m) * a.ldy;
        uint16_t hv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = j0 + r;
          const int jj = j < dff ? j : dff - 1;
          const float g = acc[nb][mb][r] * (sg ? sg[jj] : 1.f);
          const float u = acc[nb + NB / 2][mb][r] * (su ? su[jj] : 1.f);
          hv[r] = f32_to_bf16_rne(g / (1.0f + expf(-g)) * u);
        }
        if (a.vec_store && j0 + 3 < dff) {
          *reinterpret_cast<uint2*>(hrow + j0) =
              make_uint2(uint32_t(hv[0]) | (uint32_t(hv[1]) << 16), uint32_t(hv[2]) | (uint32_t(hv[3]) << 16));
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (j0 + r < dff) hrow[j0 + r] = hv[r];
        }
      }
    }
  }
}

// x_out[m][j] = x[m][perm[j]]: the activations of a down projection put in
// the stored (hidden-permuted) column order before a prefill GEMM.
__global__ __launch_bounds__(256) void gather_cols_kernel(const uint16_t* __restrict__ x, int64_t ldx,
                                                          const int32_t* __restrict__ perm, uint16_t* __restrict__ out,
                                                          int64_t M, int64_t K) {
  const int64_t total = M * K;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int64_t m = i / K, j = i % K;
    out[i] = x[m * ldx + perm[j]];
  }
}

// ---------------------------------------------------------------------------
// Skinny split-K GEMM for decode batches (17..64 tokens).  A 256-row tile
// leaves a 4096-row projection only 16 workgroups; here a workgroup of 4
// waves takes 64 weight rows x 64 tokens x one K slice (SBK = 64 per step,
// 32 KiB of LDS, so several workgroups share a CU), and the K slices of a
// row tile are spread over workgroups.  Each slice writes FP32 partial sums
// part[slice][token][launch-row]; skinny_reduce_kernel adds the slices in a
// fixed order (deterministic) and applies the epilogue.  SwiGLU tiles hold
// 32 gate rows and the same 32 up rows.
constexpr int SBM = 64, SBN = 64, SBK = 64, STHREADS = 256;
constexpr int S_TILE = SBM * ROWB;                     // 8 KiB per operand tile
constexpr int S_LOADS = SBM * (ROWB / 16) / STHREADS;  // 2

template <int EPI>
__device__ inline bool skinny_row(const SkinnyArgs& a, int tile_n, int tr, int& seg, int& n) {
  if (EPI == kSwiGLU) {
    seg = tr < SBN / 2 ? 0 : 1;
    n = tile_n * (SBN / 2) + (tr % (SBN / 2));
    return n < a.seg[0].rows;
  }
  const int row = tile_n * SBN + tr;
  seg = 0;
#pragma unroll
  for (int i = 1; i < 4; ++i)
    if (i < a.nseg && row >= a.seg[i].row0) seg = i;
  n = row - a.seg[seg].row0;
  return n < a.seg[seg].rows;
}

template <bool TR, int EPI>
__global__ __launch_bounds__(STHREADS) void skinny_kernel(const SkinnyArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t smem[4 * S_TILE];
  auto lds_x = [&](int buf) { return smem + buf * 2 * S_TILE; };
  auto lds_w = [&](int buf) { return smem + buf * 2 * S_TILE + S_TILE; };
  const int ks = blockIdx.x % a.ksplit;
  const int tile_n = blockIdx.x / a.ksplit;
  const int kb_begin = ks * a.kblocks_per_split;
  int kb_end = kb_begin + a.kblocks_per_split;
  if (kb_end > a.K / SBK) kb_end = a.K / SBK;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int ch = tid & 7;

  const uint16_t* xrow[S_LOADS];
  bool xok[S_LOADS];
  RowRef wr[S_LOADS];
#pragma unroll
  for (int i = 0; i < S_LOADS; ++i) {
    const int tr = (tid >> 3) + 32 * i;
    xok[i] = tr < a.M;
    xrow[i] = a.x + int64_t(xok[i] ? tr : 0) * a.ldx + ch * 8;
    int seg, n;
    wr[i].ok = skinny_row<EPI>(a, tile_n, tr, seg, n);
    wr[i].pool = a.pool;
    wr[i].vbase = a.seg[seg].vbase;
    wr[i].rowoff = int64_t(wr[i].ok ? n : 0) * a.row_bytes + ch * 16;
    wr[i].cvp = -1;
    wr[i].cbase = 0;
  }
  u32x4 gx[S_LOADS], gw[S_LOADS];
  auto gload = [&](int kb) {
    const int64_t koff = int64_t(kb) * ROWB;
#pragma unroll
    for (int i = 0; i < S_LOADS; ++i) {
      gx[i] = xok[i] ? *reinterpret_cast<const u32x4*>(xrow[i] + kb * SBK) : u32x4{0u, 0u, 0u, 0u};
      gw[i] = wr[i].ok ? __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(row_addr<TR>(a.phi, a.log2_page, wr[i], koff)))
                       : u32x4{0u, 0u, 0u, 0u};
    }
  };
  auto swrite = [&](int buf) {
#pragma unroll
    for (int i = 0; i < S_LOADS; ++i) {
      const int tr = (tid >> 3) + 32 * i;
      *reinterpret_cast<u32x4*>(lds_x(buf) + swz(tr, ch)) = gx[i];
      *reinterpret_cast<u32x4*>(lds_w(buf) + swz(tr, ch)) = gw[i];
    }
  };
  f32x4 acc[SBM / 16];
#pragma unroll
  for (int j = 0; j < SBM / 16; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int wrow = wave * 16;
  if (kb_begin < kb_end) {
    gload(kb_begin);
    swrite(0);
  }
  __syncthreads();
  for (int kb = kb_begin; kb < kb_end; ++kb) {
    const int buf = (kb - kb_begin) & 1;
    if (kb + 1 < kb_end) gload(kb + 1);
#pragma unroll
    for (int s = 0; s < SBK / 32; ++s) {
      const int chunk = s * 4 + (lane >> 4);
      const bf16x8_t fa = *reinterpret_cast<const bf16x8_t*>(lds_w(buf) + swz(wrow + (lane & 15), chunk));
#pragma unroll
      for (int mb = 0; mb < SBM / 16; ++mb) {
        const bf16x8_t fb = *reinterpret_cast<const bf16x8_t*>(lds_x(buf) + swz(mb * 16 + (lane & 15), chunk));
        acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[mb], 0, 0, 0);
      }
    }
    if (kb + 1 < kb_end) swrite(buf ^ 1);
    __syncthreads();
  }
  // partial sums: lane holds launch-rows wrow + 4*(lane/16) + r of token mb*16 + lane%16
  const int row0 = tile_n * SBN + wrow + 4 * (lane >> 4);
#pragma unroll
  for (int mb = 0; mb < SBM / 16; ++mb) {
    const int m = mb * 16 + (lane & 15);
    if (m >= a.M) continue;
    float* dst = a.part + (int64_t(ks) * a.M + m) * a.ldp + row0;
    *reinterpret_cast<f32x4*>(dst) = acc[mb];
  }
}

// Sum of the K slices in slice order, then the epilogue.  STORE: one thread
// per (token, launch-row); SwiGLU: one thread per (token, hidden unit).
template <int EPI>
__global__ __launch_bounds__(256) void skinny_reduce_kernel(const SkinnyArgs a) {
  const int64_t per_tok = EPI == kSwiGLU ? int64_t(a.seg[0].rows) : int64_t(a.ldp);
  const int64_t total = int64_t(a.M) * per_tok;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total; i += int64_t(gridDim.x) * blockDim.x) {
    const int m = int(i / per_tok);
    const int c = int(i % per_tok);
    if constexpr (EPI == kSwiGLU) {
      const int tile = c / (SBN / 2), j = c % (SBN / 2);
      const int rg = tile * SBN + j, ru = rg + SBN / 2;
      float g = 0.f, u = 0.f;
      for (int ks = 0; ks < a.ksplit; ++ks) {
        const float* p = a.part + (int64_t(ks) * a.M + m) * a.ldp;
        g += p[rg];
        u += p[ru];
      }
      if (a.seg[0].scale) g *= a.seg[0].scale[c];
      if (a.seg[1].scale) u *= a.seg[1].scale[c];
      static_cast<uint16_t*>(a.y)[int64_t(m) * a.ldy + c] = f32_to_bf16_rne(g / (1.0f + expf(-g)) * u);
    } else {
      int seg = 0;
#pragma unroll
      for (int k = 1; k < 4; ++k)
        if (k < a.nseg && c >= a.seg[k].row0) seg = k;
      const int n = c - a.seg[seg].row0;
      if (n >= a.seg[seg].rows) continue;
      float v = 0.f;
      for (int ks = 0; ks < a.ksplit; ++ks) v += a.part[(int64_t(ks) * a.M + m) * a.ldp + c];
      if (a.seg[seg].scale) v *= a.seg[seg].scale[n];
      const int32_t* perm = a.seg[seg].out_perm;
      static_cast<uint16_t*>(a.y)[int64_t(m) * a.ldy + a.seg[seg].out_off + (perm ? perm[n] : n)] =
          f32_to_bf16_rne(v);
    }
  }
}

}  // namespace

int gemm_lds_bytes() { return 4 * TILE_BYTES; }
int gemm_tile_rows() { return BN; }
int gemm_k_step() { return BK; }

hipError_t launch_gemm(const GemmArgs& a, bool translate, hipStream_t s) {
  const int ntiles = a.tiles_m * a.tiles_n;
  if (ntiles <= 0) return hipSuccess;
  const int blocks = (ntiles + 7) / 8 * 8;
  const size_t lds = size_t(gemm_lds_bytes());
  void (*fn)(const GemmArgs);
  if (a.mode == kSwiGLU)
    fn = translate ? gemm_kernel<true, kSwiGLU> : gemm_kernel<false, kSwiGLU>;
  else
    fn = translate ? gemm_kernel<true, kStore> : gemm_kernel<false, kStore>;
  static bool attr_set[4] = {false, false, false, false};
  const int key = (translate ? 2 : 0) + (a.mode == kSwiGLU ? 1 : 0);
  if (!attr_set[key]) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       int(lds));
    if (e != hipSuccess) return e;
    attr_set[key] = true;
  }
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(NTHREADS), lds, s, a);
  return hipGetLastError();
}

int skinny_tile_rows() { return SBN; }

hipError_t launch_skinny(const SkinnyArgs& a, bool translate, hipStream_t s) {
  const int64_t blocks = int64_t(a.tiles_n) * a.ksplit;
  if (blocks <= 0 || a.M <= 0) return hipSuccess;
  if (a.M > SBM || a.K % SBK != 0) return hipErrorInvalidValue;
  void (*fn)(const SkinnyArgs);
  if (a.mode == kSwiGLU)
    fn = translate ? skinny_kernel<true, kSwiGLU> : skinny_kernel<false, kSwiGLU>;
  else
    fn = translate ? skinny_kernel<true, kStore> : skinny_kernel<false, kStore>;
  hipLaunchKernelGGL(fn, dim3(unsigned(blocks)), dim3(STHREADS), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t per_tok = a.mode == kSwiGLU ? int64_t(a.seg[0].rows) : int64_t(a.ldp);
  int64_t rb = (int64_t(a.M) * per_tok + 255) / 256;
  if (rb > 8192) rb = 8192;
  if (a.mode == kSwiGLU)
    hipLaunchKernelGGL(skinny_reduce_kernel<kSwiGLU>, dim3(unsigned(rb)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(skinny_reduce_kernel<kStore>, dim3(unsigned(rb)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gather_cols(const uint16_t* x, int64_t ldx, const int32_t* perm, uint16_t* out, int64_t M,
                              int64_t K, hipStream_t s) {
  const int64_t total = M * K;
  if (total <= 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(gather_cols_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, x, ldx, perm, out, M, K);
  return hipGetLastError();
}

}  // namespace cloak

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
// FP8 weights: with BF16 activations (the default) the weight bytes are
// widened exactly to BF16 as they enter LDS, so only HBM traffic changes.
// In the FP8 x FP8 mode (a8) the activations were quantised per token to
// E4M3 beforehand; a K step is then 128 elements (still 128 bytes per tile
// row) and one v_mfma_f32_16x16x128_f8f6f4 per block consumes 32 bytes per
// lane of each operand.  Both operands take the same two swizzled 16-byte
// chunks per lane, so they pair the same k on both sides whatever order the
// instruction uses inside its 128-wide K slice.  The epilogue multiplies by
// the token scale, then by the weight-row scale.
//
// Output: lane l of an MFMA block holds D[4*(l/16)+r][l%16], i.e. four
// consecutive weight rows (output columns) of one token, written as one 8 B
// store.  SwiGLU mode: the tile's 256 rows are 128 gate rows and the same 128
// up rows, and each wave's four row blocks are two gate blocks and the two
// matching up blocks, so silu(g)*u is formed in registers.

#include <hip/hip_runtime.h>

#include <type_traits>

#include <mutex>
#include <set>

#include "kernels.hpp"

namespace cloak {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef int i32x8 __attribute__((ext_vector_type(8)));
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

// f(integral_constant<int, I>) for I = B .. E-1, unrolled at compile time
template <int B, int E, typename F>
__device__ inline void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
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
__device__ inline const uint8_t* row_addr(const int32_t* phi, uint64_t key, int log2_page, RowRef& r,
                                          int64_t koff) {
  const int64_t o = r.rowoff + koff;
  const int64_t vp = o >> log2_page;
  if (vp != r.cvp) {
    r.cvp = vp;
    const int64_t v = r.vbase + vp;
    r.cbase = (TR ? int64_t(uint32_t(phi[v]) ^ phi_mask(key, v)) : v) << log2_page;
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

// Weight tile of ROWS rows x one K step (64 elements) for NT threads.  BF16
// rows give 128-byte segments (8 loads of 16 B); FP8 rows give 64-byte
// segments (4 loads of 16 B), widened exactly to BF16 with
// v_cvt_scalef32_pk_bf16_fp8 when they are written to LDS, so the MFMA path
// is the same for both while FP8 weights cross HBM at one byte each.  Each
// thread keeps its rows for the whole K loop (cached page translation).
// D register sets (slots) let a caller keep D K steps in flight.
template <int ROWS, int NT, bool F8, int D = 1>
struct WTile {
  static constexpr int PER_ROW = F8 ? 4 : 8;
  static constexpr int N = ROWS * PER_ROW / NT;
  static constexpr int STEP_BYTES = F8 ? 64 : 128;
  static_assert(NT % PER_ROW == 0, "thread count must cover whole rows");
  static constexpr int ROW_STRIDE = NT / PER_ROW;   // rows between a thread's slots
  RowRef r[N];
  int tr0, c;                                       // first row, 16 B chunk in the row
  u32x4 g[D][N];

  template <typename RowFn>
  __device__ inline void init(int tid, const uint8_t* pool, const WSeg* segs, int64_t row_bytes, RowFn row_of) {
    tr0 = tid / PER_ROW;
    c = tid % PER_ROW;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      int seg = 0, n = 0;
      r[i].ok = row_of(tr0 + ROW_STRIDE * i, seg, n);
      r[i].pool = pool;
      r[i].vbase = segs[seg].vbase;
      r[i].rowoff = int64_t(r[i].ok ? n : 0) * row_bytes + c * 16;
      r[i].cvp = -1;
      r[i].cbase = 0;
    }
  }
  // Rows past the tensor read its row 0 (rowoff was set so): no branch
  // around the loads, so a caller's later loads stay in flight while it
  // waits for these.  ZERO clears such rows; callers that never store those
  // rows' results skip it (the select would make every load of the slot
  // complete wherever the compiler places it).
  template <bool TR, int S = 0, bool ZERO = true>
  __device__ inline void load(const int32_t* phi, uint64_t key, int log2_page, int kb) {
    const int64_t koff = int64_t(kb) * STEP_BYTES;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const u32x4 v =
          __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(row_addr<TR>(phi, key, log2_page, r[i], koff)));
      g[S][i] = !ZERO || r[i].ok ? v : u32x4{0u, 0u, 0u, 0u};
    }
  }
  template <int S = 0>
  __device__ inline void store(uint8_t* tile) const {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if constexpr (F8) {
        const uint32_t w[4] = {g[S][i].x, g[S][i].y, g[S][i].z, g[S][i].w};
        uint32_t o[8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          o[2 * j] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w[j], 1.0f, false));
          o[2 * j + 1] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w[j], 1.0f, true));
        }
        const int row = tr0 + ROW_STRIDE * i;
        *reinterpret_cast<u32x4*>(tile + swz(row, 2 * c)) = u32x4{o[0], o[1], o[2], o[3]};
        *reinterpret_cast<u32x4*>(tile + swz(row, 2 * c + 1)) = u32x4{o[4], o[5], o[6], o[7]};
      } else {
        *reinterpret_cast<u32x4*>(tile + swz(tr0 + ROW_STRIDE * i, c)) = g[S][i];
      }
    }
  }
};

// XCD-aware tile order: consecutive workgroup ids go to different XCDs, so
// give each XCD a contiguous run of tiles of a grouped order (groups of
// GROUP_M token tiles, token tile fastest inside a group).  The 32
// workgroups an XCD runs at once then cover about 8 token tiles x 4 weight
// tiles, and each X and W slice they fetch serves 4 and 8 of them from the
// XCD's L2, instead of 32 token tiles each fetching its own X slice.
__device__ inline bool tile_coords(const GemmArgs& a, int& tile_m, int& tile_n) {
  constexpr int GROUP_M = 8;
  const int ntiles = a.tiles_m * a.tiles_n;
  const int b = blockIdx.x;
  const int per_xcd = (ntiles + 7) / 8;
  const int xcd = b % 8, slot = b / 8;
  const int t_id = xcd * per_xcd + slot;
  if (t_id >= ntiles) return false;
  const int per_group = GROUP_M * a.tiles_n;
  const int first_m = (t_id / per_group) * GROUP_M;
  const int group_m = min(a.tiles_m - first_m, GROUP_M);
  const int in_group = t_id % per_group;
  tile_m = first_m + in_group % group_m;
  tile_n = in_group / group_m;
  return true;
}

// Tile rows of a wave's NB_ row blocks (the wave owns WN_ of the 256 rows).
// SwiGLU: NB_/2 gate blocks, then the up blocks of the same hidden units.
template <int EPI, int NB_ = NB, int WN_ = WN>
__device__ inline void wave_rows(int wn, int (&wrow)[NB_]) {
#pragma unroll
  for (int nb = 0; nb < NB_; ++nb)
    wrow[nb] =
        EPI == kSwiGLU ? (nb < NB_ / 2 ? 0 : BN / 2) + wn * (WN_ / 2) + (nb % (NB_ / 2)) * 16 : wn * WN_ + nb * 16;
}

// Results of a wave's NB_ x MB_ blocks (WM_ tokens, WN_ rows): lane l of
// block (nb, mb) holds rows wrow[nb] + 4*(l/16) + r (r = 0..3) of token
// mb*16 + l%16 of the wave's token range.
template <int EPI, bool A8, int NB_ = NB, int MB_ = MB, int WM_ = WM, int WN_ = WN>
__device__ __forceinline__ void gemm_epilogue(const GemmArgs& a, const f32x4 (&acc)[NB_][MB_], int tile_m, int tile_n, int wm,
                                     int wn, const int (&wrow)[NB_], int lane) {
  constexpr int NB = NB_, MB = MB_, WM = WM_, WN = WN_;
  const int r4 = 4 * (lane >> 4);
  const int tok = lane & 15;
  if constexpr (EPI == kStore) {
#pragma clang loop unroll(full)
    for (int nb = 0; nb < NB; ++nb) {
      const int tr0 = wrow[nb] + r4;  // first of this lane's 4 tile rows
      int seg, n0;
      const bool ok0 = tile_row<EPI>(a, tile_n, tr0, seg, n0);
      if (!ok0) continue;
      const int rows = a.seg[seg].rows;
      const int32_t* perm = a.seg[seg].out_perm;
      const float* scale = a.seg[seg].scale;
      const int out_off = a.seg[seg].out_off;
#pragma clang loop unroll(full)
      for (int mb = 0; mb < MB; ++mb) {
        const int m = tile_m * BM + wm * WM + mb * 16 + tok;
        if (m >= a.M) continue;
        uint16_t* yrow = static_cast<uint16_t*>(a.y) + int64_t(m) * a.ldy + out_off;
        // a8: the token scale first, then the weight-row scale
        const float ts = A8 ? a.sx[m] : 1.f;
        float v[4] = {acc[nb][mb][0] * ts, acc[nb][mb][1] * ts, acc[nb][mb][2] * ts, acc[nb][mb][3] * ts};
        if (!perm && a.vec_store && n0 + 3 < rows) {
          uint32_t lo, hi;
          float s0 = scale ? scale[n0] : 1.f, s1 = scale ? scale[n0 + 1] : 1.f;
          float s2 = scale ? scale[n0 + 2] : 1.f, s3 = scale ? scale[n0 + 3] : 1.f;
          lo = uint32_t(f32_to_bf16_rne(v[0] * s0)) | (uint32_t(f32_to_bf16_rne(v[1] * s1)) << 16);
          hi = uint32_t(f32_to_bf16_rne(v[2] * s2)) | (uint32_t(f32_to_bf16_rne(v[3] * s3)) << 16);
          *reinterpret_cast<uint2*>(yrow + n0) = make_uint2(lo, hi);
        } else {
#pragma clang loop unroll(full)
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
#pragma clang loop unroll(full)
    for (int nb = 0; nb < NB / 2; ++nb) {
      const int j0 = tile_n * (BN / 2) + wn * (WN / 2) + nb * 16 + r4;
      if (j0 >= dff) continue;
#pragma clang loop unroll(full)
      for (int mb = 0; mb < MB; ++mb) {
        const int m = tile_m * BM + wm * WM + mb * 16 + tok;
        if (m >= a.M) continue;
        uint16_t* hrow = static_cast<uint16_t*>(a.y) + int64_t(m) * a.ldy;
        const float ts = A8 ? a.sx[m] : 1.f;
        uint16_t hv[4];
#pragma clang loop unroll(full)
        for (int r = 0; r < 4; ++r) {
          const int j = j0 + r;
          const int jj = j < dff ? j : dff - 1;
          const float g = acc[nb][mb][r] * ts * (sg ? sg[jj] : 1.f);
          const float u = acc[nb + NB / 2][mb][r] * ts * (su ? su[jj] : 1.f);
          hv[r] = f32_to_bf16_rne(g / (1.0f + expf(-g)) * u);
        }
        if (a.vec_store && j0 + 3 < dff) {
          *reinterpret_cast<uint2*>(hrow + j0) =
              make_uint2(uint32_t(hv[0]) | (uint32_t(hv[1]) << 16), uint32_t(hv[2]) | (uint32_t(hv[3]) << 16));
        } else {
#pragma clang loop unroll(full)
          for (int r = 0; r < 4; ++r)
            if (j0 + r < dff) hrow[j0 + r] = hv[r];
        }
      }
    }
  }
}

// F8: FP8 weights; A8: FP8 x FP8 MFMA on quantised activations (needs F8)
template <bool TR, int EPI, bool F8, bool A8>
__global__ __launch_bounds__(NTHREADS, 1) void gemm_kernel(const GemmArgs a) {
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  // buffer b: X tile at smem + 2b*TILE_BYTES, W tile right after it
  auto lds_x = [&](int buf) { return smem + buf * 2 * TILE_BYTES; };
  auto lds_w = [&](int buf) { return smem + buf * 2 * TILE_BYTES + TILE_BYTES; };

  int tile_m, tile_n;
  if (!tile_coords(a, tile_m, tile_n)) return;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;

  // activation slots: rows (tid >> 3) + 64 i, 16 B chunk (tid & 7); a K step
  // is 128 bytes of a row in both modes
  const int ch = tid & 7;
  const uint8_t* xrow[LOADS];
  bool xok[LOADS];
  const int64_t ldx_bytes = A8 ? a.ldx : a.ldx * 2;
#pragma unroll
  for (int i = 0; i < LOADS; ++i) {
    const int tr = (tid >> 3) + 64 * i;
    const int m = tile_m * BM + tr;
    xok[i] = m < a.M;
    xrow[i] = reinterpret_cast<const uint8_t*>(a.x) + int64_t(xok[i] ? m : 0) * ldx_bytes + ch * 16;
  }
  // a8 reads the FP8 weight bytes as they are (128 elements per K step)
  WTile<BN, NTHREADS, F8 && !A8> wt;
  wt.init(tid, a.pool, a.seg, a.row_bytes,
          [&](int tr, int& seg, int& n) { return tile_row<EPI>(a, tile_n, tr, seg, n); });

  u32x4 gx[LOADS];
  auto gload = [&](int kb) {
#pragma unroll
    for (int i = 0; i < LOADS; ++i)
      gx[i] = xok[i] ? *reinterpret_cast<const u32x4*>(xrow[i] + int64_t(kb) * ROWB) : u32x4{0u, 0u, 0u, 0u};
    wt.template load<TR>(a.phi, a.phi_key, a.log2_page, kb);
  };
  auto swrite = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LOADS; ++i) {
      const int tr = (tid >> 3) + 64 * i;
      *reinterpret_cast<u32x4*>(lds_x(buf) + swz(tr, ch)) = gx[i];
    }
    wt.store(lds_w(buf));
  };

  f32x4 acc[NB][MB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < MB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  int wrow[NB];
  wave_rows<EPI>(wn, wrow);

  const int nk = a.K / (A8 ? 2 * BK : BK);
  gload(0);
  swrite(0);
  __syncthreads();
  for (int kb = 0; kb < nk; ++kb) {
    const int buf = kb & 1;
    if (kb + 1 < nk) gload(kb + 1);
    // weight fragments of the wave's NB row blocks stay in registers while
    // the MB token fragments are read one at a time
    if constexpr (A8) {
      const int c0 = 2 * (lane >> 4);
      auto frag = [&](const uint8_t* tile, int r) {
        const u32x4 lo = *reinterpret_cast<const u32x4*>(tile + swz(r, c0));
        const u32x4 hi = *reinterpret_cast<const u32x4*>(tile + swz(r, c0 + 1));
        return i32x8{int(lo.x), int(lo.y), int(lo.z), int(lo.w), int(hi.x), int(hi.y), int(hi.z), int(hi.w)};
      };
      i32x8 fa[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) fa[nb] = frag(lds_w(buf), wrow[nb] + (lane & 15));
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        const i32x8 fb = frag(lds_x(buf), wm * WM + mb * 16 + (lane & 15));
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[nb][mb] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(fa[nb], fb, acc[nb][mb], 0, 0, 0, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < BK / 32; ++s) {
        const int chunk = s * 4 + (lane >> 4);
        bf16x8_t fa[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          fa[nb] = *reinterpret_cast<const bf16x8_t*>(lds_w(buf) + swz(wrow[nb] + (lane & 15), chunk));
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
          const bf16x8_t fb =
              *reinterpret_cast<const bf16x8_t*>(lds_x(buf) + swz(wm * WM + mb * 16 + (lane & 15), chunk));
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            acc[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[nb], fb, acc[nb][mb], 0, 0, 0);
        }
      }
    }
    if (kb + 1 < nk) swrite(buf ^ 1);
    __syncthreads();
  }

  gemm_epilogue<EPI, A8>(a, acc, tile_m, tile_n, wm, wn, wrow, lane);
}

// ---------------------------------------------------------------------------
// BF16 prefill GEMM with direct global -> LDS loads.  The register-staged
// kernel above can keep only one K step in flight (its staging registers and
// 128 FP32 accumulators fill the 256 VGPRs of two waves per SIMD), so each
// K step waits out a full memory round trip.  Here global_load_lds_dwordx4
// writes each lane's 16 bytes straight into LDS, so no registers are spent
// on staging and the tile ring can be deeper: DSTAGES stages of 32 K
// elements (64-byte tile rows, 32 KiB per stage for both operands), loads
// issued DSTAGES - 1 stages ahead.  A wave's load fills 1 KiB of LDS in lane
// order (16 rows x 4 chunks), so the XOR swizzle that keeps fragment reads
// conflict-free is applied on the global side: the lane that fills LDS slot
// s of tile row r fetches chunk s ^ ((r >> 1) & 3) of that row.  Each lane
// keeps two fixed weight rows for the whole K loop (cached page
// translation, as above).  Waits are explicit: before consuming stage kb a
// lane waits until only the loads of the DMA_AHEAD younger stages remain,
// then the workgroup barrier makes every lane's stage kb visible and frees
// the buffer the next stage is loaded into.
constexpr int DBK = 32;                     // K elements per stage
constexpr int DROWB = DBK * 2;              // bytes per tile row (64)
constexpr int DCH = DROWB / 16;             // 16-byte chunks per tile row
constexpr int DRPL = 1024 / DROWB;          // tile rows one wave load fills
constexpr int DTILE = BM * DROWB;           // bytes per operand per stage
constexpr int DSTAGES = 4;
constexpr int DWAVES = 8;                   // waves per workgroup of the BF16 prefill GEMM
constexpr int DSTAGE_BYTES = 2 * DTILE;
constexpr int DMA_AHEAD = DSTAGES - 2;      // younger stages still in flight at a wait
static_assert(DSTAGES * DSTAGE_BYTES <= 4 * TILE_BYTES, "ring exceeds the dynamic LDS reserved");

// chunk swizzle: the 8 consecutive rows one LDS pass serves land on 8
// distinct 16-byte slots of a 128-byte bank window
__device__ inline int dkey(int row) { return DCH == 4 ? (row >> 1) & 3 : row & 7; }
__device__ inline int dswz(int row, int chunk) { return row * DROWB + ((chunk ^ dkey(row)) << 4); }

// s_waitcnt vmcnt(N) lgkmcnt(0), expcnt untouched
template <int N>
__device__ inline void wait_vm_lgkm0() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (0 << 8) | ((N >> 4) << 14));
}

// WAVES = 8: a 2 x 4 wave grid of 128 x 64 wave tiles (two waves per SIMD);
// WAVES = 4: 2 x 2 of 128 x 128 (one wave per SIMD, accumulators in the
// accumulator registers).
template <int WAVES>
struct DmaGeom {
  static constexpr int NT = 64 * WAVES;
  static constexpr int WGN = WAVES / 2;          // waves along the weight rows
  static constexpr int WTM = BM / 2, WTN = BN / WGN;
  static constexpr int MBK = WTM / 16, NBK = WTN / 16;
  static constexpr int LOADS = BM / DRPL / WAVES;   // wave loads per operand per stage
};

template <bool TR, int EPI, int WAVES>
__global__ __launch_bounds__(64 * WAVES, 1) void gemm_dma_kernel(const GemmArgs a) {
  using G = DmaGeom<WAVES>;
  constexpr int NB = G::NBK, MB = G::MBK, WM = G::WTM, WN = G::WTN, DLOADS = G::LOADS;
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
  int tile_m, tile_n;
  if (!tile_coords(a, tile_m, tile_n)) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / G::WGN, wn = wave % G::WGN;

  // load slots: tile row DRPL * (DLOADS * wave + j) + lane / DCH of both operands
  const uint8_t* xptr[DLOADS];
  RowRef wr[DLOADS];
#pragma unroll
  for (int j = 0; j < DLOADS; ++j) {
    const int tr = DRPL * (DLOADS * wave + j) + lane / DCH;
    const int c = (lane % DCH) ^ dkey(tr);
    const int m = tile_m * BM + tr;
    // rows past M or past the tensor read row 0 (valid memory); their
    // results are never stored
    xptr[j] = reinterpret_cast<const uint8_t*>(a.x) + int64_t(m < a.M ? m : 0) * a.ldx * 2 + c * 16;
    int seg = 0, n = 0;
    const bool ok = tile_row<EPI>(a, tile_n, tr, seg, n);
    wr[j].pool = a.pool;
    wr[j].vbase = a.seg[seg].vbase;
    wr[j].rowoff = int64_t(ok ? n : 0) * a.row_bytes + c * 16;
    wr[j].cvp = -1;
    wr[j].cbase = 0;
    wr[j].ok = true;
  }

  f32x4 acc[NB][MB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < MB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  int wrow[NB];
  wave_rows<EPI, NB, WN>(wn, wrow);

  // iterations kb < 0 only issue the first DSTAGES - 1 stages
  const int nk = a.K / DBK;
  for (int kb = 1 - DSTAGES; kb < nk; ++kb) {
    if (kb >= 0) {
      if (kb + DMA_AHEAD < nk)
        wait_vm_lgkm0<DMA_AHEAD * 2 * DLOADS>();
      else
        wait_vm_lgkm0<0>();
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
    }
    // fragment reads of stage kb go out first, so their latency overlaps the
    // address work and issue of the next stage's loads
    const uint8_t* xs = smem + ((kb < 0 ? 0 : kb) % DSTAGES) * DSTAGE_BYTES;
    const uint8_t* ws = xs + DTILE;
    auto tok_frag = [&](int mb, int chunk) {
      return *reinterpret_cast<const bf16x8_t*>(xs + dswz(wm * WM + mb * 16 + (lane & 15), chunk));
    };
    bf16x8_t fa[NB], fb0, fb1;
    if (kb >= 0) {
      const int chunk = lane >> 4;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
        fa[nb] = *reinterpret_cast<const bf16x8_t*>(ws + dswz(wrow[nb] + (lane & 15), chunk));
      fb0 = tok_frag(0, chunk);
      fb1 = tok_frag(1, chunk);
    }
    const int ks = kb + DSTAGES - 1;   // stage issued now, into the buffer freed by the barrier
    if (ks < nk) {
      uint8_t* base = smem + (ks % DSTAGES) * DSTAGE_BYTES;
#pragma unroll
      for (int j = 0; j < DLOADS; ++j) {
        const int r0 = DRPL * (DLOADS * wave + j);
        const uint8_t* xsrc = xptr[j] + int64_t(ks) * DROWB;
        const uint8_t* wsrc = row_addr<TR>(a.phi, a.phi_key, a.log2_page, wr[j], int64_t(ks) * DROWB);
        __builtin_amdgcn_global_load_lds(xsrc, base + r0 * DROWB, 16, 0, 0);
        __builtin_amdgcn_global_load_lds(wsrc, base + DTILE + r0 * DROWB, 16, 0, 0);
      }
    }
    if (kb < 0) continue;
#pragma unroll
    for (int s = 0; s < DBK / 32; ++s) {
      const int chunk = s * 4 + (lane >> 4);
      if (s > 0) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          fa[nb] = *reinterpret_cast<const bf16x8_t*>(ws + dswz(wrow[nb] + (lane & 15), chunk));
        fb0 = tok_frag(0, chunk);
        fb1 = tok_frag(1, chunk);
      }
      // token fragments two blocks ahead of the MFMAs that use them
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        bf16x8_t fbn = fb1;
        if (mb + 2 < MB) fbn = tok_frag(mb + 2, chunk);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[nb][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[nb], fb0, acc[nb][mb], 0, 0, 0);
        fb0 = fb1;
        fb1 = fbn;
      }
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        __builtin_amdgcn_sched_group_barrier(0x008, NB, 0);
        if (mb + 2 < MB) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
    }
    asm volatile("" ::: "memory");
  }
  gemm_epilogue<EPI, false, NB, MB, WM, WN>(a, acc, tile_m, tile_n, wm, wn, wrow, lane);
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

// Nearest E4M3 (OCP "FN" variant) code of a binary32 value, ties to the even
// code, saturating at 448, NaN -> 0x7F.  Below 2^-6 the codes are the
// multiples of 2^-9 (code = rint(|v| * 512), exact scaling); above, the 23
// fraction bits are rounded to 3 and a carry out of the fraction moves the
// code to the next binade by plain addition.
__device__ inline float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

// One workgroup per token row: max |x| over the row, s = max / 448 (1 for a
// zero row), then q[j] = code(x[perm[j]] / s) with the IEEE binary32 quotient.
__global__ __launch_bounds__(256) void quant_rows_kernel(const uint16_t* __restrict__ x, int64_t ldx,
                                                         const int32_t* __restrict__ perm, uint8_t* __restrict__ q,
                                                         float* __restrict__ s, int64_t K, int vec) {
  __shared__ float red[4];
  const int64_t m = blockIdx.x;
  const uint16_t* xr = x + m * ldx;
  uint8_t* qr = q + m * K;
  const int t = threadIdx.x;
  float amax = 0.f;
  if (vec) {
    for (int64_t k = int64_t(t) * 8; k < K; k += 256 * 8) {
      const u32x4 w = *reinterpret_cast<const u32x4*>(xr + k);
      const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        amax = fmaxf(amax, fabsf(bf16_bits_to_f32(ww[i] & 0xffffu)));
        amax = fmaxf(amax, fabsf(bf16_bits_to_f32(ww[i] >> 16)));
      }
    }
  } else {
    for (int64_t k = t; k < K; k += 256) amax = fmaxf(amax, fabsf(bf16_bits_to_f32(xr[k])));
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) amax = fmaxf(amax, __shfl_xor(amax, d));
  if ((t & 63) == 0) red[t >> 6] = amax;
  __syncthreads();
  amax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  float sc = amax / 448.0f;
  if (sc == 0.f) sc = 1.0f;
  if (t == 0) s[m] = sc;
  if (vec) {
    for (int64_t k = int64_t(t) * 8; k < K; k += 256 * 8) {
      const u32x4 w = *reinterpret_cast<const u32x4*>(xr + k);
      const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
      uint32_t out[2] = {0u, 0u};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const uint32_t lo = e4m3_code(bf16_bits_to_f32(ww[i] & 0xffffu) / sc);
        const uint32_t hi = e4m3_code(bf16_bits_to_f32(ww[i] >> 16) / sc);
        out[i >> 1] |= (lo | (hi << 8)) << (16 * (i & 1));
      }
      *reinterpret_cast<uint2*>(qr + k) = make_uint2(out[0], out[1]);
    }
  } else {
    for (int64_t k = t; k < K; k += 256) {
      const int64_t src = perm ? perm[k] : k;
      qr[k] = uint8_t(e4m3_code(bf16_bits_to_f32(xr[src]) / sc));
    }
  }
}

// The same with the gather through perm (a down projection's hidden order):
// the row is read once in its own order with 16-byte loads, for the maximum
// and into LDS, then the codes are formed in stored order from LDS, four per
// 16-byte load of perm.  Same arithmetic per element as quant_rows_kernel.
// Needs K % 8 == 0, 16-byte aligned rows, perm and q rows 4-byte aligned,
// and K * 2 bytes of LDS.
__global__ __launch_bounds__(256) void quant_rows_gather_kernel(const uint16_t* __restrict__ x, int64_t ldx,
                                                                const int32_t* __restrict__ perm,
                                                                uint8_t* __restrict__ q, float* __restrict__ s,
                                                                int64_t K) {
  extern __shared__ __attribute__((aligned(16))) uint8_t xs_raw[];
  uint16_t* xs = reinterpret_cast<uint16_t*>(xs_raw);
  __shared__ float red[4];
  const int64_t m = blockIdx.x;
  const uint16_t* xr = x + m * ldx;
  uint8_t* qr = q + m * K;
  const int t = threadIdx.x;
  float amax = 0.f;
  for (int64_t k = int64_t(t) * 8; k < K; k += 256 * 8) {
    const u32x4 w = *reinterpret_cast<const u32x4*>(xr + k);
    *reinterpret_cast<u32x4*>(xs + k) = w;
    const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      amax = fmaxf(amax, fabsf(bf16_bits_to_f32(ww[i] & 0xffffu)));
      amax = fmaxf(amax, fabsf(bf16_bits_to_f32(ww[i] >> 16)));
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) amax = fmaxf(amax, __shfl_xor(amax, d));
  if ((t & 63) == 0) red[t >> 6] = amax;
  __syncthreads();
  amax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  float sc = amax / 448.0f;
  if (sc == 0.f) sc = 1.0f;
  if (t == 0) s[m] = sc;
  for (int64_t k = int64_t(t) * 4; k < K; k += 256 * 4) {
    const u32x4 p = *reinterpret_cast<const u32x4*>(perm + k);
    const uint32_t pp[4] = {p.x, p.y, p.z, p.w};
    uint32_t out = 0u;
#pragma unroll
    for (int i = 0; i < 4; ++i) out |= e4m3_code(bf16_bits_to_f32(xs[pp[i]]) / sc) << (8 * i);
    *reinterpret_cast<uint32_t*>(qr + k) = out;
  }
}

// ---------------------------------------------------------------------------
// Skinny split-K GEMM for decode batches (5..256 tokens).  A 256-row tile
// leaves a 4096-row projection only 16 workgroups; here a workgroup of 4
// waves takes 64 weight rows x a 16/32/64/128/256-token tile x one K slice
// (SBK = 64 per step; 20 to 80 KiB of LDS), and the K slices of a row tile
// are spread over workgroups.  Each slice writes FP32 partial sums
// part[slice][token][launch-row]; skinny_reduce_kernel adds the slices in a
// fixed order (deterministic) and applies the epilogue.  SwiGLU tiles hold
// 32 gate rows and the same 32 up rows.
constexpr int SBK = 64, STHREADS = 256;
// weight rows per tile: 128 from 128-token tiles, which halves the activation
// bytes staged per weight byte (every row tile stages the whole token tile;
// measured +5% on the 4096/14336 layer at M=128), else 64.  256-token tiles
// run 8 waves (two per SIMD) so that each wave still owns a 64 x 64 block.
template <int SBM>
constexpr int sbn_for() { return SBM >= 128 ? 128 : 64; }
template <int SBM>
constexpr int snt_for() { return SBM == 256 ? 512 : STHREADS; }

template <int EPI, int SBN>
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

// SBM = token tile (16 .. 256): the batch is padded only to SBM.
template <int SBM>
constexpr int skinny_lds_bytes() { return 2 * (SBM + sbn_for<SBM>()) * ROWB; }

template <int SBM, bool TR, int EPI, bool F8>
__global__ __launch_bounds__(snt_for<SBM>()) void skinny_kernel(const SkinnyArgs a) {
  constexpr int SBN = sbn_for<SBM>();
  constexpr int NT = snt_for<SBM>();
  constexpr int S_WTILE = SBN * ROWB;
  constexpr int XTILE = SBM * ROWB;
  constexpr int XCH = SBM * (ROWB / 16);   // 16-byte chunks of the token tile
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];   // skinny_lds_bytes<SBM>()
  auto lds_x = [&](int buf) { return smem + buf * (XTILE + S_WTILE); };
  auto lds_w = [&](int buf) { return smem + buf * (XTILE + S_WTILE) + XTILE; };
  const int ks = blockIdx.x % a.ksplit;
  const int tile_n = blockIdx.x / a.ksplit;
  const int kb_begin = ks * a.kblocks_per_split;
  int kb_end = kb_begin + a.kblocks_per_split;
  if (kb_end > a.K / SBK) kb_end = a.K / SBK;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int ch = tid & 7;

  // token tile: XCH 16-byte chunks, chunk idx = tid + NT*i -> row idx/8, chunk idx%8
  constexpr int XL = (XCH + NT - 1) / NT;
  bool xslot[XL], xok[XL];
  int xr[XL];
  const uint16_t* xrow[XL];
#pragma unroll
  for (int i = 0; i < XL; ++i) {
    const int idx = tid + NT * i;
    xslot[i] = idx < XCH;
    xr[i] = idx >> 3;
    xok[i] = xslot[i] && xr[i] < a.M;
    xrow[i] = a.x + int64_t(xok[i] ? xr[i] : 0) * a.ldx + ch * 8;
  }
  // SD K steps are held in registers: the loads of steps kb+1 .. kb+SD are
  // in flight while step kb is multiplied out of LDS (tiles up to 64 tokens;
  // the larger ones fill a CU with fewer workgroups and keep one step ahead)
  constexpr int SD = SBM <= 64 ? 3 : 1;
  WTile<SBN, NT, F8, SD> wt;
  wt.init(tid, a.pool, a.seg, a.row_bytes,
          [&](int tr, int& seg, int& n) { return skinny_row<EPI, SBN>(a, tile_n, tr, seg, n); });
  u32x4 gx[SD][XL];
  // padding tokens read token 0 (valid memory; their sums are never stored),
  // so the loads carry no branch
  auto gload = [&](auto slot, int kb) {
    constexpr int S = decltype(slot)::value;
#pragma unroll
    for (int i = 0; i < XL; ++i) gx[S][i] = *reinterpret_cast<const u32x4*>(xrow[i] + kb * SBK);
    wt.template load<TR, S, false>(a.phi, a.phi_key, a.log2_page, kb);   // padding rows are never stored
  };
  auto swrite = [&](auto slot, int buf) {
    constexpr int S = decltype(slot)::value;
#pragma unroll
    for (int i = 0; i < XL; ++i)
      if (xslot[i]) *reinterpret_cast<u32x4*>(lds_x(buf) + swz(xr[i], ch)) = gx[S][i];
    wt.template store<S>(lds_w(buf));
  };
  // wave grid: WR waves along the SBN rows x WT along the tokens.  Tiles of
  // 128+ tokens use 2 x (waves / 2) (each wave 64 rows x 64 tokens), which
  // reads fewer fragment bytes from LDS per MFMA than 4 x 1.
  constexpr int NW = NT / 64;
  constexpr int WR = SBM >= 128 ? 2 : 4, WT = NW / WR;
  constexpr int RB = SBN / WR / 16, TB = SBM / WT / 16;   // 16-blocks per wave
  const int gr = wave % WR, gt = wave / WR;   // this wave's place in the grid
  f32x4 acc[RB][TB];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int j = 0; j < TB; ++j) acc[b][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int wrow = gr * (SBN / WR);
  const int klast = kb_end - 1;
  if (kb_begin < kb_end) {
    static_for<0, SD>([&](auto slot) { gload(slot, min(kb_begin + int(decltype(slot)::value), klast)); });
    swrite(std::integral_constant<int, 0>{}, 0);
  }
  __syncthreads();
  // one K step from LDS buffer buf; slot S held step kb (already in LDS) and
  // is refilled with step kb + SD (the last step again near the end, rather
  // than a branch around the loads)
  // (LAST: the step may be the slice's last, so the write of the next one is
  // guarded; steps of the steady state write it unconditionally, which keeps
  // the wait counts exact)
  auto kstep = [&](auto slot, auto last, int kb) {
    constexpr int S = decltype(slot)::value;
    constexpr bool LAST = decltype(last)::value;
    const int buf = (kb - kb_begin) & 1;
    gload(slot, min(kb + SD, klast));
#pragma unroll
    for (int s = 0; s < SBK / 32; ++s) {
      const int chunk = s * 4 + (lane >> 4);
      bf16x8_t fa[RB];
#pragma unroll
      for (int b = 0; b < RB; ++b)
        fa[b] = *reinterpret_cast<const bf16x8_t*>(lds_w(buf) + swz(wrow + b * 16 + (lane & 15), chunk));
#pragma unroll
      for (int j = 0; j < TB; ++j) {
        const int mb = gt * TB + j;
        const bf16x8_t fb = *reinterpret_cast<const bf16x8_t*>(lds_x(buf) + swz(mb * 16 + (lane & 15), chunk));
#pragma unroll
        for (int b = 0; b < RB; ++b) acc[b][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[b], fb, acc[b][j], 0, 0, 0);
      }
    }
    if (!LAST || kb + 1 < kb_end) swrite(std::integral_constant<int, (S + 1) % SD>{}, buf ^ 1);
    __syncthreads();
  };
  int kb = kb_begin;
  for (; kb + SD < kb_end; kb += SD)
    static_for<0, SD>([&](auto slot) { kstep(slot, std::false_type{}, kb + int(decltype(slot)::value)); });
  static_for<0, SD>([&](auto slot) {
    if (kb + int(decltype(slot)::value) < kb_end) kstep(slot, std::true_type{}, kb + int(decltype(slot)::value));
  });
  // partial sums: lane holds launch-rows wrow + 16 b + 4*(lane/16) + r of
  // token (gt*TB + j)*16 + lane%16
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const int row0 = tile_n * SBN + wrow + b * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int j = 0; j < TB; ++j) {
      const int m = (gt * TB + j) * 16 + (lane & 15);
      if (m >= a.M) continue;
      float* dst = a.part + (int64_t(ks) * a.M + m) * a.ldp + row0;
      *reinterpret_cast<f32x4*>(dst) = acc[b][j];
    }
  }
}

// BF16 weights at 65..256 tokens: 8-wave tiles of 128 or 256 tokens x 128
// weight rows with direct global -> LDS loads.  One such workgroup fills a
// CU, so with register staging every K step would wait out a full memory
// round trip; here global_load_lds_dwordx4 writes each lane's 16 bytes
// straight into a ring of LDS stages (one K step of the token and weight
// tiles each: 4 x 32 KiB for 128 tokens, 3 x 48 KiB for 256), issued
// stages - 1 steps ahead.  A wave load fills 8 tile
// rows in lane order, so the XOR swizzle of the fragment reads is applied on
// the global side: the lane filling slot s of tile row r fetches chunk
// s ^ (r & 7).  Padding tokens read token 0 and padding rows read row 0
// (valid memory; their results are never stored).
template <int SBM>
constexpr int sds_stages() { return SBM == 256 ? 3 : 4; }
template <int SBM>
constexpr int sds_stage_bytes() { return (SBM + 128) * ROWB; }

// A8: FP8 weights meet per-token E4M3 activations (quantised beforehand) in
// v_mfma_f32_16x16x128_f8f6f4; a K step is then 128 elements, still 128 bytes
// of every tile row, so the ring, the loads and the swizzle are the same.
template <int SBM, bool TR, int EPI, bool A8>
__global__ __launch_bounds__(512) void skinny_dma_kernel(const SkinnyArgs a) {
  constexpr int SBN = 128, NW = 8;
  constexpr int SDS_STAGES = sds_stages<SBM>(), SDS_STAGE_BYTES = sds_stage_bytes<SBM>();
  constexpr int XT = SBM * ROWB;
  constexpr int XLD = SBM / 8 / NW, WLD = SBN / 8 / NW;   // wave loads per stage: 4 token, 2 weight
  constexpr int KSTEP = A8 ? ROWB : SBK;                   // elements per K step
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];   // sds_stages * sds_stage_bytes
  const int ks = blockIdx.x % a.ksplit;
  const int tile_n = blockIdx.x / a.ksplit;
  const int kb_begin = ks * a.kblocks_per_split;
  int kb_end = kb_begin + a.kblocks_per_split;
  if (kb_end > a.K / KSTEP) kb_end = a.K / KSTEP;
  const int nloc = kb_end - kb_begin;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

  const uint8_t* xptr[XLD];
#pragma unroll
  for (int j = 0; j < XLD; ++j) {
    const int r = 8 * (XLD * wave + j) + (lane >> 3);
    const int c = (lane & 7) ^ (r & 7);
    xptr[j] = reinterpret_cast<const uint8_t*>(a.x) + int64_t(r < a.M ? r : 0) * a.ldx * (A8 ? 1 : 2) + c * 16;
  }
  RowRef wr[WLD];
#pragma unroll
  for (int j = 0; j < WLD; ++j) {
    const int tr = 8 * (WLD * wave + j) + (lane >> 3);
    const int c = (lane & 7) ^ (tr & 7);
    int seg = 0, n = 0;
    const bool ok = skinny_row<EPI, SBN>(a, tile_n, tr, seg, n);
    wr[j].pool = a.pool;
    wr[j].vbase = a.seg[seg].vbase;
    wr[j].rowoff = int64_t(ok ? n : 0) * a.row_bytes + c * 16;
    wr[j].cvp = -1;
    wr[j].cbase = 0;
    wr[j].ok = true;
  }
  // 2 x 4 wave grid, each wave 64 weight rows x 64 tokens
  constexpr int WR = 2, RB = SBN / WR / 16, TB = SBM / (NW / WR) / 16;
  const int gr = wave % WR, gt = wave / WR;
  const int wrow = gr * (SBN / WR);
  f32x4 acc[RB][TB];
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int j = 0; j < TB; ++j) acc[b][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // iterations i < 0 only issue the first SDS_STAGES - 1 steps
  for (int i = 1 - SDS_STAGES; i < nloc; ++i) {
    if (i >= 0) {
      // this lane's loads of step i are done once only the younger steps'
      // remain (up to stages - 2 of them); the barrier then publishes every
      // lane's step i and frees the buffer step i + stages - 1 is loaded into
      static_assert(SDS_STAGES <= 4, "wait chain covers two younger steps");
      if (SDS_STAGES == 4 && i + 2 < nloc)
        wait_vm_lgkm0<2 * (XLD + WLD)>();
      else if (i + 1 < nloc)
        wait_vm_lgkm0<XLD + WLD>();
      else
        wait_vm_lgkm0<0>();
      __builtin_amdgcn_s_barrier();
      asm volatile("" ::: "memory");
    }
    const int in = i + SDS_STAGES - 1;
    if (in < nloc) {
      uint8_t* base = smem + (in % SDS_STAGES) * SDS_STAGE_BYTES;
      const int64_t koff = int64_t(kb_begin + in) * ROWB;
#pragma unroll
      for (int j = 0; j < XLD; ++j) {
        const uint8_t* xsrc = xptr[j] + koff;
        __builtin_amdgcn_global_load_lds(xsrc, base + 8 * (XLD * wave + j) * ROWB, 16, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < WLD; ++j) {
        const uint8_t* wsrc = row_addr<TR>(a.phi, a.phi_key, a.log2_page, wr[j], koff);
        __builtin_amdgcn_global_load_lds(wsrc, base + XT + 8 * (WLD * wave + j) * ROWB, 16, 0, 0);
      }
    }
    if (i < 0) continue;
    const uint8_t* xs = smem + (i % SDS_STAGES) * SDS_STAGE_BYTES;
    const uint8_t* wsm = xs + XT;
    if constexpr (A8) {
      // a lane's 32 bytes of a 128-element K step: the same two swizzled
      // chunks on both operands, so k pairs up whatever order the
      // instruction uses inside its K slice
      const int c0 = 2 * (lane >> 4);
      auto frag = [&](const uint8_t* tile, int r) {
        const u32x4 lo = *reinterpret_cast<const u32x4*>(tile + swz(r, c0));
        const u32x4 hi = *reinterpret_cast<const u32x4*>(tile + swz(r, c0 + 1));
        return i32x8{int(lo.x), int(lo.y), int(lo.z), int(lo.w), int(hi.x), int(hi.y), int(hi.z), int(hi.w)};
      };
      i32x8 fa[RB];
#pragma unroll
      for (int b = 0; b < RB; ++b) fa[b] = frag(wsm, wrow + b * 16 + (lane & 15));
#pragma unroll
      for (int j = 0; j < TB; ++j) {
        const i32x8 fb = frag(xs, (gt * TB + j) * 16 + (lane & 15));
#pragma unroll
        for (int b = 0; b < RB; ++b)
          acc[b][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(fa[b], fb, acc[b][j], 0, 0, 0, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int s = 0; s < SBK / 32; ++s) {
        const int chunk = s * 4 + (lane >> 4);
        bf16x8_t fa[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b)
          fa[b] = *reinterpret_cast<const bf16x8_t*>(wsm + swz(wrow + b * 16 + (lane & 15), chunk));
#pragma unroll
        for (int j = 0; j < TB; ++j) {
          const int mb = gt * TB + j;
          const bf16x8_t fb = *reinterpret_cast<const bf16x8_t*>(xs + swz(mb * 16 + (lane & 15), chunk));
#pragma unroll
          for (int b = 0; b < RB; ++b)
            acc[b][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[b], fb, acc[b][j], 0, 0, 0);
        }
      }
    }
    asm volatile("" ::: "memory");
  }
#pragma unroll
  for (int b = 0; b < RB; ++b) {
    const int row0 = tile_n * SBN + wrow + b * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int j = 0; j < TB; ++j) {
      const int m = (gt * TB + j) * 16 + (lane & 15);
      if (m >= a.M) continue;
      float* dst = a.part + (int64_t(ks) * a.M + m) * a.ldp + row0;
      *reinterpret_cast<f32x4*>(dst) = acc[b][j];
    }
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
      const int half = a.tile_rows / 2;
      const int tile = c / half, j = c % half;
      const int rg = tile * a.tile_rows + j, ru = rg + half;
      float g = 0.f, u = 0.f;
      for (int ks = 0; ks < a.ksplit; ++ks) {
        const float* p = a.part + (int64_t(ks) * a.M + m) * a.ldp;
        g += p[rg];
        u += p[ru];
      }
      if (a.a8) {
        g *= a.sx[m];
        u *= a.sx[m];
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
      if (a.a8) v *= a.sx[m];
      if (a.seg[seg].scale) v *= a.seg[seg].scale[n];
      const int32_t* perm = a.seg[seg].out_perm;
      static_cast<uint16_t*>(a.y)[int64_t(m) * a.ldy + a.seg[seg].out_off + (perm ? perm[n] : n)] =
          f32_to_bf16_rne(v);
    }
  }
}

// ---------------------------------------------------------------------------
// MoE experts on MFMA, for calls whose active experts average 2+ tokens.  The
// tile list (moe_tiles_kernel) names, per token tile, the active-expert slot
// and the tile's first token; a workgroup takes one token tile (up to
// MOE_TM of that expert's (token, slot) pairs, gathered row by row) by one
// 64-row weight tile over the whole K, with the skinny kernel's double-
// buffered loaders (page-translated weight rows cached per lane, FP8 rows
// widened exactly), and writes the results directly: SwiGLU tiles hold 32
// gate and the same 32 up rows, paired through LDS after the K loop; down
// tiles scale each result by the slot's router weight.
constexpr int MOE_TM = 32;     // tokens per tile
constexpr int MOE_TN = 64;     // weight rows per tile

__global__ __launch_bounds__(1024) void moe_tiles_kernel(const MoeArgs a) {
  __shared__ int32_t scan[1024];
  const int n = a.M * a.topk;
  const int na = a.route[0];
  const int32_t* act_count = a.route + 1 + 2 * a.E;
  int32_t* tiles = a.route + 1 + 3 * a.E + n;   // [0] count, then (slot, first token) pairs
  const int t = threadIdx.x;
  int own = 0;
  for (int s = t; s < na; s += blockDim.x) own += (act_count[s] + MOE_TM - 1) / MOE_TM;
  scan[t] = own;
  __syncthreads();
  for (int off = 1; off < int(blockDim.x); off <<= 1) {
    const int v = t >= off ? scan[t - off] : 0;
    __syncthreads();
    scan[t] += v;
    __syncthreads();
  }
  int pos = scan[t] - own;
  for (int s = t; s < na; s += blockDim.x)
    for (int tok0 = 0; tok0 < act_count[s]; tok0 += MOE_TM) {
      tiles[1 + 2 * pos] = s;
      tiles[2 + 2 * pos] = tok0;
      ++pos;
    }
  if (t == int(blockDim.x) - 1) tiles[0] = scan[t];
}

template <int EPI, bool TR, bool F8>
__global__ __launch_bounds__(STHREADS) void moe_mfma_kernel(const MoeArgs a) {
  constexpr int XTILE = MOE_TM * ROWB, WTILE = MOE_TN * ROWB;
  extern __shared__ __attribute__((aligned(16))) uint8_t smem[];   // 2 * (XTILE + WTILE)
  auto lds_x = [&](int buf) { return smem + buf * (XTILE + WTILE); };
  auto lds_w = [&](int buf) { return smem + buf * (XTILE + WTILE) + XTILE; };
  const int n = a.M * a.topk;
  const int32_t* tiles = a.route + 1 + 3 * a.E + n;
  const int tile = blockIdx.x;
  if (tile >= tiles[0]) return;
  const int s = tiles[1 + 2 * tile], tok0 = tiles[2 + 2 * tile];
  const int e = a.route[1 + s], st = a.route[1 + a.E + s], cnt = a.route[1 + 2 * a.E + s];
  const int ntok = cnt - tok0 < MOE_TM ? cnt - tok0 : MOE_TM;
  const int32_t* ent = a.route + 1 + 3 * a.E + st + tok0;
  const MoeExpert& ex = a.experts[e];
  const int tile_n = blockIdx.y;
  const int K = EPI == kSwiGLU ? a.d_model : a.d_ffn;
  const int64_t row_bytes = int64_t(K) * (F8 ? 1 : 2);
  const int rows = EPI == kSwiGLU ? a.d_ffn : a.d_model;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int ch = tid & 7;
  // token rows: MOE_TM rows x 8 chunks of 16 B = one chunk per thread
  static_assert(MOE_TM * 8 == STHREADS, "one activation chunk per thread");
  const int xr = tid >> 3;
  const bool xok = xr < ntok;
  const int pair = xok ? ent[xr] : 0;
  const uint16_t* xrow = (EPI == kSwiGLU ? a.x + int64_t(pair / a.topk) * a.d_model
                                         : a.h + int64_t(pair) * a.d_ffn) + ch * 8;
  WSeg segs[2] = {};
  segs[0].vbase = EPI == kSwiGLU ? ex.vbase[0] : ex.vbase[2];
  segs[1].vbase = ex.vbase[1];
  WTile<MOE_TN, STHREADS, F8> wt;
  wt.init(tid, a.pool, segs, row_bytes, [&](int tr, int& seg, int& nn) {
    if (EPI == kSwiGLU) {
      seg = tr < MOE_TN / 2 ? 0 : 1;
      nn = tile_n * (MOE_TN / 2) + tr % (MOE_TN / 2);
    } else {
      seg = 0;
      nn = tile_n * MOE_TN + tr;
    }
    return nn < rows;
  });
  u32x4 gx;
  auto gload = [&](int kb) {
    gx = xok ? *reinterpret_cast<const u32x4*>(xrow + kb * SBK) : u32x4{0u, 0u, 0u, 0u};
    wt.template load<TR>(a.phi, a.phi_key, a.log2_page, kb);
  };
  auto swrite = [&](int buf) {
    *reinterpret_cast<u32x4*>(lds_x(buf) + swz(xr, ch)) = gx;
    wt.store(lds_w(buf));
  };
  // 4 waves along the 64 rows, each 16 rows x all MOE_TM tokens
  constexpr int TB = MOE_TM / 16;
  f32x4 acc[TB];
#pragma unroll
  for (int j = 0; j < TB; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int wrow = wave * 16;
  const int nk = K / SBK;
  gload(0);
  swrite(0);
  __syncthreads();
  for (int kb = 0; kb < nk; ++kb) {
    const int buf = kb & 1;
    if (kb + 1 < nk) gload(kb + 1);
#pragma unroll
    for (int q = 0; q < SBK / 32; ++q) {
      const int chunk = q * 4 + (lane >> 4);
      const bf16x8_t fa = *reinterpret_cast<const bf16x8_t*>(lds_w(buf) + swz(wrow + (lane & 15), chunk));
#pragma unroll
      for (int j = 0; j < TB; ++j) {
        const bf16x8_t fb = *reinterpret_cast<const bf16x8_t*>(lds_x(buf) + swz(j * 16 + (lane & 15), chunk));
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[j], 0, 0, 0);
      }
    }
    if (kb + 1 < nk) swrite(buf ^ 1);
    __syncthreads();
  }
  // lane holds tile rows wrow + 4*(lane/16) + r of token j*16 + lane%16
  const int r4 = wrow + 4 * (lane >> 4);
  if constexpr (EPI == kSwiGLU) {
    float* red = reinterpret_cast<float*>(smem);   // [MOE_TN][MOE_TM]; every buffer is free after the loop
#pragma unroll
    for (int j = 0; j < TB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(r4 + r) * MOE_TM + j * 16 + (lane & 15)] = acc[j][r];
    __syncthreads();
    for (int i = tid; i < (MOE_TN / 2) * MOE_TM; i += STHREADS) {
      const int u = i / MOE_TM, m = i % MOE_TM;
      const int unit = tile_n * (MOE_TN / 2) + u;
      if (m >= ntok || unit >= a.d_ffn) continue;
      float g = red[u * MOE_TM + m], v = red[(u + MOE_TN / 2) * MOE_TM + m];
      if (ex.scale_off[0] >= 0) g *= a.scales[ex.scale_off[0] + unit];
      if (ex.scale_off[1] >= 0) v *= a.scales[ex.scale_off[1] + unit];
      a.h[int64_t(ent[m]) * a.d_ffn + unit] = f32_to_bf16_rne(g / (1.0f + expf(-g)) * v);
    }
  } else {
#pragma unroll
    for (int j = 0; j < TB; ++j) {
      const int m = j * 16 + (lane & 15);
      if (m >= ntok) continue;
      const int p = ent[m];
      const float wgt = a.wts[p];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int nrow = tile_n * MOE_TN + r4 + r;
        if (nrow >= a.d_model) continue;
        float v = acc[j][r];
        if (ex.scale_off[2] >= 0) v *= a.scales[ex.scale_off[2] + nrow];
        a.yp[int64_t(p) * a.d_model + nrow] = v * wgt;
      }
    }
  }
}

}  // namespace

int gemm_lds_bytes() { return 4 * TILE_BYTES; }

hipError_t launch_moe_mfma(const MoeArgs& a, bool translate, hipStream_t s) {
  const int n = a.M * a.topk;
  if (n <= 0) return hipSuccess;
  if (a.d_model % SBK != 0 || a.d_ffn % SBK != 0) return hipErrorInvalidValue;
  const bool f8 = a.wtype == kFP8;
  using Fn = void (*)(const MoeArgs);
  Fn sw, dn;
  if (f8) {
    sw = translate ? moe_mfma_kernel<kSwiGLU, true, true> : moe_mfma_kernel<kSwiGLU, false, true>;
    dn = translate ? moe_mfma_kernel<kStore, true, true> : moe_mfma_kernel<kStore, false, true>;
  } else {
    sw = translate ? moe_mfma_kernel<kSwiGLU, true, false> : moe_mfma_kernel<kSwiGLU, false, false>;
    dn = translate ? moe_mfma_kernel<kStore, true, false> : moe_mfma_kernel<kStore, false, false>;
  }
  const unsigned max_tiles = unsigned(moe_max_tiles(n, a.E));
  const size_t lds = size_t(2) * (MOE_TM + MOE_TN) * ROWB;
  hipLaunchKernelGGL(moe_tiles_kernel, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(sw, dim3(max_tiles, unsigned((a.d_ffn + MOE_TN / 2 - 1) / (MOE_TN / 2))), dim3(STHREADS), lds, s,
                     a);
  hipLaunchKernelGGL(dn, dim3(max_tiles, unsigned((a.d_model + MOE_TN - 1) / MOE_TN)), dim3(STHREADS), lds, s, a);
  return hipGetLastError();
}

int64_t moe_max_tiles(int64_t pairs, int64_t experts) {
  const int64_t slots = pairs < experts ? pairs : experts;
  return (pairs + MOE_TM - 1) / MOE_TM + slots;
}
int gemm_tile_rows() { return BN; }
int gemm_k_step() { return BK; }
int gemm_k_step_a8() { return 2 * BK; }

hipError_t launch_quant_rows(const uint16_t* x, int64_t ldx, const int32_t* perm, uint8_t* q, float* s, int64_t M,
                             int64_t K, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  if (M > INT32_MAX) return hipErrorInvalidValue;
  const int vec = (!perm && K % 8 == 0 && ldx % 8 == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(q) % 8 == 0)
                      ? 1
                      : 0;
  // a gathered row fits in LDS (up to 32768 elements): one read of x, codes from LDS
  if (perm && K % 8 == 0 && K <= 32768 && ldx % 8 == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0 &&
      reinterpret_cast<uintptr_t>(perm) % 16 == 0 && reinterpret_cast<uintptr_t>(q) % 4 == 0) {
    const int lds = int(K * 2);   // at most 64 KiB, the default dynamic LDS limit
    hipLaunchKernelGGL(quant_rows_gather_kernel, dim3(unsigned(M)), dim3(256), size_t(lds), st, x, ldx, perm, q, s, K);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(quant_rows_kernel, dim3(unsigned(M)), dim3(256), 0, st, x, ldx, perm, q, s, K, vec);
  return hipGetLastError();
}

// Dynamic LDS above the default limit is allowed per kernel and device:
// raised once for each (device, kernel) pair, thread-safely.
static hipError_t raise_lds_limit(const void* fn, int lds) {
  static std::mutex mu;
  static std::set<std::pair<int, const void*>> raised;
  int dev = 0;
  if (hipError_t e = hipGetDevice(&dev)) return e;
  std::lock_guard<std::mutex> lock(mu);
  if (raised.count({dev, fn})) return hipSuccess;
  if (hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds)) return e;
  raised.insert({dev, fn});
  return hipSuccess;
}

hipError_t launch_gemm(const GemmArgs& a, bool translate, hipStream_t s) {
  const int ntiles = a.tiles_m * a.tiles_n;
  if (ntiles <= 0) return hipSuccess;
  const int blocks = (ntiles + 7) / 8 * 8;
  const size_t lds = size_t(gemm_lds_bytes());
  void (*fn)(const GemmArgs);
  const bool f8 = a.f8 != 0, a8 = a.a8 != 0;
  if (a8 && !f8) return hipErrorInvalidValue;
  const bool sw = a.mode == kSwiGLU;
  if (a8)
    fn = translate ? (sw ? gemm_kernel<true, kSwiGLU, true, true> : gemm_kernel<true, kStore, true, true>)
                   : (sw ? gemm_kernel<false, kSwiGLU, true, true> : gemm_kernel<false, kStore, true, true>);
  else if (f8)
    fn = translate ? (sw ? gemm_kernel<true, kSwiGLU, true, false> : gemm_kernel<true, kStore, true, false>)
                   : (sw ? gemm_kernel<false, kSwiGLU, true, false> : gemm_kernel<false, kStore, true, false>);
  else
    fn = translate ? (sw ? gemm_dma_kernel<true, kSwiGLU, DWAVES> : gemm_dma_kernel<true, kStore, DWAVES>)
                   : (sw ? gemm_dma_kernel<false, kSwiGLU, DWAVES> : gemm_dma_kernel<false, kStore, DWAVES>);
  const int threads = f8 ? NTHREADS : 64 * DWAVES;

  if (hipError_t e = raise_lds_limit(reinterpret_cast<const void*>(fn), int(lds))) return e;
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(threads), lds, s, a);
  return hipGetLastError();
}

int skinny_tile_rows(int64_t M) { return M > 64 ? sbn_for<128>() : sbn_for<64>(); }

template <int SBM, bool F8>
void (*skinny_fn2(bool translate, int mode))(const SkinnyArgs) {
  if (mode == kSwiGLU) return translate ? skinny_kernel<SBM, true, kSwiGLU, F8> : skinny_kernel<SBM, false, kSwiGLU, F8>;
  return translate ? skinny_kernel<SBM, true, kStore, F8> : skinny_kernel<SBM, false, kStore, F8>;
}

template <int SBM, bool A8>
void (*skinny_dma_fn2(bool translate, int mode))(const SkinnyArgs) {
  if (mode == kSwiGLU)
    return translate ? skinny_dma_kernel<SBM, true, kSwiGLU, A8> : skinny_dma_kernel<SBM, false, kSwiGLU, A8>;
  return translate ? skinny_dma_kernel<SBM, true, kStore, A8> : skinny_dma_kernel<SBM, false, kStore, A8>;
}

template <int SBM>
void (*skinny_dma_fn(bool translate, int mode, bool a8))(const SkinnyArgs) {
  return a8 ? skinny_dma_fn2<SBM, true>(translate, mode) : skinny_dma_fn2<SBM, false>(translate, mode);
}

template <int SBM>
void (*skinny_fn(bool translate, int mode, bool f8))(const SkinnyArgs) {
  return f8 ? skinny_fn2<SBM, true>(translate, mode) : skinny_fn2<SBM, false>(translate, mode);
}

hipError_t launch_skinny(const SkinnyArgs& a, bool translate, hipStream_t s) {
  const int64_t blocks = int64_t(a.tiles_n) * a.ksplit;
  if (blocks <= 0 || a.M <= 0) return hipSuccess;
  if (a.M > kSkinnyMaxTokens || a.K % SBK != 0 || a.tile_rows != skinny_tile_rows(a.M)) return hipErrorInvalidValue;
  const bool f8 = a.f8 != 0, a8 = a.a8 != 0;
  // FP8 x FP8 runs only on the direct-to-LDS tiles (above 64 tokens), in K steps of 128
  if (a8 && (!f8 || a.M <= 64 || a.K % (2 * SBK) != 0 || !a.sx)) return hipErrorInvalidValue;
  void (*fn)(const SkinnyArgs);
  int lds;
  if (a.M <= 16) fn = skinny_fn<16>(translate, a.mode, f8), lds = skinny_lds_bytes<16>();
  else if (a.M <= 32) fn = skinny_fn<32>(translate, a.mode, f8), lds = skinny_lds_bytes<32>();
  else if (a.M <= 64) fn = skinny_fn<64>(translate, a.mode, f8), lds = skinny_lds_bytes<64>();
  else if (f8 && !a8 && a.M <= 128) fn = skinny_fn<128>(translate, a.mode, f8), lds = skinny_lds_bytes<128>();
  else if (f8 && !a8) fn = skinny_fn<256>(translate, a.mode, f8), lds = skinny_lds_bytes<256>();
  else if (a.M <= 128) fn = skinny_dma_fn<128>(translate, a.mode, a8), lds = sds_stages<128>() * sds_stage_bytes<128>();
  else fn = skinny_dma_fn<256>(translate, a.mode, a8), lds = sds_stages<256>() * sds_stage_bytes<256>();
  const bool wide = a.M > 128 || (a.M > 64 && (!f8 || a8));   // 8-wave tiles
  if (lds > 64 * 1024)
    if (hipError_t e = raise_lds_limit(reinterpret_cast<const void*>(fn), lds)) return e;
  hipLaunchKernelGGL(fn, dim3(unsigned(blocks)), dim3(unsigned(wide ? 512 : STHREADS)), size_t(lds), s, a);
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

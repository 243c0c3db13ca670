// Decode GEMV over cloaked weights (CloakLM, arXiv 2606.18400, Section 4.2:
// weights live in scattered physical pages; inference is bandwidth-bound,
// so placement must not cost bandwidth).
//
// Shape of the work on gfx950:
//  * A weight row is streamed in 1 KiB "chunks": one wave-wide load of 16 B
//    per lane.  Rows are multiples of 16 B and pages powers of two >= 1 KiB,
//    so a chunk that starts 1 KiB-aligned in the tensor's stream sits inside
//    one page: the virtual->physical translation is ONE scalar load of the
//    page map per chunk (a second one only for rows whose size is not a
//    multiple of 1 KiB, where a chunk can cross a page boundary).
//  * The waves of a workgroup split a row's chunks (wave w takes chunks
//    w, w+W, ...) and every wave works on R rows at once, so each lane keeps
//    R independent 16 B loads in flight per chunk.
//  * The activations are gathered once per workgroup (through the hidden
//    permutation when the tensor's K is the permuted hidden dimension) into
//    registers: a wave only ever needs x at its own chunk positions.
//  * Dot products: v_dot2_f32_bf16 on bf16 pairs (FP8 weights are widened to
//    bf16 with v_cvt_scalef32_pk_bf16_fp8, exact for every E4M3 value), FMA
//    for f32; accumulation in f32.
//  * Reduction: a transposing butterfly over the 64 lanes (R*MT values are
//    reduced in about R*MT + 6 shuffles instead of 6*R*MT), then a sum over
//    the waves through LDS; the epilogue applies FP8 row scales, the output
//    scatter of gate/up rows, or the SwiGLU product of paired gate/up rows.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>

#include "kernels.hpp"

namespace cloak {
namespace {

typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2_t;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// The page map is read through the constant address space so that its
// wave-uniform lookups become scalar loads (lgkmcnt), which never make the
// vector weight loads wait for each other.
typedef const int32_t __attribute__((address_space(4)))* scalar_i32_ptr;

// Wave-uniform by construction (derived from the workgroup id and loop
// counters); readfirstlane tells the compiler so.
__device__ inline int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
  return int64_t((uint64_t(hi) << 32) | lo);
}

template <bool MASKED>
__device__ inline int64_t page_of(const int32_t* phi, uint64_t key, int64_t vpage) {
  const int64_t v = uniform64(vpage);
  const uint32_t e = uint32_t(((scalar_i32_ptr)phi)[v]);
  return int64_t(MASKED ? e ^ phi_mask(key, v) : e);
}

constexpr int kChunkBytes = 1024;
constexpr int kMaxWaves = 8;

template <int WT> struct WTraits;
template <> struct WTraits<kF32> { static constexpr int EPL = 4; static constexpr int XW = 4; };
template <> struct WTraits<kBF16> { static constexpr int EPL = 8; static constexpr int XW = 4; };
template <> struct WTraits<kFP8> { static constexpr int EPL = 16; static constexpr int XW = 8; };

__device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

__device__ inline bf16x2_t as_bf16x2(uint32_t v) { return __builtin_bit_cast(bf16x2_t, v); }

// One tensor of a launch, as the kernel uses it.
struct SegView {
  int64_t vbase, npages;
  const int32_t* out_perm;
  const float* scale;
  int32_t rows, row0, out_off;
};

__device__ inline SegView seg_at(const GemvArgs& a, int i) {
  // i is wave-uniform: one batch of scalar loads from the argument segment
  const WSeg& w = a.seg[i];
  SegView v;
  v.vbase = w.vbase;
  v.npages = w.npages;
  v.out_perm = w.out_perm;
  v.scale = w.scale;
  v.rows = w.rows;
  v.row0 = w.row0;
  v.out_off = w.out_off;
  return v;
}

// Rows of one group all belong to one tensor: the host starts every tensor
// on a multiple of R launch-rows.  SwiGLU groups pair R/2 gate rows
// (segment 0) with the same R/2 up rows (segment 1).
template <int R, int EPI>
__device__ inline int group_segment(const GemvArgs& a, int grp) {
  if (EPI == kSwiGLU) return 0;
  int s = 0;
#pragma unroll
  for (int i = 1; i < 4; ++i)
    if (i < a.nseg && grp * R >= a.seg[i].row0) s = i;
  return __builtin_amdgcn_readfirstlane(s);
}

template <int WT>
__device__ inline void load_x(const GemvArgs& a, int c, int m, int lane, uint32_t (&xr)[WTraits<WT>::XW]) {
  constexpr int EPL = WTraits<WT>::EPL;
  constexpr int XW = WTraits<WT>::XW;
  const int k0 = c * 64 * EPL + lane * EPL;
  const bool tok = m < a.mcount;
  const int64_t row = int64_t(a.m0 + (tok ? m : 0)) * a.ldx;   // a valid row for every lane
  if (a.x_vec && tok && k0 + EPL <= a.K) {
    // a lane's EPL activations are consecutive: XW / 4 aligned 16-byte loads
    const uint8_t* xb = static_cast<const uint8_t*>(a.x) + (row + k0) * (WT == kF32 ? 4 : 2);
#pragma unroll
    for (int j = 0; j < XW / 4; ++j) {
      const u32x4 v = reinterpret_cast<const u32x4*>(xb)[j];
      xr[4 * j] = v.x;
      xr[4 * j + 1] = v.y;
      xr[4 * j + 2] = v.z;
      xr[4 * j + 3] = v.w;
    }
    return;
  }
  // element by element (the gather of a down projection through pi, row
  // tails): every index first, then every element, each batch without
  // branches; out-of-range elements read a valid one and are zeroed
  int kk[EPL];
  bool ok[EPL];
#pragma unroll
  for (int e = 0; e < EPL; ++e) {
    ok[e] = tok && k0 + e < a.K;
    kk[e] = ok[e] ? k0 + e : 0;
  }
  if (a.x_perm) {
#pragma unroll
    for (int e = 0; e < EPL; ++e) kk[e] = a.x_perm[kk[e]];
  }
  if constexpr (WT == kF32) {
    const float* xp = static_cast<const float*>(a.x) + row;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const float v = xp[kk[e]];
      xr[e] = ok[e] ? __float_as_uint(v) : 0u;
    }
  } else {
    const uint16_t* xp = static_cast<const uint16_t*>(a.x) + row;
    uint32_t v[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) v[e] = xp[kk[e]];
#pragma unroll
    for (int e = 0; e < EPL; e += 2) xr[e / 2] = (ok[e] ? v[e] : 0u) | ((ok[e + 1] ? v[e + 1] : 0u) << 16);
  }
}

// Where chunk c of stored row n lives: the physical pages holding its first
// byte (p0) and, for a chunk that crosses a page boundary (rows whose size
// is not a multiple of 1 KiB), the next one (p1); `inpage` is the chunk's
// offset in p0.  All wave-uniform: scalar loads only.
struct ChunkLoc {
  int64_t p0, p1, inpage;
};

// TR: 0 untranslated twin, 1 plain page map, 2 masked page map
template <int TR>
__device__ inline ChunkLoc locate(const GemvArgs& a, const SegView& v, int n, int c) {
  const int64_t o = int64_t(n) * a.row_bytes + int64_t(c) * kChunkBytes;
  const int64_t page_bytes = int64_t(1) << a.log2_page;
  const int64_t vp = o >> a.log2_page;
  ChunkLoc L;
  L.inpage = o & (page_bytes - 1);
  const int64_t vpage = v.vbase + vp;
  // the second lookup is unconditional (index clamped to the tensor's last
  // page) so that both scalar loads of every row can be in flight together
  const int64_t vnext = vp + 1 < v.npages ? vpage + 1 : vpage;
  L.p0 = TR ? page_of<TR == 2>(a.phi, a.phi_key, vpage) : vpage;
  L.p1 = TR ? page_of<TR == 2>(a.phi, a.phi_key, vnext) : vnext;
  return L;
}

// This lane's 16 B of a located chunk (zero past the end of the row).
__device__ inline u32x4 load_chunk(const GemvArgs& a, const ChunkLoc& L, int lane, bool lane_ok) {
  const int64_t page_bytes = int64_t(1) << a.log2_page;
  const int64_t lo = L.inpage + int64_t(lane) * 16;
  const bool second = lo >= page_bytes;
  const int64_t phys = second ? L.p1 : L.p0;
  const uint8_t* addr = a.pool + (phys << a.log2_page) + (second ? lo - page_bytes : lo);
  u32x4 w = {0u, 0u, 0u, 0u};
  if (lane_ok) w = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(addr));
  return w;
}

// The same for rows of whole KiB (every chunk complete and inside one page):
// a scalar base plus the lane's offset, with no per-lane address arithmetic
// and no branch.  Callers point rows past the tensor at row 0 (valid
// memory; those rows are never stored).
__device__ inline u32x4 load_whole_chunk(const GemvArgs& a, const ChunkLoc& L, int lane) {
  const uint8_t* base = a.pool + ((L.p0 << a.log2_page) + L.inpage);
  return __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(base + lane * 16));
}

// `one` (1.0) is the FP8 conversions' scale operand; a caller may pass a
// value the compiler cannot see through to pin the conversions in place.
template <int WT>
__device__ inline float dot_chunk(const u32x4 w, const uint32_t (&x)[WTraits<WT>::XW], float acc,
                                  float one = 1.0f) {
  if constexpr (WT == kF32) {
    acc = fmaf(__uint_as_float(w.x), __uint_as_float(x[0]), acc);
    acc = fmaf(__uint_as_float(w.y), __uint_as_float(x[1]), acc);
    acc = fmaf(__uint_as_float(w.z), __uint_as_float(x[2]), acc);
    acc = fmaf(__uint_as_float(w.w), __uint_as_float(x[3]), acc);
  } else if constexpr (WT == kBF16) {
    acc = __builtin_amdgcn_fdot2_f32_bf16(as_bf16x2(w.x), as_bf16x2(x[0]), acc, false);
    acc = __builtin_amdgcn_fdot2_f32_bf16(as_bf16x2(w.y), as_bf16x2(x[1]), acc, false);
    acc = __builtin_amdgcn_fdot2_f32_bf16(as_bf16x2(w.z), as_bf16x2(x[2]), acc, false);
    acc = __builtin_amdgcn_fdot2_f32_bf16(as_bf16x2(w.w), as_bf16x2(x[3]), acc, false);
  } else {
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bf16x2_t lo = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(ws[i], one, false);
      const bf16x2_t hi = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(ws[i], one, true);
      acc = __builtin_amdgcn_fdot2_f32_bf16(lo, as_bf16x2(x[2 * i]), acc, false);
      acc = __builtin_amdgcn_fdot2_f32_bf16(hi, as_bf16x2(x[2 * i + 1]), acc, false);
    }
  }
  return acc;
}

// Transposing butterfly: on entry v[0..V) are per-lane partials; on exit
// v[0] of lane l is the 64-lane sum of value index (l >> (6 - log2 V)).
// Stage with partner distance D and COUNT live values: a lane keeps the
// half selected by its D bit and adds the partner's copy of that half;
// once one value is left, the remaining stages are plain xor sums.  Every
// count and index is a compile-time constant, so v stays in registers.
template <int D, int COUNT, int V>
struct LaneReduce {
  __device__ static inline void run(float (&v)[V], int lane) {
    const bool upper = (lane & D) != 0;
    if constexpr (COUNT > 1) {
      constexpr int H = COUNT / 2;
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const float send = upper ? v[i] : v[i + H];
        const float keep = upper ? v[i + H] : v[i];
        v[i] = keep + __shfl_xor(send, D);
      }
      if constexpr (D > 1) LaneReduce<D / 2, H, V>::run(v, lane);
    } else {
      v[0] += __shfl_xor(v[0], D);
      if constexpr (D > 1) LaneReduce<D / 2, 1, V>::run(v, lane);
    }
  }
};

template <int V>
__device__ inline void lane_reduce(float (&v)[V], int lane) {
  LaneReduce<32, V, V>::run(v, lane);
}

template <int N> struct Log2 { static constexpr int value = 1 + Log2<N / 2>::value; };
template <> struct Log2<1> { static constexpr int value = 0; };

template <int WT, int R, int CPW, int TR, int EPI>
struct GroupLoads {
  u32x4 w[CPW][R];
};

// Issue every weight load of group `grp` for this wave (page lookups first,
// as one batch of scalar loads, then R*CPW independent 16 B loads per lane).
template <int WT, int R, int CPW, int TR, int EPI>
__device__ inline void issue_group(const GemvArgs& a, int grp, int wave, int nwaves, int lane,
                                   GroupLoads<WT, R, CPW, TR, EPI>& L) {
  constexpr int EPL = WTraits<WT>::EPL;
  const SegView sv = seg_at(a, EPI == kSwiGLU ? 0 : group_segment<R, EPI>(a, grp));
  const SegView up = seg_at(a, EPI == kSwiGLU ? 1 : 0);
  if ((a.row_bytes & (kChunkBytes - 1)) == 0) {
    // whole-KiB rows: every lane of a chunk is in the row and in one page
#pragma unroll
    for (int i = 0; i < CPW; ++i) {
      const int c = wave + i * nwaves;
      if (c >= a.nchunks) {   // wave-uniform: this wave has no chunk in slot i
#pragma unroll
        for (int r = 0; r < R; ++r) L.w[i][r] = u32x4{0u, 0u, 0u, 0u};
        continue;
      }
      ChunkLoc loc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int n = EPI == kSwiGLU ? grp * (R / 2) + (r % (R / 2)) : grp * R + r - sv.row0;
        const SegView v = (EPI == kSwiGLU && r >= R / 2) ? up : sv;
        loc[r] = locate<TR>(a, v, n < v.rows ? n : 0, c);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) L.w[i][r] = load_whole_chunk(a, loc[r], lane);
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < CPW; ++i) {
    const int c = wave + i * nwaves;
    const bool c_ok = c < a.nchunks;
    const int cc = c_ok ? c : 0;
    const bool lane_ok = (cc * 64 * EPL + lane * EPL) < a.K;
    ChunkLoc loc[R];
    bool rok[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int n = EPI == kSwiGLU ? grp * (R / 2) + (r % (R / 2)) : grp * R + r - sv.row0;
      const SegView v = (EPI == kSwiGLU && r >= R / 2) ? up : sv;
      rok[r] = c_ok && n < v.rows;
      // rows past the end look up row 0 (always valid) and skip their load
      loc[r] = locate<TR>(a, v, rok[r] ? n : 0, cc);
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      L.w[i][r] = rok[r] ? load_chunk(a, loc[r], lane, lane_ok) : u32x4{0u, 0u, 0u, 0u};
  }
}

// Zeros: what a wave's chunk slot past the end of a row loads instead of
// weights, so that every slot is loaded on every path (the activations of
// such a slot are zero as well).  64 KiB, one KiB per workgroup modulo 64,
// so that those reads spread over the L2 channels instead of all waiting
// on the same few lines.
constexpr int kZeroKiB = 64;
__device__ const u32x4 kZeroChunks[kZeroKiB][64] = {};

// The loads of a whole-KiB group in two halves (PART 1 and 2): by chunk slot
// when a wave has several, else by row.  Each accumulator still sums its
// chunk slots in order, so the split leaves every result unchanged.
template <int R, int CPW, int PART>
__device__ constexpr bool in_part(int i, int r) {
  const bool first = CPW >= 2 ? i < CPW / 2 : r < R / 2;
  return PART == 1 ? first : !first;
}

// Issue one half of group `grp` for this wave, with no branch: page
// lookups as one batch of scalar loads, then one 16 B load per lane for
// every slot and row of the half.
template <int PART, int WT, int R, int CPW, int TR, int EPI>
__device__ inline void issue_whole(const GemvArgs& a, int grp, bool live, int wave, int nwaves, int lane,
                                   GroupLoads<WT, R, CPW, TR, EPI>& L) {
  const SegView sv = seg_at(a, EPI == kSwiGLU ? 0 : group_segment<R, EPI>(a, grp));
  const SegView up = seg_at(a, EPI == kSwiGLU ? 1 : 0);
#pragma unroll
  for (int i = 0; i < CPW; ++i) {
    const int c = wave + i * nwaves;
    const bool use = live && c < a.nchunks;   // wave-uniform
    const int cc = c < a.nchunks ? c : 0;
    uint64_t pb[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!in_part<R, CPW, PART>(i, r)) continue;
      const int n = EPI == kSwiGLU ? grp * (R / 2) + (r % (R / 2)) : grp * R + r - sv.row0;
      const SegView v = (EPI == kSwiGLU && r >= R / 2) ? up : sv;
      const ChunkLoc loc = locate<TR>(a, v, n < v.rows ? n : 0, cc);
      pb[r] = uint64_t(a.pool) + uint64_t((loc.p0 << a.log2_page) + loc.inpage);
    }
    // the empty asm keeps every lookup on every path (else the compiler
    // moves them under a branch, and the loads with them)
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (in_part<R, CPW, PART>(i, r)) asm volatile("" : "+s"(pb[r]));
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!in_part<R, CPW, PART>(i, r)) continue;
      const uint64_t base = use ? pb[r] : uint64_t(kZeroChunks[blockIdx.x % kZeroKiB]);
      L.w[i][r] = __builtin_nontemporal_load(
          reinterpret_cast<const __attribute__((address_space(1))) u32x4*>(base + uint64_t(lane) * 16));
    }
  }
}

// Orders the loop body: products before this point stay before it, loads
// after it stay after it, and products after it cannot move above it (the
// accumulators pass through an empty asm statement that also orders memory).
// Returns 1.0 through the same barrier, for the FP8 conversions after it,
// which depend on the weights alone and would otherwise move up.
template <int V>
__device__ inline float order_after(float (&v)[V]) {
#pragma unroll
  for (int j = 0; j < V; ++j) asm volatile("" : "+v"(v[j])::"memory");
  float one = 1.0f;
  asm volatile("" : "+s"(one));
  return one;
}

// Groups a workgroup of the staggered loop holds the outputs of in LDS; the
// launcher sizes the grid so that no workgroup has more.
constexpr int kOutGroups = 32;

// Reduce a group's per-lane partials over the lanes and the waves and
// compute its outputs.  Lane t < R*MT of wave 0 gets output t: its value
// and its element index in y, or -1 where there is none (a row past the
// tensor or a token past the batch).  Per-row scales and the output
// permutation are read with scalar loads, which never wait on the weight
// loads in flight.
template <int WT, int MT, int R, int EPI, int MAXW>
__device__ inline void reduce_group(const GemvArgs& a, int g, int it, float (&v)[R * MT],
                                    float (&red)[2][MAXW][R * MT], int wave, int nwaves, int lane, float& out,
                                    int64_t& at) {
  constexpr int V = R * MT;
  constexpr int LOG2V = Log2<V>::value;
  lane_reduce<V>(v, lane);
  const int buf = it & 1;
  if ((lane & ((64 >> LOG2V) - 1)) == 0) red[buf][wave][lane >> (6 - LOG2V)] = v[0];
  __syncthreads();
  at = -1;
  out = 0.f;
  if (wave != 0) return;
  const int t = lane;
  if constexpr (EPI == kStore) {
    const SegView sv = seg_at(a, group_segment<R, EPI>(a, g));
    float sc[R];
    int col[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int n = g * R + r - sv.row0;
      const int nc = n < sv.rows ? n : 0;
      sc[r] = sv.scale ? ((const float __attribute__((address_space(4)))*)sv.scale)[nc] : 1.0f;
      col[r] = sv.out_off + (sv.out_perm ? ((scalar_i32_ptr)sv.out_perm)[nc] : n);
    }
    if (t < V) {
      float sum = 0.f;
      for (int ww = 0; ww < nwaves; ++ww) sum += red[buf][ww][t];
      const int r = t / MT, m = t % MT;
      float k = sc[0];
      int cl = col[0];
#pragma unroll
      for (int q = 1; q < R; ++q) {
        k = r == q ? sc[q] : k;
        cl = r == q ? col[q] : cl;
      }
      if (sv.scale) sum *= k;
      out = sum;
      if (g * R + r - sv.row0 < sv.rows && m < a.mcount) at = int64_t(a.m0 + m) * a.ldy + cl;
    }
  } else {
    const SegView gv = seg_at(a, 0), uv = seg_at(a, 1);
    float gsc[R / 2], usc[R / 2];
#pragma unroll
    for (int r = 0; r < R / 2; ++r) {
      const int h = g * (R / 2) + r;
      const int hc = h < gv.rows ? h : 0;
      gsc[r] = gv.scale ? ((const float __attribute__((address_space(4)))*)gv.scale)[hc] : 1.0f;
      usc[r] = uv.scale ? ((const float __attribute__((address_space(4)))*)uv.scale)[hc] : 1.0f;
    }
    if (t < V / 2) {
      float gs = 0.f, us = 0.f;
      for (int ww = 0; ww < nwaves; ++ww) {
        gs += red[buf][ww][t];
        us += red[buf][ww][t + V / 2];
      }
      const int r = t / MT, m = t % MT;
      float gk = gsc[0], uk = usc[0];
#pragma unroll
      for (int q = 1; q < R / 2; ++q) {
        gk = r == q ? gsc[q] : gk;
        uk = r == q ? usc[q] : uk;
      }
      if (gv.scale) gs *= gk;
      if (uv.scale) us *= uk;
      out = gs / (1.0f + expf(-gs)) * us;
      const int h = g * (R / 2) + r;
      if (h < gv.rows && m < a.mcount) at = int64_t(a.m0 + m) * a.ldy + h;
    }
  }
}

template <int WT>
__device__ inline void store_out(const GemvArgs& a, int64_t at, float val) {
  if (at < 0) return;
  if constexpr (WT == kF32) {
    static_cast<float*>(a.y)[at] = val;
  } else {
    static_cast<uint16_t*>(a.y)[at] = f32_to_bf16_rne(val);
  }
}

// MAXW: most waves per workgroup (8; 16 for the wide single-token variant)
template <int WT, int MT, int R, int CPW, int TR, int EPI, int MAXW = kMaxWaves>
__global__ __launch_bounds__(MAXW * 64) void gemv_kernel(const GemvArgs a) {
  constexpr int XW = WTraits<WT>::XW;
  constexpr int V = R * MT;
  constexpr int LOG2V = Log2<V>::value;
  // prefetch the next group's weights while reducing the current one when
  // the second register set fits
  constexpr bool PF = CPW * R <= 16;
  static_assert((1 << LOG2V) == V && V <= 64, "R*MT must be a power of two <= 64");
  __shared__ float red[2][MAXW][V];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwaves = blockDim.x >> 6;

  using Loads = GroupLoads<WT, R, CPW, TR, EPI>;
  Loads cur;
  const int grid = int(gridDim.x);

  // BF16 at one token: the first group's weights go out before the
  // activations are gathered, so that their latency overlaps the gather's
  // (through a permutation, two dependent loads): 4096/14336 layer step
  // 79.3 -> 78.3 us.  With more tokens the gather is the larger part, and
  // FP8 q/k/v and o launches lose more than they gain: that order measured
  // slower for both (BF16 4 tokens 86.1 -> 88.0 us; FP8 one-token step
  // 93.5 -> 95.1 us).
  constexpr bool kWeightsFirst = MT == 1 && WT != kFP8;
  if constexpr (kWeightsFirst)
    if (PF && int(blockIdx.x) < a.groups) issue_group<WT, R, CPW, TR, EPI>(a, blockIdx.x, wave, nwaves, lane, cur);

  uint32_t xr[CPW][MT][XW];
#pragma unroll
  for (int i = 0; i < CPW; ++i) {
    const int c = wave + i * nwaves;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      if (c < a.nchunks) {
        load_x<WT>(a, c, m, lane, xr[i][m]);
      } else {
#pragma unroll
        for (int e = 0; e < XW; ++e) xr[i][m][e] = 0u;
      }
    }
  }

  if constexpr (PF && WT == kFP8 && MAXW == kMaxWaves) {
    if ((a.row_bytes & (kChunkBytes - 1)) == 0 && a.groups <= grid * kOutGroups &&
        (MT > 1 || a.groups >= 2 * grid)) {
      // (activations before the weights: loads younger than the loop's
      // own would make the loop's waits count them on every pass)
      // FP8 rows of whole KiB: staggered prefetch.  Each half of the next
      // group is requested as soon as the same half of this group has been
      // used, while the other half is still arriving, so a wave keeps loads
      // in flight through the conversions and products; with a single
      // prefetch it has none from the end of a group's loads until those
      // are done.  The loop body has no branch around a load and no store,
      // so the compiler can wait for exactly the half it needs: the outputs
      // wait in LDS and are stored after the loop.  BF16 rows, whose
      // products are short, measured slower this way, and so did
      // single-token launches with fewer than two groups per workgroup
      // (nothing to overlap) and the 16-wave single-token variant (FP8
      // down, 27 KiB rows: 28.2 -> 27.8 us without): all keep the single
      // prefetch below.
      __shared__ float ov[kOutGroups][V];
      __shared__ int64_t oat[kOutGroups][V];
      // (unconditional, like every load of the loop, so that the count of
      // loads in flight is the same on every path into it)
      issue_whole<1>(a, blockIdx.x, int(blockIdx.x) < a.groups, wave, nwaves, lane, cur);
      issue_whole<2>(a, blockIdx.x, int(blockIdx.x) < a.groups, wave, nwaves, lane, cur);
      // the products of one half of the current group, accumulated into v
      auto dots = [&](auto part, float (&v)[V], float one) {
        constexpr int P = decltype(part)::value;
#pragma unroll
        for (int i = 0; i < CPW; ++i)
#pragma unroll
          for (int r = 0; r < R; ++r)
            if (in_part<R, CPW, P>(i, r))
#pragma unroll
              for (int m = 0; m < MT; ++m)
                v[r * MT + m] = dot_chunk<WT>(cur.w[i][r], xr[i][m], v[r * MT + m], one);
      };
      const std::integral_constant<int, 1> first;
      const std::integral_constant<int, 2> second;
      int it = 0;
      int g = blockIdx.x;
      // every group but the workgroup's last: use it and load the next
      for (; g + grid < a.groups; g += grid, ++it) {
        const int gn = g + grid;
        float v[V];
#pragma unroll
        for (int j = 0; j < V; ++j) v[j] = 0.f;
        dots(first, v, 1.0f);
        order_after(v);
        issue_whole<1>(a, gn, true, wave, nwaves, lane, cur);
        dots(second, v, order_after(v));
        order_after(v);
        issue_whole<2>(a, gn, true, wave, nwaves, lane, cur);
        float out;
        int64_t at;
        reduce_group<WT, MT, R, EPI, MAXW>(a, g, it, v, red, wave, nwaves, lane, out, at);
        if (wave == 0 && lane < V) {
          ov[it][lane] = out;
          oat[it][lane] = at;
        }
      }
      // the last group: nothing more to load
      if (g < a.groups) {
        float v[V];
#pragma unroll
        for (int j = 0; j < V; ++j) v[j] = 0.f;
        dots(first, v, 1.0f);
        dots(second, v, 1.0f);
        float out;
        int64_t at;
        reduce_group<WT, MT, R, EPI, MAXW>(a, g, it, v, red, wave, nwaves, lane, out, at);
        if (wave == 0 && lane < V) {
          ov[it][lane] = out;
          oat[it][lane] = at;
        }
        ++it;
      }
      // each lane reads back only what it wrote: no barrier needed
      if (wave == 0 && lane < V)
        for (int k = 0; k < it; ++k) store_out<WT>(a, oat[k][lane], ov[k][lane]);
      return;
    }
  }

  if constexpr (!kWeightsFirst)
    if (PF && int(blockIdx.x) < a.groups) issue_group<WT, R, CPW, TR, EPI>(a, blockIdx.x, wave, nwaves, lane, cur);
  int it = 0;
  for (int g = blockIdx.x; g < a.groups; g += grid, ++it) {
    if constexpr (!PF) issue_group<WT, R, CPW, TR, EPI>(a, g, wave, nwaves, lane, cur);
    float v[V];
#pragma unroll
    for (int j = 0; j < V; ++j) v[j] = 0.f;
#pragma unroll
    for (int i = 0; i < CPW; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int m = 0; m < MT; ++m) v[r * MT + m] = dot_chunk<WT>(cur.w[i][r], xr[i][m], v[r * MT + m]);
    if constexpr (PF) {
      const int gn = g + grid;
      if (gn < a.groups) issue_group<WT, R, CPW, TR, EPI>(a, gn, wave, nwaves, lane, cur);
    }
    lane_reduce<V>(v, lane);
    const int buf = it & 1;
    if ((lane & ((64 >> LOG2V) - 1)) == 0) red[buf][wave][lane >> (6 - LOG2V)] = v[0];
    __syncthreads();

    const int t = threadIdx.x;
    if constexpr (EPI == kStore) {
      if (t < V) {
        float sum = 0.f;
        for (int ww = 0; ww < nwaves; ++ww) sum += red[buf][ww][t];
        const int r = t / MT, m = t % MT;
        const SegView sv = seg_at(a, group_segment<R, EPI>(a, g));
        const int n = g * R + r - sv.row0;
        if (n < sv.rows && m < a.mcount) {
          if (sv.scale) sum *= sv.scale[n];
          const int col = sv.out_off + (sv.out_perm ? sv.out_perm[n] : n);
          const int64_t idx = int64_t(a.m0 + m) * a.ldy + col;
          if constexpr (WT == kF32) {
            static_cast<float*>(a.y)[idx] = sum;
          } else {
            static_cast<uint16_t*>(a.y)[idx] = f32_to_bf16_rne(sum);
          }
        }
      }
    } else {
      if (t < V / 2) {
        float gs = 0.f, us = 0.f;
        for (int ww = 0; ww < nwaves; ++ww) {
          gs += red[buf][ww][t];
          us += red[buf][ww][t + V / 2];
        }
        const int r = t / MT, m = t % MT;
        const int h = g * (R / 2) + r;
        if (h < a.seg[0].rows && m < a.mcount) {
          if (a.seg[0].scale) gs *= a.seg[0].scale[h];
          if (a.seg[1].scale) us *= a.seg[1].scale[h];
          const float hv = gs / (1.0f + expf(-gs)) * us;
          const int64_t idx = int64_t(a.m0 + m) * a.ldy + h;
          if constexpr (WT == kF32) {
            static_cast<float*>(a.y)[idx] = hv;
          } else {
            static_cast<uint16_t*>(a.y)[idx] = f32_to_bf16_rne(hv);
          }
        }
      }
    }
  }
}

using KernelFn = void (*)(const GemvArgs);

// Largest token tile that keeps a wave's activations (CPW * MT * XW words)
// in registers without spilling at 256 VGPRs.
int max_mtile(int wt, int cpw) {
  if (wt == kFP8) return cpw <= 1 ? 8 : cpw == 2 ? 4 : cpw == 4 ? 2 : 1;
  return cpw <= 2 ? 8 : cpw == 4 ? 4 : 2;
}

// Rows per group: 8, or 4 for rows of more than 16 KiB (4+ chunks per wave),
// where 4 rows keep the next-group prefetch within the register budget.
constexpr int rows_for(int cpw) { return cpw >= 4 ? 4 : 8; }

// Single-token launches over rows of 17..32 chunks (e.g. a 14336-wide down
// projection) use up to 16 waves of 2 chunks and 4 rows each: twice the
// waves of the 8-wave layout with the same bytes in flight per wave, which
// keeps more loads outstanding per CU (the kernel then fits in 128 VGPRs).
constexpr int kWideWaves = 16;
constexpr int kWideCpw = 2, kWideRows = 4;
bool use_wide(int nchunks, int mtile) {
  return mtile == 1 && nchunks > 2 * kMaxWaves && nchunks <= kWideCpw * kWideWaves;
}

template <int WT, int CPW, int TR, int EPI>
KernelFn pick_mt(int mt) {
  constexpr int kMax = WT == kFP8 ? (CPW <= 1 ? 8 : CPW == 2 ? 4 : CPW == 4 ? 2 : 1)
                                  : (CPW <= 2 ? 8 : CPW == 4 ? 4 : 2);
  constexpr int R = rows_for(CPW);
  if (mt <= 1) return gemv_kernel<WT, 1, R, CPW, TR, EPI>;
  if (mt <= 2 || kMax == 2) return gemv_kernel<WT, (kMax < 2 ? 1 : 2), R, CPW, TR, EPI>;
  if (mt <= 4 || kMax == 4) return gemv_kernel<WT, (kMax < 4 ? 1 : 4), R, CPW, TR, EPI>;
  return gemv_kernel<WT, (kMax < 8 ? 1 : 8), R, CPW, TR, EPI>;
}

template <int WT, int TR, int EPI>
KernelFn pick_cpw(int cpw, int mt) {
  switch (cpw) {
    case 1: return pick_mt<WT, 1, TR, EPI>(mt);
    case 2: return pick_mt<WT, 2, TR, EPI>(mt);
    case 4: return pick_mt<WT, 4, TR, EPI>(mt);
    default: return pick_mt<WT, 8, TR, EPI>(mt);
  }
}

template <int WT, int EPI>
KernelFn pick_tr(int tr, int cpw, int mt) {
  return tr == 2 ? pick_cpw<WT, 2, EPI>(cpw, mt) : tr == 1 ? pick_cpw<WT, 1, EPI>(cpw, mt)
                                                 : pick_cpw<WT, 0, EPI>(cpw, mt);
}

KernelFn pick(int wt, int tr, int cpw, int mt, int epi) {
  if (epi == kSwiGLU) {
    if (wt == kF32) return pick_tr<kF32, kSwiGLU>(tr, cpw, mt);
    if (wt == kBF16) return pick_tr<kBF16, kSwiGLU>(tr, cpw, mt);
    return pick_tr<kFP8, kSwiGLU>(tr, cpw, mt);
  }
  if (wt == kF32) return pick_tr<kF32, kStore>(tr, cpw, mt);
  if (wt == kBF16) return pick_tr<kBF16, kStore>(tr, cpw, mt);
  return pick_tr<kFP8, kStore>(tr, cpw, mt);
}

template <int WT, int EPI>
KernelFn pick_wide_tr(int tr) {
  return tr == 2   ? gemv_kernel<WT, 1, kWideRows, kWideCpw, 2, EPI, kWideWaves>
         : tr == 1 ? gemv_kernel<WT, 1, kWideRows, kWideCpw, 1, EPI, kWideWaves>
                   : gemv_kernel<WT, 1, kWideRows, kWideCpw, 0, EPI, kWideWaves>;
}

KernelFn pick_wide(int wt, int tr, int epi) {
  if (epi == kSwiGLU) {
    if (wt == kF32) return pick_wide_tr<kF32, kSwiGLU>(tr);
    if (wt == kBF16) return pick_wide_tr<kBF16, kSwiGLU>(tr);
    return pick_wide_tr<kFP8, kSwiGLU>(tr);
  }
  if (wt == kF32) return pick_wide_tr<kF32, kStore>(tr);
  if (wt == kBF16) return pick_wide_tr<kBF16, kStore>(tr);
  return pick_wide_tr<kFP8, kStore>(tr);
}

int resident_blocks(KernelFn fn, int threads) {
  static std::mutex mu;
  static std::map<std::tuple<int, void*, int>, int> cache;   // (device, kernel, threads)
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(dev, reinterpret_cast<void*>(fn), threads);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn), threads, 0) !=
      hipSuccess)
    return 0;
  const int n = cus * (per_cu > 0 ? per_cu : 1);
  cache[key] = n;
  return n;
}

// ------------------------------------------------------------------ MoE experts
// A mixture-of-experts layer over cloaked expert tensors.  The route kernel
// sorts the call's (token, slot) pairs by (expert, pair) and cuts the sorted
// list into one run per active expert; the SwiGLU and down kernels give every
// active expert a column of workgroups whose waves each stream a few rows of
// that expert once per MT of its tokens, translating pages per 1 KiB chunk
// like the GEMV; the combine kernel adds each token's weighted slot results
// in slot order.  Every result bit is independent of scheduling.

constexpr int kMoeWaves = 4;
constexpr int kMoeUnits = 2;      // hidden units (gate + up rows) per wave of the SwiGLU kernel
constexpr int kMoeDownRows = 8;   // down rows per wave (down rows are d_ffn long, usually short)
constexpr int kMoeLoads = 16;     // 16 B loads per lane issued together (rows x 1 KiB chunks)
constexpr int kMoeRouteThreads = 1024;
constexpr int kMoePairBits = 12;  // pair index < 4096 in the sort key

// Calls of at most 64 pairs: one wave sorts the keys in registers (bitonic
// network over lanes), finds the runs with a ballot and writes the same
// tables as the workgroup version below.
__global__ __launch_bounds__(64) void moe_route_wave_kernel(const MoeArgs a) {
  const int n = a.M * a.topk;
  const int l = threadIdx.x;
  int32_t key = INT32_MAX;
  if (l < n) {
    int e = a.ids[l];
    if (e < 0 || e >= a.E) e = a.E;
    key = (e << kMoePairBits) | l;
  }
  for (int k = 2; k <= 64; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int32_t p = __shfl_xor(key, j);
      const bool lower = (l & j) == 0, asc = (l & k) == 0;
      key = (lower == asc) ? min(key, p) : max(key, p);
    }
  }
  const int e = key >> kMoePairBits;
  const bool valid = e < a.E;
  const int32_t prev = __shfl_up(key, 1);
  const bool opens = valid && (l == 0 || (prev >> kMoePairBits) != e);
  const unsigned long long runs = __ballot(opens);
  const int n_valid = __popcll(__ballot(valid));
  int32_t* act_expert = a.route + 1;
  int32_t* act_start = act_expert + a.E;
  int32_t* act_count = act_start + a.E;
  int32_t* ent = act_count + a.E;
  if (valid) ent[l] = key & ((1 << kMoePairBits) - 1);
  if (opens) {
    const int slot = __popcll(runs & ((1ull << l) - 1));
    const unsigned long long later = l < 63 ? runs & ~((2ull << l) - 1) : 0ull;
    const int end = later ? __ffsll((long long)later) - 1 : n_valid;
    act_expert[slot] = e;
    act_start[slot] = l;
    act_count[slot] = end - l;
  }
  if (l == 0) a.route[0] = __popcll(runs);
}

__global__ __launch_bounds__(kMoeRouteThreads) void moe_route_kernel(const MoeArgs a) {
  extern __shared__ int32_t sh[];
  const int n = a.M * a.topk;
  int N2 = 1;
  while (N2 < n) N2 <<= 1;
  int32_t* keys = sh;                       // [N2] (expert << 12) | pair, invalid experts sort last
  int32_t* part = sh + N2;                  // [threads] run counts, then their inclusive scan
  int32_t* sstart = part + kMoeRouteThreads;  // [min(E, n)] start of each active expert's run
  __shared__ int32_t n_valid;
  const int T = blockDim.x, t = threadIdx.x;
  if (t == 0) n_valid = 0;
  for (int i = t; i < N2; i += T) {
    int32_t key = INT32_MAX;
    if (i < n) {
      int e = a.ids[i];
      if (e < 0 || e >= a.E) e = a.E;
      key = (e << kMoePairBits) | i;
    }
    keys[i] = key;
  }
  __syncthreads();
  for (int k = 2; k <= N2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = t; i < N2; i += T) {
        const int l = i ^ j;
        if (l > i) {
          const int32_t x = keys[i], y = keys[l];
          if ((x > y) == ((i & k) == 0)) {
            keys[i] = y;
            keys[l] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  // runs: position p opens one when its expert differs from position p-1's
  const int per = (n + T - 1) / T;
  const int lo = t * per, hi = min(n, lo + per);
  int runs = 0, valid = 0;
  for (int p = lo; p < hi; ++p) {
    const int e = keys[p] >> kMoePairBits;
    if (e < a.E) {
      ++valid;
      if (p == 0 || (keys[p - 1] >> kMoePairBits) != e) ++runs;
    }
  }
  part[t] = runs;
  atomicAdd(&n_valid, valid);   // an integer sum: any order gives the same value
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t* act_expert = a.route + 1;
  int32_t* act_start = act_expert + a.E;
  int32_t* act_count = act_start + a.E;
  int32_t* ent = act_count + a.E;
  int s = part[t] - runs;
  for (int p = lo; p < hi; ++p) {
    const int e = keys[p] >> kMoePairBits;
    if (e >= a.E) break;
    ent[p] = keys[p] & ((1 << kMoePairBits) - 1);
    if (p == 0 || (keys[p - 1] >> kMoePairBits) != e) {
      act_expert[s] = e;
      act_start[s] = p;
      sstart[s] = p;
      ++s;
    }
  }
  __syncthreads();
  const int na = part[T - 1];
  for (int r = t; r < na; r += T) act_count[r] = (r + 1 < na ? sstart[r + 1] : n_valid) - sstart[r];
  if (t == 0) a.route[0] = na;
}

// Active slot s of a call: its expert, first sorted entry and pair count.
// Single-token calls skip routing: slot j is pair j of expert ids[j] (a slot
// naming no expert returns false and is skipped).
__device__ inline bool moe_slot(const MoeArgs& a, int s, int& e, int& st, int& cnt) {
  if (a.direct) {
    if (s >= a.topk) return false;
    e = a.ids[s];
    st = s;
    cnt = 1;
    return e >= 0 && e < a.E;
  }
  if (s >= a.route[0]) return false;
  e = a.route[1 + s];
  st = a.route[1 + a.E + s];
  cnt = a.route[1 + 2 * a.E + s];
  return true;
}

// Pair of sorted entry i (the identity in single-token calls).
__device__ inline int moe_entry(const MoeArgs& a, int i) { return a.direct ? i : a.route[1 + 3 * a.E + i]; }

// This lane's 16 B of chunk c of row `row` of a tensor (zero past the row).
template <int TR>
__device__ inline u32x4 moe_load(const MoeArgs& a, int64_t vbase, int64_t npages, int64_t row, int64_t row_bytes,
                                 int c, int lane, bool ok) {
  const int64_t o = row * row_bytes + int64_t(c) * kChunkBytes;
  const int64_t page_bytes = int64_t(1) << a.log2_page;
  const int64_t vp = o >> a.log2_page;
  const int64_t inpage = o & (page_bytes - 1);
  const int64_t vpage = vbase + vp;
  const int64_t vnext = vp + 1 < npages ? vpage + 1 : vpage;
  const int64_t p0 = TR ? page_of<TR == 2>(a.phi, a.phi_key, vpage) : vpage;
  const int64_t p1 = TR ? page_of<TR == 2>(a.phi, a.phi_key, vnext) : vnext;
  const int64_t lo = inpage + int64_t(lane) * 16;
  const bool second = lo >= page_bytes;
  const uint8_t* addr = a.pool + ((second ? p1 : p0) << a.log2_page) + (second ? lo - page_bytes : lo);
  u32x4 w = {0u, 0u, 0u, 0u};
  if (ok) w = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(addr));
  return w;
}

// bf16 activations matching this lane's weight elements of chunk c.
template <int WT>
__device__ inline void moe_x(const uint16_t* row, int K, int c, int lane, bool ok, uint32_t (&xr)[WTraits<WT>::XW]) {
  constexpr int EPL = WTraits<WT>::EPL;
  const int k0 = c * 64 * EPL + lane * EPL;
#pragma unroll
  for (int q = 0; q < WTraits<WT>::XW / 4; ++q) {
    u32x4 v = {0u, 0u, 0u, 0u};
    if (ok && k0 < K) v = *reinterpret_cast<const u32x4*>(row + k0 + q * 8);
    xr[4 * q] = v.x;
    xr[4 * q + 1] = v.y;
    xr[4 * q + 2] = v.z;
    xr[4 * q + 3] = v.w;
  }
}

// NR rows of one expert tensor set (gate and up, or down) times MT tokens:
// per-lane partial sums in v[r * MT + m].  Rows are (tensor ti[r], row rr[r]).
template <int WT, int TR, int NR, int MT>
__device__ inline void moe_rows(const MoeArgs& a, const MoeExpert& ex, const int (&ti)[NR], const int (&rr)[NR],
                                const bool (&rok)[NR], int64_t row_bytes, const uint16_t* xbase, int K,
                                const int (&xrow)[MT], int lane, float (&v)[NR * MT]) {
  constexpr int XW = WTraits<WT>::XW;
  constexpr int CH = kMoeLoads / NR > 0 ? kMoeLoads / NR : 1;   // chunks per pass
  const int nch = int((row_bytes + kChunkBytes - 1) / kChunkBytes);
  for (int c0 = 0; c0 < nch; c0 += CH) {
    u32x4 w[CH][NR];
#pragma unroll
    for (int cc = 0; cc < CH; ++cc) {
      const int c = c0 + cc;
      const bool ok = c < nch && int64_t(c) * kChunkBytes + int64_t(lane) * 16 < row_bytes;
#pragma unroll
      for (int r = 0; r < NR; ++r)
        w[cc][r] = moe_load<TR>(a, ex.vbase[ti[r]], ex.npages[ti[r]], rok[r] ? rr[r] : 0, row_bytes,
                                c < nch ? c : 0, lane, ok && rok[r]);
    }
#pragma unroll
    for (int cc = 0; cc < CH; ++cc) {
      const int c = c0 + cc;
      if (c >= nch) break;
      const bool ok = int64_t(c) * kChunkBytes + int64_t(lane) * 16 < row_bytes;
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        uint32_t xr[XW];
        moe_x<WT>(xbase + int64_t(xrow[m] < 0 ? 0 : xrow[m]) * K, K, c, lane, ok && xrow[m] >= 0, xr);
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r * MT + m] = dot_chunk<WT>(w[cc][r], xr, v[r * MT + m]);
      }
    }
  }
}

template <int WT, int TR, int MT>
__global__ __launch_bounds__(kMoeWaves * 64) void moe_swiglu_kernel(const MoeArgs a) {
  constexpr int NR = 2 * kMoeUnits;
  constexpr int V = NR * MT;
  constexpr int STRIDE = 64 / V;   // value j of the reduction sits in lane j * STRIDE; up values 32 lanes on
  int e, st, cnt;
  if (!moe_slot(a, blockIdx.x, e, st, cnt)) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int unit0 = (int(blockIdx.y) * kMoeWaves + wave) * kMoeUnits;
  if (unit0 >= a.d_ffn) return;
  const MoeExpert ex = a.experts[e];
  const int64_t row_bytes = int64_t(a.d_model) * (WT == kFP8 ? 1 : 2);
  int ti[NR], rr[NR];
  bool rok[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    ti[r] = r / kMoeUnits;
    rr[r] = unit0 + r % kMoeUnits;
    rok[r] = rr[r] < a.d_ffn;
  }
  for (int t0 = 0; t0 < cnt; t0 += MT) {
    int pair[MT], xrow[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      pair[m] = t0 + m < cnt ? moe_entry(a, st + t0 + m) : -1;
      xrow[m] = pair[m] < 0 ? -1 : pair[m] / a.topk;
    }
    float v[V];
#pragma unroll
    for (int j = 0; j < V; ++j) v[j] = 0.f;
    moe_rows<WT, TR, NR, MT>(a, ex, ti, rr, rok, row_bytes, a.x, a.d_model, xrow, lane, v);
    lane_reduce<V>(v, lane);
    const float mine = v[0];
    const float upv = __shfl(mine, (lane + 32) & 63);
    if (lane < 32 && lane % STRIDE == 0) {
      const int j = lane / STRIDE;
      const int u = unit0 + j / MT, m = j % MT;
      if (u < a.d_ffn && pair[m] >= 0) {
        float gs = mine, us = upv;
        if (ex.scale_off[0] >= 0) gs *= a.scales[ex.scale_off[0] + u];
        if (ex.scale_off[1] >= 0) us *= a.scales[ex.scale_off[1] + u];
        a.h[int64_t(pair[m]) * a.d_ffn + u] = f32_to_bf16_rne(gs / (1.0f + expf(-gs)) * us);
      }
    }
  }
}

template <int WT, int TR, int MT>
__global__ __launch_bounds__(kMoeWaves * 64) void moe_down_kernel(const MoeArgs a) {
  constexpr int NR = kMoeDownRows;
  constexpr int V = NR * MT;
  constexpr int STRIDE = 64 / V;
  int e, st, cnt;
  if (!moe_slot(a, blockIdx.x, e, st, cnt)) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int row0 = (int(blockIdx.y) * kMoeWaves + wave) * kMoeDownRows;
  if (row0 >= a.d_model) return;
  const MoeExpert ex = a.experts[e];
  const int64_t row_bytes = int64_t(a.d_ffn) * (WT == kFP8 ? 1 : 2);
  int ti[NR], rr[NR];
  bool rok[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    ti[r] = 2;
    rr[r] = row0 + r;
    rok[r] = rr[r] < a.d_model;
  }
  for (int t0 = 0; t0 < cnt; t0 += MT) {
    int pair[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) pair[m] = t0 + m < cnt ? moe_entry(a, st + t0 + m) : -1;
    float v[V];
#pragma unroll
    for (int j = 0; j < V; ++j) v[j] = 0.f;
    moe_rows<WT, TR, NR, MT>(a, ex, ti, rr, rok, row_bytes, a.h, a.d_ffn, pair, lane, v);
    lane_reduce<V>(v, lane);
    if (lane % STRIDE == 0) {
      const int j = lane / STRIDE;
      const int n = row0 + j / MT, m = j % MT;
      if (n < a.d_model && pair[m] >= 0) {
        float acc = v[0];
        if (ex.scale_off[2] >= 0) acc *= a.scales[ex.scale_off[2] + n];
        a.yp[int64_t(pair[m]) * a.d_model + n] = acc * a.wts[pair[m]];
      }
    }
  }
}

// One thread per 4 outputs of a token: the weighted slot results in slot order.
__global__ __launch_bounds__(256) void moe_combine_kernel(const MoeArgs a) {
  const int m = blockIdx.x;
  const int n0 = (int(blockIdx.y) * 256 + int(threadIdx.x)) * 4;
  if (n0 >= a.d_model) return;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 8
  for (int j = 0; j < a.topk; ++j) {
    const int pi = m * a.topk + j;
    const int e = a.ids[pi];
    if (e >= 0 && e < a.E) {
      const float4 p = *reinterpret_cast<const float4*>(a.yp + int64_t(pi) * a.d_model + n0);
      acc.x += p.x;
      acc.y += p.y;
      acc.z += p.z;
      acc.w += p.w;
    }
  }
  const uint32_t lo = uint32_t(f32_to_bf16_rne(acc.x)) | (uint32_t(f32_to_bf16_rne(acc.y)) << 16);
  const uint32_t hi = uint32_t(f32_to_bf16_rne(acc.z)) | (uint32_t(f32_to_bf16_rne(acc.w)) << 16);
  *reinterpret_cast<uint2*>(a.y + int64_t(m) * a.d_model + n0) = make_uint2(lo, hi);
}

using MoeFn = void (*)(const MoeArgs);

template <int WT, int TR>
void pick_moe_mt(int mt, MoeFn& sw, MoeFn& dn) {
  if (mt <= 1) {
    sw = moe_swiglu_kernel<WT, TR, 1>;
    dn = moe_down_kernel<WT, TR, 1>;
  } else if (mt <= 2) {
    sw = moe_swiglu_kernel<WT, TR, 2>;
    dn = moe_down_kernel<WT, TR, 2>;
  } else if (mt <= 4) {
    sw = moe_swiglu_kernel<WT, TR, 4>;
    dn = moe_down_kernel<WT, TR, 4>;
  } else {
    sw = moe_swiglu_kernel<WT, TR, 8>;
    dn = moe_down_kernel<WT, TR, 8>;
  }
}

template <int WT>
void pick_moe(int tr, int mt, MoeFn& sw, MoeFn& dn) {
  if (tr == 2)
    pick_moe_mt<WT, 2>(mt, sw, dn);
  else if (tr == 1)
    pick_moe_mt<WT, 1>(mt, sw, dn);
  else
    pick_moe_mt<WT, 0>(mt, sw, dn);
}

}  // namespace

int gemv_cpw(int nchunks) {
  int cpw = 1;
  while ((nchunks + cpw - 1) / cpw > kMaxWaves) cpw *= 2;
  return cpw;
}

int gemv_max_tokens(int wtype, int nchunks) { return max_mtile(wtype, gemv_cpw(nchunks)); }

int gemv_rows(int nchunks, int mtile) { return use_wide(nchunks, mtile) ? kWideRows : rows_for(gemv_cpw(nchunks)); }

hipError_t launch_gemv(const GemvArgs& a, int wtype, int mtile, bool translate, hipStream_t s) {
  // masked maps get their own instantiation, so plain maps pay nothing for them
  const int tr = translate ? (a.phi_key ? 2 : 1) : 0;
  if (a.groups <= 0) return hipSuccess;
  const bool wide = use_wide(a.nchunks, mtile);
  int cpw = wide ? kWideCpw : gemv_cpw(a.nchunks);
  // FP8 rows of 2..8 KiB at one token over many rows (gate/up, fused q/k/v):
  // two chunks per wave keep twice the loads in flight per wave, with half
  // the waves to reduce over (measured: SwiGLU 5120 -> 2 x 27648 from 69.7
  // to 62.0 us; the 5120-row o projection is better with one chunk)
  if (wtype == kFP8 && mtile == 1 && a.nchunks > 1 && a.nchunks <= kMaxWaves &&
      int64_t(a.groups) * rows_for(1) >= 6144)
    cpw = 2;
  if (cpw > 8 || mtile > max_mtile(wtype, cpw) || a.mcount > mtile) return hipErrorInvalidValue;
  const int waves = (a.nchunks + cpw - 1) / cpw;
  const int threads = waves * 64;
  KernelFn fn = wide ? pick_wide(wtype, tr, a.mode) : pick(wtype, tr, cpw, mtile, a.mode);
  int blocks = resident_blocks(fn, threads);
  if (blocks <= 0) blocks = a.groups;
  // the staggered loop holds at most kOutGroups groups' outputs per workgroup
  blocks = std::max(blocks, (a.groups + kOutGroups - 1) / kOutGroups);
  if (blocks > a.groups) blocks = a.groups;
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(threads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_moe(const MoeArgs& a, bool translate, hipStream_t s) {
  const int n = a.M * a.topk;
  if (n <= 0) return hipSuccess;
  if (n > (1 << kMoePairBits) || a.E >= (1 << (31 - kMoePairBits)) || a.d_model % 4 != 0)
    return hipErrorInvalidValue;
  const int tr = translate ? (a.phi_key ? 2 : 1) : 0;
  // token tile from the pairs an active expert averages: every extra pass
  // re-streams the expert's rows (measured on 128 experts of 2048/768: 4-token
  // tiles beat 2-token tiles from 2 pairs per expert, 8-token tiles beat two
  // 4-token passes at 16)
  const int per_expert = (n + a.E - 1) / a.E;
  const int mt = a.M == 1 ? 1 : per_expert <= 1 ? 2 : per_expert <= 4 ? 4 : 8;
  MoeFn sw, dn;
  if (a.wtype == kFP8)
    pick_moe<kFP8>(tr, mt, sw, dn);
  else
    pick_moe<kBF16>(tr, mt, sw, dn);
  int n2 = 1;
  while (n2 < n) n2 <<= 1;
  const unsigned slots = unsigned(n < a.E ? n : a.E);
  const size_t route_lds = size_t(n2 + kMoeRouteThreads + slots) * 4;
  if (a.M == 1 && a.topk <= 64) {
    // one token: each slot is its own expert pass, no routing kernel (results are the same:
    // a one-token pass does not depend on where its pair sits in a sorted list)
    MoeArgs d = a;
    d.direct = 1;
    const unsigned per_sw = kMoeWaves * kMoeUnits, per_dn = kMoeWaves * kMoeDownRows;
    hipLaunchKernelGGL(sw, dim3(unsigned(a.topk), unsigned((a.d_ffn + per_sw - 1) / per_sw)), dim3(kMoeWaves * 64),
                       0, s, d);
    hipLaunchKernelGGL(dn, dim3(unsigned(a.topk), unsigned((a.d_model + per_dn - 1) / per_dn)),
                       dim3(kMoeWaves * 64), 0, s, d);
    hipLaunchKernelGGL(moe_combine_kernel, dim3(1u, unsigned((a.d_model + 1023) / 1024)), dim3(256), 0, s, d);
    return hipGetLastError();
  }
  if (n <= 64)
    hipLaunchKernelGGL(moe_route_wave_kernel, dim3(1), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(moe_route_kernel, dim3(1), dim3(kMoeRouteThreads), route_lds, s, a);
  if (per_expert >= 2 && a.d_model % 64 == 0 && a.d_ffn % 64 == 0) {
    // experts averaging 2+ tokens: token tiles on MFMA stream each expert's rows once per 32 tokens
    // (measured on 128 experts of 2048/768: 264 us per layer at 256 tokens against 996 on the VALU
    // kernels, 2+ tokens per expert being where the VALU passes start to re-stream rows)
    if (hipError_t e = launch_moe_mfma(a, translate, s)) return e;
  } else {
    const unsigned per_sw = kMoeWaves * kMoeUnits, per_dn = kMoeWaves * kMoeDownRows;
    hipLaunchKernelGGL(sw, dim3(slots, unsigned((a.d_ffn + per_sw - 1) / per_sw)), dim3(kMoeWaves * 64), 0, s, a);
    hipLaunchKernelGGL(dn, dim3(slots, unsigned((a.d_model + per_dn - 1) / per_dn)), dim3(kMoeWaves * 64), 0, s,
                       a);
  }
  hipLaunchKernelGGL(moe_combine_kernel, dim3(unsigned(a.M), unsigned((a.d_model + 1023) / 1024)), dim3(256), 0, s,
                     a);
  return hipGetLastError();
}

}  // namespace cloak

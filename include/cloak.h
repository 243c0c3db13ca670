/*
 * cloak.h -- C-ABI of libcloak, the MI355X (gfx950) cloaked linear layer.
 *
 * CloakLM (arXiv 2606.18400) hides where model weights sit in accelerator
 * memory: tensors are placed in a seeded random order (inter-layer shuffle,
 * Section 4.2 and Table 1a), each FFN's hidden neurons are permuted
 * (intra-layer shuffle, named in the abstract; optionally the attention
 * heads too), and the resulting byte
 * streams are cut into pages scattered over a pool through a seeded
 * virtual->physical page map that is re-randomised periodically (Section 4.2,
 * paragraph on physical page remapping; Table 1b).  All randomness is drawn from one seed
 * before any weight is transferred (Section 5, Implementation Details).
 *
 * In this library the page map is resolved in software, inside the kernels
 * that stream the weights (GEMV, GEMM, fused SwiGLU FFN), and the remap is a
 * device kernel that swaps page pairs in place.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Weights are nn.Linear arrays W[N][K] (row n = output channel n, K
 *   contiguous); y[M][N] = x[M][K] . W^T.  Activations x and results y are
 *   row-major with leading dimension K (resp. the output width).
 * - Element types: CLOAK_F32 weights take f32 activations and give f32
 *   results; CLOAK_BF16 and CLOAK_FP8_E4M3 weights take bf16 activations and
 *   give bf16 results (rounded to nearest even).  FP8 weights carry one f32
 *   scale per output row: W[n][k] = e4m3(q[n][k]) * s[n] (OCP E4M3, max 448).
 *   Accumulation is always f32.
 * - Pointers named h_* are host memory, d_* device memory of the device that
 *   cloak_layout_to_device() was called on.  `stream` is a hipStream_t passed
 *   as void* (NULL = the null stream).
 * - Ownership: the caller owns every large device buffer (the pool, x, y,
 *   workspaces).  The library owns the layout and its small device tables
 *   (page map, hidden permutations, FP8 scales), freed by cloak_layout_free().
 * - Errors: every int-returning call returns CLOAK_OK (0) or a negative
 *   cloak_status; arguments are checked before anything is launched, no call
 *   aborts, and cloak_last_error() gives a message for the calling thread.
 * - Asynchrony: device calls enqueue on `stream` and return; only
 *   cloak_load() and cloak_unload() synchronise (they stage host memory).
 *   Read-only calls may run concurrently on several streams; cloak_remap()
 *   moves pages, so the caller must order it after every kernel that reads
 *   the pool and before every later one (the paper's synchronisation point).
 *
 * Layout definition (every library and oracle implementation follows this)
 * ----------------------------------------------------------------------
 * Generator: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014).  Sub-stream for
 * (seed, tag, idx) starts from mix64(seed ^ mix64((tag << 32) | idx)).  Tags:
 * 1 tensor order, 2 hidden permutation of layer idx, 3 page map, 4 upload
 * order of tensor idx, 5 remap matching (keyed by the remap seed), 6 attention
 * heads of layer idx.
 * With CLOAK_CSPRNG, word j of sub-stream (seed, tag, idx) is instead bytes
 * 8(j%4) .. 8(j%4)+7, little-endian, of SHA-256(seed_le64 || tag_le32 ||
 * idx_le32 || (j/4)_le64) (FIPS 180-4), which reveals neither the seed nor
 * other words.
 * bounded(n) rejects the (2^64 mod n) lowest outputs and returns r mod n;
 * permutations are Fisher-Yates (Durstenfeld), i from n-1 down to 1 swapping
 * a[i] with a[bounded(i+1)]; gather convention (slot j holds a[j]).
 *   sigma   = FY(T, tag 1)           tensor sigma[i] is i-th in the page stream
 *   pi_l    = FY(d_ffn, tag 2, l)    gate_s[j] = gate[pi[j]], up_s[j] = up[pi[j]],
 *                                    down_s[:, j] = down[:, pi[j]]
 *   heads_l (only for a layer whose q/k/v/o give head_dim = hd > 0; Hq = q.N/hd,
 *           Hkv = k.N/hd, G = Hq/Hkv) one stream g = sub-stream(tag 6, l) draws
 *           rho = FY(Hkv, g), then theta_c = FY(G, g) for c = 0..Hkv-1, then
 *           chi = FY(hd, g).  Stored kv head c holds logical head rho[c];
 *           stored query head c*G+i holds logical head rho[c]*G + theta_c[i];
 *           value dimension d of a head holds logical dimension chi[d]:
 *             q_s[(c*G+i)*hd + d]    = q[(rho[c]*G + theta_c[i])*hd + d]
 *             k_s[c*hd + d]          = k[rho[c]*hd + d]
 *             v_s[c*hd + d]          = v[rho[c]*hd + chi[d]]
 *             o_s[:, (c*G+i)*hd + d] = o[:, (rho[c]*G + theta_c[i])*hd + chi[d]]
 *           Attention over the stored heads (query head h reads kv head h/G)
 *           followed by o_s computes the logical layer exactly (rotary
 *           dimensions are not moved).
 *   vbase   each tensor starts on a fresh virtual page, tensors in sigma order,
 *           npages = ceil(N*K*elt / page_bytes), zero padded
 *   phi     = FY(P, tag 3) over all P = pool_bytes/page_bytes pages; virtual
 *           page v lives at physical page phi[v]; pages V..P-1 are free
 *   remap   s = FY(P, tag 5, idx 0); pair (s[2i], s[2i+1]); each pair swaps
 *           contents; phi' = tau o phi
 *   uniform remap (CLOAK_REMAP_UNIFORM) rho = FY(P, tag 5, idx 1); the contents
 *           of physical page p move to rho[p]; phi' = rho o phi.  In place as
 *           two passes of disjoint swaps: for each cycle c_0 -> c_1 -> ... of
 *           rho (c_0 its smallest page, c_{i+1} = rho[c_i], length k), pass 1
 *           swaps c_i with c_{k-i} (0 < i < k-i), pass 2 swaps c_0 with c_1
 *           and c_i with c_{k+1-i} (2 <= i, 2i < k+1); each pass in ascending
 *           order of its pairs' lower page
 *   masked map (CLOAK_MASKED_MAP) the k-th upload of the device page map uses
 *           key_k = the k-th nonzero word of the counter-mode SHA-256 stream
 *           (seed, tag 8, idx 0) and stores entry v as phi[v] XOR m_k(v): with
 *           k0 / k1 the low / high 32 bits of key_k (k1 | 1), h = v ^ k0,
 *           h = (h ^ h>>16) * k1, h = (h ^ h>>15) * 0x2C1B3C6D,
 *           m_k(v) = (h ^ h>>16) ^ k0 (32-bit arithmetic; obfuscation, not a cipher).
 *   decoys  (optional, cloak_pool_decoy) free virtual page v in [V, P) takes the
 *           stream w = sub-stream(decoy_seed, tag 7, v); element e of the page uses
 *           outputs 3e, 3e+1, 3e+2 of w; S = sum of their twelve 16-bit pieces,
 *           C = 2S - 786420.  f32/bf16 decoys: C*5 * 2^-25 (bf16 nearest even);
 *           fp8 decoys: E4M3(C*3 * 2^-12), nearest even, saturating at 448.  Element
 *           type: the dtype holding the most tensor bytes (ties fp8, bf16, f32; bf16
 *           without tensors).  decoy_seed must not be derived from the layout seed:
 *           SplitMix64 is invertible, so decoy bytes would reveal it.
 */
#ifndef CLOAK_H
#define CLOAK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cloak_layout cloak_layout; /* opaque, owned by the library */

typedef enum {
  CLOAK_OK = 0,
  CLOAK_EINVAL = -1, /* bad argument (null pointer, out-of-range index, bad size) */
  CLOAK_ENOMEM = -2, /* pool too small for the layout, or host/device allocation failed */
  CLOAK_EHIP = -3,   /* a HIP runtime call failed; cloak_last_error() has its message */
  CLOAK_ESHAPE = -4, /* shapes inconsistent (duplicate tensor, hidden sizes disagree, K mismatch) */
  CLOAK_EDTYPE = -5, /* dtype not supported by this call */
  CLOAK_ESTATE = -6  /* call not valid in the layout's state (no device tables, native layout) */
} cloak_status;

typedef enum { CLOAK_F32 = 0, CLOAK_BF16 = 1, CLOAK_FP8_E4M3 = 2 } cloak_dtype;

typedef enum {
  CLOAK_Q = 0, CLOAK_K = 1, CLOAK_V = 2, CLOAK_O = 3,
  CLOAK_GATE = 4, CLOAK_UP = 5, CLOAK_DOWN = 6,
  CLOAK_EMBED = 7, CLOAK_HEAD = 8
} cloak_kind;

/* One weight tensor, nn.Linear orientation: n_out rows of k_in elements.
 * `layer` groups gate/up/down under one hidden permutation (any value fits in
 * 32 bits; embed/head conventionally use -1) and q/k/v/o under one head
 * permutation.  `head_dim` > 0 on q, k, v and o of a layer (all four, same
 * value, layer >= 0) asks for that layer's attention-head permutation; 0
 * leaves attention unpermuted and must be 0 for every other kind. */
typedef struct {
  int32_t layer;
  int32_t kind;  /* cloak_kind */
  int64_t n_out;
  int64_t k_in;
  int32_t dtype; /* cloak_dtype */
  int32_t head_dim;
} cloak_shape;

/* Layout flags. */
#define CLOAK_IDENTITY 1u /* sigma, pi and phi are identities: plain contiguous layer order */
#define CLOAK_NATIVE   2u /* with CLOAK_IDENTITY: kernels address the pool contiguously with
                             no page translation (the uncloaked comparator); remap refused */
#define CLOAK_CSPRNG   4u /* every draw of the layout (tags 1-6, and the remap matchings of
                             this layout) takes its words from counter-mode SHA-256 instead
                             of SplitMix64 (definition above); decoys keep SplitMix64 */
#define CLOAK_MASKED_MAP 8u /* the page map on the device is stored masked (definition
                             above) under a key that changes at every upload of the map
                             (cloak_layout_to_device, every remap slice) and reaches the
                             kernels only as a launch argument */
#define CLOAK_REMAP_UNIFORM 16u /* every remap of this layout re-draws the whole page map
                             uniformly (definition above): phi' = rho o phi for a fresh
                             rho, in two passes of page-pair swaps (about twice the
                             traffic of the matching remap, still no scratch page) */

/* cloak_query() selectors. */
#define CLOAK_QUERY_P            1  /* int64: pages in the pool                        */
#define CLOAK_QUERY_V            2  /* int64: virtual pages used by tensors             */
#define CLOAK_QUERY_T            3  /* int64: number of tensors                         */
#define CLOAK_QUERY_PAGE_BYTES   4  /* int64                                            */
#define CLOAK_QUERY_PHI          5  /* int32[P]: current page map                       */
#define CLOAK_QUERY_SIGMA        6  /* int32[T]: tensor order                           */
#define CLOAK_QUERY_PI           7  /* int32[d_ffn]: hidden permutation of layer `index`*/
#define CLOAK_QUERY_VBASE        8  /* int64[T]                                          */
#define CLOAK_QUERY_NPAGES       9  /* int64[T]                                          */
#define CLOAK_QUERY_CONTIGUITY  10  /* double: share of in-tensor page successions that
                                       stay physically adjacent (Table 2 statistic)     */
#define CLOAK_QUERY_UPLOAD_ORDER 11 /* int32[npages of tensor `index`]                  */
#define CLOAK_QUERY_REMAPS      12  /* int64: remaps applied since build                */
#define CLOAK_QUERY_TENSOR      13  /* int64: index of tensor (layer = index >> 8,
                                       kind = index & 255), or -1                        */
#define CLOAK_QUERY_DFFN        14  /* int64: hidden size of layer `index` (0 if no FFN) */
#define CLOAK_QUERY_REMAP_PENDING 15 /* int64: page pairs of the remap in progress not yet
                                        swapped (0 if none)                              */
#define CLOAK_QUERY_ROW_PERM    16  /* int32[N] of tensor `index`: stored row j holds
                                       logical row p[j] (identity if rows stay put)      */
#define CLOAK_QUERY_COL_PERM    17  /* int32[K] of tensor `index`: stored column j holds
                                       logical column p[j] (identity if columns stay)   */
#define CLOAK_QUERY_SHAPE       18  /* int64[4] of tensor `index`: n_out, k_in, dtype,
                                       head_dim                                          */
#define CLOAK_QUERY_MAP_KEY     19  /* uint64: key of the page map now on the device (0 if
                                       the map is stored plain or not uploaded)         */

/* Workspace selectors for cloak_ws_bytes(). */
#define CLOAK_OP_LINEAR 1   /* index = tensor */
#define CLOAK_OP_MLP    2   /* index = layer  */
#define CLOAK_OP_SWIGLU 3   /* index = layer  */
#define CLOAK_OP_DOWN   4   /* index = layer  */

/* Draw the layout from `seed` for `n_shapes` tensors (Section 5: all
 * permutations and page placements are fixed before any transfer).  Host
 * only, touches no device.  page_bytes must be a power of two >= 1024 and
 * divide pool_bytes.  Errors: EINVAL (sizes, kinds, dtypes, head_dim on a
 * non-attention kind), ESHAPE (duplicate (layer, kind), inconsistent hidden
 * sizes, q/k/v/o of a head-permuted layer missing or not whole heads),
 * ENOMEM (the tensors need more than P pages).  On success *out owns the layout. */
int cloak_layout_build(uint64_t seed, const cloak_shape* shapes, int32_t n_shapes,
                       uint64_t page_bytes, uint64_t pool_bytes, uint32_t flags,
                       cloak_layout** out);

/* Free the layout drawn by cloak_layout_build (the host-side secret of
 * Section 5, Implementation Details: permutations and page placement) and its
 * device tables.  Waits for nothing: the caller must not free while kernels
 * that use the layout are in flight.  NULL is a no-op; always returns CLOAK_OK. */
int cloak_layout_free(cloak_layout* layout);

/* Allocate and upload the device tables on the current device: the page map
 * (Table 1b; the virtual->physical indirection of Section 4.1 that the
 * kernels resolve), the hidden and head permutations, the FP8 scale table and
 * the remap pair list.  Required before any device call.  Idempotent.
 * Errors: EINVAL (null layout), EHIP (allocation or copy failed; nothing is
 * kept). */
int cloak_layout_to_device(cloak_layout* layout, void* stream);

/* Copy a property of the layout into `out`: the tensor order (Section 4.2,
 * Table 1a), the page map (Table 1b), the hidden permutations (abstract), the
 * contiguity statistic of Table 2, remap state.  out_bytes must be large
 * enough (sizes listed with the selectors); `index` selects the tensor or
 * layer where a selector needs one.  Host only.  EINVAL on an unknown
 * selector, a bad index or a short buffer. */
int cloak_query(const cloak_layout* layout, int32_t what, int64_t index, void* out,
                uint64_t out_bytes);

/* Copy the device page map table as stored (masked on CLOAK_MASKED_MAP
 * layouts) into h_out[P] (for verification of the Table 1b indirection the
 * kernels read).  Synchronises `stream`.  ESTATE before
 * cloak_layout_to_device, EINVAL on a null h_out. */
int cloak_device_map_read(const cloak_layout* layout, int32_t* h_out, void* stream);

/* Zero the whole pool (free pages and padding hold zeros): the page pool of
 * Section 4.2 whose pages the layout scatters tensors over.  d_pool must be
 * 256-byte aligned and at least pool_bytes long; the caller owns it.
 * Enqueued on `stream`. */
int cloak_pool_init(const cloak_layout* layout, void* d_pool, void* stream);

/* Fill every free virtual page (V..P-1, at its current physical page) with
 * decoy values (definition above) so that pages without weights look like
 * weights.  Optional; call after cloak_pool_init, before or after loads (it
 * touches no tensor page).  A remap carries decoys along with their pages.
 * The paper leaves free pages unspecified (Section 4.2). */
int cloak_pool_decoy(const cloak_layout* layout, void* d_pool, uint64_t decoy_seed, void* stream);

/* Host image of cloak_pool_decoy on a host pool buffer of pool_bytes. */
int cloak_pool_decoy_host(const cloak_layout* layout, void* h_pool, uint64_t h_pool_bytes,
                          uint64_t decoy_seed);

/* Upload tensor `tensor` from its logical nn.Linear array h_src ([N][K] of
 * the tensor's storage type; FP8 as raw E4M3 bytes) into the pool: apply the
 * hidden permutation, cut the stream into pages and copy page v to physical
 * page phi[v], pages in the seeded upload order (Section 4.2: the transfer
 * order is permuted; Section 5: layout fixed before transfer).  h_scales
 * ([N] f32, logical order) is required for FP8 and must be NULL otherwise.
 * The FIRST upload of each tensor must follow the tensor order sigma
 * (CLOAK_QUERY_SIGMA): a tensor that is not sigma[number of tensors uploaded
 * so far] is refused with ESTATE, so the bus never sees tensors in their
 * architectural order; a tensor already uploaded may be sent again.
 * Synchronises `stream` before returning. */
int cloak_load(cloak_layout* layout, void* d_pool, int32_t tensor, const void* h_src,
               const float* h_scales, void* stream);

/* Upload every tensor, in the tensor order sigma (the library iterates
 * sigma; Section 4.2, Section 5): h_srcs[t] is tensor t's logical array (t the
 * index in the shape list given to cloak_layout_build), h_scales[t] its FP8
 * row scales or NULL; h_scales itself may be NULL when no tensor is FP8.
 * Every entry is checked before the first page is sent (EINVAL).  Then as
 * cloak_load for each tensor.  Synchronises `stream`. */
int cloak_load_all(cloak_layout* layout, void* d_pool, const void* const* h_srcs,
                   const float* const* h_scales, void* stream);

/* Inverse of cloak_load (for verification): follow the page map (Table 1b)
 * and undo the hidden permutation (abstract) to gather tensor `tensor` from
 * the pool into the logical array h_dst ([N][K] of its storage type,
 * caller-owned host memory).  Synchronises `stream`.  EINVAL on a bad
 * tensor index or null h_dst, ESTATE before cloak_layout_to_device. */
int cloak_unload(const cloak_layout* layout, const void* d_pool, int32_t tensor, void* h_dst,
                 void* stream);

/* Host-side image of cloak_load (Section 4.2 placement): write tensor
 * `tensor`'s pages into a host buffer h_pool of pool_bytes (the same bytes
 * cloak_load writes to the device).  No device needed; any order.  FP8 scales
 * are not part of the pool image.  EINVAL on a short buffer or bad index. */
int cloak_pack_host(const cloak_layout* layout, int32_t tensor, const void* h_src,
                    void* h_pool, uint64_t h_pool_bytes);

/* Bytes of device workspace `op` needs for `index` at M tokens (for the
 * projections of Section 4.2's bandwidth-bound inference): the FP32
 * partial sums of the split-K decode GEMM (5..256 tokens; 257..1024 tokens
 * run as pieces of at most 256 that reuse one piece's workspace), for a down
 * projection called through cloak_linear its activations gathered through
 * pi, and for FP8 weights from 65 tokens the per-token E4M3 activations and
 * their scales (M*K + 4*M bytes, each rounded up to 256).  0 if none;
 * UINT64_MAX on bad arguments. */
uint64_t cloak_ws_bytes(const cloak_layout* layout, int32_t op, int32_t index, int64_t M);

/* Workspace of cloak_linear_fused for these n tensors at M tokens (as
 * cloak_ws_bytes; UINT64_MAX on bad arguments). */
uint64_t cloak_linear_fused_ws_bytes(const cloak_layout* layout, const int32_t* tensors, int32_t n,
                                     int64_t M);

/* The cloaked linear layer: the weights stay resident and are read in place
 * on every forward pass (Section 2.3), from pages the layout scattered
 * (Section 4.2, Table 1b), at the bandwidth the performance paragraph of
 * Section 4.2 requires of a bandwidth-bound step.
 * y[M][N] = x[M][K] . W^T for tensor `tensor`, with x and y in LOGICAL
 * order: for gate/up (and head-permuted q/k/v) the kernel scatters stored
 * row j to column p[j]; for down (and head-permuted o) it gathers x through
 * the column permutation while staging it.  Weights are read straight
 * from the scattered pages (virtual tile -> physical page resolved in the
 * kernel).  M = 0 is a no-op.  Workspace as reported by cloak_ws_bytes.
 * x 16-byte aligned; errors EINVAL (sizes, null buffers, short workspace),
 * ESTATE (no device tables, wrong device), EHIP (launch failed). */
int cloak_linear(const cloak_layout* layout, const void* d_pool, int32_t tensor,
                 const void* d_x, int64_t M, void* d_y, void* d_ws, uint64_t ws_bytes,
                 void* stream);

/* cloak_linear over several tensors with the same K in one launch (e.g.
 * q, k, v; Section 4.2 performance paragraph): y is [M][sum N_i], tensor i's
 * columns at offset sum_{j<i} N_j.  n <= 4; ESHAPE if K or dtype differ or a
 * tensor with permuted columns is fused with others. */
int cloak_linear_fused(const cloak_layout* layout, const void* d_pool, const int32_t* tensors,
                       int32_t n, const void* d_x, int64_t M, void* d_y, void* d_ws,
                       uint64_t ws_bytes, void* stream);

/* cloak_linear_fused with x and y in STORED order: x's column j feeds the
 * tensors' stored column j, y's column j is stored row j (no scatter of
 * permuted rows, no gather of permuted columns; CLOAK_QUERY_ROW_PERM /
 * COL_PERM give the orders).  For callers that keep a whole block in stored
 * order, where the intra-layer permutations cancel between consecutive
 * projections (abstract): the decoder step runs q/k/v, attention and o, and
 * gate/up and down, this way.  Workspace: cloak_linear_fused_ws_bytes. */
int cloak_linear_stored(const cloak_layout* layout, const void* d_pool, const int32_t* tensors, int32_t n,
                        const void* d_x, int64_t M, void* d_y, void* d_ws, uint64_t ws_bytes,
                        void* stream);

/* SwiGLU FFN of layer `layer` under the intra-layer shuffle (abstract: the
 * hidden neurons of each FFN are permuted): y = (silu(x Wg^T) * (x Wu^T)) Wd^T,
 * with silu(z) = z / (1 + e^-z), run directly on the shuffled weights: the
 * hidden activations stay in permuted order (bf16 for bf16/fp8 weights, f32
 * for f32) in the workspace, so the permutation cancels between up/gate and
 * down.  x, y: [M][d_model] in logical order.  Workspace: cloak_mlp_ws_bytes.
 * Errors: EINVAL (layer lacks gate/up/down, null buffers, short workspace). */
uint64_t cloak_mlp_ws_bytes(const cloak_layout* layout, int32_t layer, int64_t M);
int cloak_mlp(const cloak_layout* layout, const void* d_pool, int32_t layer, const void* d_x,
              int64_t M, void* d_y, void* d_ws, uint64_t ws_bytes, void* stream);

/* cloak_mlp for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * kernels and results, with the workspace taken from a static device array of
 * CLOAK_MLP_NOALLOC_MAX_BYTES per GPU (held until the process ends; its device
 * address is looked up once per device on the first call there).  The caller
 * still owns x and y.  No call allocates or frees memory.  Calls whose
 * cloak_mlp_ws_bytes exceeds the maximum are refused with EINVAL (64 MiB
 * covers a 4096/14336 BF16 layer up to 2048 tokens and a 5120/27648 FP8 layer
 * up to 128).  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (several streams, several threads) race and give
 * undefined results; calls on one stream are ordered and safe.  Nothing in the
 * array needs to start at zero: a call reads only bytes it has written. */
#define CLOAK_MLP_NOALLOC_MAX_BYTES (64ull << 20)
int cloak_mlp_noalloc(const cloak_layout* layout, const void* d_pool, int32_t layer, const void* d_x,
                      int64_t M, void* d_y, void* stream);

/* First half of cloak_mlp (abstract, intra-layer shuffle), one launch: h[M][d_ffn] = silu(x Wg^T) * (x Wu^T)
 * with h left in the layer's PERMUTED hidden order (column j holds hidden
 * unit pi[j]); each workgroup reads matching gate and up rows.  h is bf16
 * (f32 for f32 weights). */
int cloak_swiglu(const cloak_layout* layout, const void* d_pool, int32_t layer, const void* d_x,
                 int64_t M, void* d_h, void* d_ws, uint64_t ws_bytes, void* stream);

/* Second half of cloak_mlp (abstract, intra-layer shuffle), one launch: y[M][d_model] = h . Wd^T for h in the
 * permuted hidden order cloak_swiglu produces (down's stored columns carry
 * the same permutation, so nothing is gathered).  Workspaces: cloak_ws_bytes
 * with CLOAK_OP_SWIGLU / CLOAK_OP_DOWN. */
int cloak_down(const cloak_layout* layout, const void* d_pool, int32_t layer, const void* d_h,
               int64_t M, void* d_y, void* d_ws, uint64_t ws_bytes, void* stream);

/* Bandwidth calibration for the bandwidth-bound decode that the performance
 * paragraph of Section 4.2 speaks of (not part of the cloaked path): stream every byte of
 * d_src once with non-temporal 16-byte loads, as the weight-reading kernels
 * do, and fold them into one word that is written to *d_out only when it
 * equals a constant.  Gives the device's plain streaming-read rate, the
 * practical ceiling the decode kernels are compared with.  bytes: multiple of
 * 16; d_src 16-byte aligned.  Asynchronous on `stream`. */
int cloak_stream_read(const void* d_src, uint64_t bytes, uint32_t* d_out, void* stream);

/* Mixture-of-experts layer over cloaked experts (the paper serves a Qwen 3
 * MoE model, Section 5; experts are ordinary cloaked tensors: each expert e is
 * the FFN group of layer first_layer + e, with its own hidden permutation and
 * its own place in the tensor order).  For token m:
 *   y[m] = sum_j d_weights[m][j] * FFN_{d_ids[m][j]}(x[m]),
 * FFN_e = down_e(silu(gate_e x) * up_e x); slots whose id lies outside
 * [0, n_experts) are skipped.  x, y: [M][d_model] bf16; d_ids int32 and
 * d_weights f32 [M][top_k] on the device (routing is the caller's).  Experts
 * are BF16 or FP8 (per-row scales) with one d_model and d_ffn.  The hidden
 * activations are rounded to bf16, the weighted expert outputs kept in f32 and
 * added per token in slot order.  Calls of more than 4096 (token, slot) pairs
 * run in consecutive chunks of floor(4096 / top_k) tokens on one workspace;
 * top_k <= 4096.  x 16-byte, y 8-byte and the workspace 256-byte aligned.
 * Workspace: cloak_moe_ws_bytes.  Errors: EINVAL (experts missing or inconsistent, sizes,
 * workspace). */
uint64_t cloak_moe_ws_bytes(const cloak_layout* layout, int32_t first_layer, int32_t n_experts, int32_t top_k,
                            int64_t M);
int cloak_moe(const cloak_layout* layout, const void* d_pool, int32_t first_layer, int32_t n_experts,
              int32_t top_k, const void* d_x, int64_t M, const int32_t* d_ids, const float* d_weights,
              void* d_y, void* d_ws, uint64_t ws_bytes, void* stream);

/* Per-token FP8 quantisation of activations, as the FP8 x FP8 MFMA path
 * applies it to x before a projection with FP8 weights and more than 256
 * tokens (the paper names FP8 weights with per-channel scales; this
 * activation format is this library's reading): for each row m of the bf16
 * array d_x ([M][ldx] elements, ldx >= K),
 *   s[m] = max_k |x[m][k]| / 448 in binary32 (1 if the row is all zero),
 *   q[m][k] = E4M3 code nearest to the binary32 quotient x[m][k] / s[m]
 *             (ties to the even code, saturating at +-448, OCP E4M3FN).
 * d_q receives [M][K] bytes, d_s M floats (caller-owned device buffers).
 * Enqueues on `stream`.  M = 0 is a no-op; EINVAL on null buffers, K < 1 or
 * ldx < K. */
int cloak_quantize_fp8(const void* d_x, int64_t M, int64_t K, int64_t ldx, void* d_q, void* d_s,
                       void* stream);

/* Re-randomise page placement in place (Section 4.2, physical page
 * remapping: the map is re-drawn from time to time and no memory is added
 * for it).  Default: draw the matching tau from remap_seed, swap every page
 * pair in the pool on `stream`, and set phi' = tau o phi on host and device
 * (one pass, each pool byte read and written once).  On CLOAK_REMAP_UNIFORM
 * layouts: draw rho from remap_seed and run its two passes of swaps (one
 * launch each), phi' = rho o phi.  Refused (ESTATE) on CLOAK_NATIVE layouts
 * and while an incremental remap is in progress.  Device memory stays as it
 * was: no allocation, the pair list goes into a table made by
 * cloak_layout_to_device. */
int cloak_remap(cloak_layout* layout, void* d_pool, uint64_t remap_seed, void* stream);

/* Incremental remap (spreads one remap over several serving steps, so no
 * single step pays the whole move; the paper leaves the cadence to the
 * operator, Section 4.2 and Figure 7).  cloak_remap_begin draws tau (or rho
 * and its two passes, on CLOAK_REMAP_UNIFORM layouts) from remap_seed; each
 * cloak_remap_step then swaps the next max_pairs page pairs (pairs in the
 * order of the definition; a step never runs pairs of both passes, so a
 * bounded step stops at the end of pass 1; max_pairs <= 0 runs everything
 * left, one launch per pass) on `stream` and updates phi for exactly those
 * pages, host and device, in stream order.  Between steps the pool and phi are a
 * complete, consistent layout, so any cloak_* call may run between them;
 * after the last pair the result equals cloak_remap(remap_seed).
 * *remaining (may be NULL) receives the pairs still to swap.
 * cloak_remap_begin: ESTATE on native layouts or while a remap is in
 * progress.  cloak_remap_step: ESTATE when none is in progress.  The host
 * variant applies a step to a pool image (tests; no device needed). */
int cloak_remap_begin(cloak_layout* layout, uint64_t remap_seed);
int cloak_remap_step(cloak_layout* layout, void* d_pool, int64_t max_pairs, int64_t* remaining,
                     void* stream);
int cloak_remap_step_host(cloak_layout* layout, void* h_pool, uint64_t h_pool_bytes, int64_t max_pairs,
                          int64_t* remaining);

/* Hardware-translated twin (the paper's own mechanism, Section 4.2: the
 * shuffled placement is resolved by the GPU's MMU and kernels read plain
 * contiguous addresses).  Allocates every physical page of the pool as its
 * own virtual-memory allocation (page_bytes must be a multiple of the
 * device's allocation granularity, 2 MiB on MI355X) and maps them twice: in
 * physical order at *d_pool_view, which the caller then passes as d_pool to
 * every cloak_* call (cloak_pool_init, cloak_load, cloak_linear, ...), and in
 * virtual order (virtual page v on physical page phi[v]) at a tensor view the
 * library keeps.  While the twin exists the weight-reading kernels of that
 * layout run untranslated on the tensor view; a remap swaps pages through
 * the pool view, synchronises `stream`, then re-points the swapped pages'
 * virtual addresses (host calls, not stream-ordered: no other stream may be
 * reading the layout).  The library owns the memory; cloak_vmm_pool_free
 * (or cloak_layout_free) releases it.  ESTATE before cloak_layout_to_device,
 * on native layouts, during a remap, or where the device has no virtual
 * memory management; EINVAL on a page size below the granularity. */
int cloak_vmm_pool_create(cloak_layout* layout, void** d_pool_view);
int cloak_vmm_pool_free(cloak_layout* layout);

/* Host-side remap (Section 4.2, physical page remapping) of a pool image
 * h_pool (pool_bytes) and of the layout's page map; the same result
 * cloak_remap produces on the device, matching or uniform as the layout's
 * flags say.  Updates only the host copy of phi: do not mix with device calls
 * on one layout.  ESTATE on native layouts or during an incremental remap. */
int cloak_remap_host(cloak_layout* layout, void* h_pool, uint64_t h_pool_bytes,
                     uint64_t remap_seed);

/* ------------------------------------------------------------------------
 * Decoder step for the serving loop.  The engine keeps KV state on the
 * device (Section 4.1: the serving engine manages KV-cache blocks); only the
 * weights are cloaked.  A model binds a layout whose tensors are, per layer
 * l, (l, q) (l, k) (l, v) (l, o) (l, gate) (l, up) (l, down) in BF16, plus
 * (-1, embed) [vocab][d_model] and (-1, head) [vocab][d_model].
 * ------------------------------------------------------------------------ */
typedef struct cloak_model cloak_model; /* opaque, owned by the library */

typedef struct {
  int32_t n_layers, d_model, n_heads, n_kv_heads, head_dim, d_ffn, vocab;
  int32_t block_size;  /* tokens per KV block */
  int64_t num_blocks;  /* KV blocks per layer */
  float rope_theta;    /* rotate-half RoPE base */
  float norm_eps;      /* RMSNorm epsilon */
} cloak_model_config;

/* One step's batch: n_tokens new tokens of n_seqs sequences (a prefill chunk
 * or one decode token each), all arrays on the device.  Tokens of a sequence
 * are consecutive in the arrays with consecutive positions; its KV blocks are
 * block_table[seq][0 .. ceil(ctx/block_size)).  Attention work: n_tiles tiles
 * of <= 16 consecutive tokens of one sequence (tile_seq/tok0/ntok), the
 * context cut into n_splits slices of split_keys keys.  The first n_single
 * tiles are expected to hold one token each (decode tokens): they run on the
 * single-token attention path, which still computes any tile correctly but
 * is slow on long ones.  0 <= n_single <= n_tiles. */
typedef struct {
  int32_t n_tokens, n_seqs, max_blocks, n_logits;
  int32_t n_tiles, n_splits, split_keys, n_single;
  const int32_t* d_tokens;       /* [n_tokens] token ids (< vocab)            */
  const int32_t* d_positions;    /* [n_tokens]                                */
  const int32_t* d_tok_seq;      /* [n_tokens] sequence slot of each token    */
  const int32_t* d_block_table;  /* [n_seqs][max_blocks] KV block ids         */
  const int32_t* d_tile_seq;     /* [n_tiles]                                 */
  const int32_t* d_tile_tok0;    /* [n_tiles]                                 */
  const int32_t* d_tile_ntok;    /* [n_tiles]                                 */
  const int32_t* d_logit_rows;   /* [n_logits] token rows that get logits     */
  int32_t* d_out_tokens;         /* [n_logits] greedy argmax                  */
  void* d_out_logits;            /* [n_logits][vocab] bf16, or NULL           */
} cloak_step;

/* Serving model over a cloaked layout (Section 4.1: the engine's KV blocks;
 * Section 5.2: iteration latency of prefill and decode).  Bind a layout, its pool, RMSNorm gains (d_gains: [2*n_layers+1][d_model]
 * bf16 in the order attn_0, mlp_0, ..., final; NULL = all ones) and the KV
 * cache (d_kv: [n_layers][2][num_blocks][n_kv_heads][block_size][head_dim]
 * bf16, caller-owned).  head_dim must be 128 and n_heads/n_kv_heads <= 8.
 * Errors: EINVAL, ESHAPE (missing tensor or shapes that disagree with cfg). */
int cloak_model_create(const cloak_layout* layout, const void* d_pool, const cloak_model_config* cfg,
                       const void* d_gains, void* d_kv, cloak_model** out);
int cloak_model_free(cloak_model* model);

/* Workspace of cloak_model_step (Section 4.1 serving step) for steps of at
 * most max_tokens tokens, max_logits logit rows and max_tiles * max_splits
 * attention slices.  UINT64_MAX on bad arguments. */
uint64_t cloak_model_ws_bytes(const cloak_model* model, int64_t max_tokens, int64_t max_logits,
                              int64_t max_tiles, int64_t max_splits);

/* Run one decoder step on `stream`: embedding -> layers (RMSNorm, fused
 * q/k/v projection, RoPE + KV write, paged attention, o projection,
 * residual, RMSNorm, cloak_swiglu, cloak_down, residual) -> final RMSNorm of
 * the logit rows -> head projection -> argmax.  Enqueues only. */
int cloak_model_step(cloak_model* model, const cloak_step* step, void* d_ws, uint64_t ws_bytes,
                     void* stream);

/* Message describing the last error on the calling thread ("" if none);
 * every call above reports its failures here (the error convention at the
 * top of this file).  The string is owned by the library and valid until the
 * thread's next call. */
const char* cloak_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CLOAK_H */

"""Seeded synthetic inputs: weights, activations, FP8 quantised weights, traces.

This module holds none of the cloaking arithmetic (no shuffles, no page maps,
no products).  It only produces the numbers the cloaked layer is fed, so the
HIP path and the CPU oracle can be given identical inputs without sharing any
code.  The paper evaluates Llama 3.1 8B, Qwen 3 14B and Qwen 3 MoE 30B
checkpoints (Section 5, Setup); none are available here, so random weights of
the same kinds of shapes stand in for them:

* weights ~ N(0, 0.02) drawn in FP32 from ``PCG64(1234 + tensor_index)``,
  rounded to nearest-even into the storage type;
* FP8 E4M3 weights: one FP32 scale per output row ``s[n] = max|W[n,:]| / 448``
  and ``q = E4M3(W / s)`` rounded to nearest-even, saturating at +-448 (OCP
  8-bit floating point specification); the stored model *is* (q, s);
* activations ~ N(0, 1) from ``PCG64(5678)`` (or a caller seed), rounded to
  the activation type.
"""

import numpy as np

WEIGHT_STD = 0.02


def f32_to_bf16_rne(f):
    """float32 array -> bfloat16 bit patterns (uint16), nearest-even."""
    u = np.ascontiguousarray(f, dtype=np.float32).view(np.uint32)
    rounding = np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))
    out = ((u + rounding) >> np.uint32(16)).astype(np.uint16)
    nan = (u & np.uint32(0x7FFFFFFF)) > np.uint32(0x7F800000)
    if nan.any():
        out[nan] = 0x7FC0
    return out


def bf16_to_f32(bits):
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def f32_to_e4m3_rne(v):
    """float array -> OCP E4M3FN bit patterns (uint8), nearest-even, saturating."""
    v = np.asarray(v, dtype=np.float64)
    a = np.abs(v)
    _, ex = np.frexp(a)
    e = np.where(a < 2.0 ** -6, -6, ex - 1).astype(np.int64)
    r = np.rint(a / np.power(2.0, e - 3)).astype(np.int64)   # 8..16 normal, 0..8 subnormal
    bits = 8 * (e + 6) + r
    bits = np.minimum(bits, 0x7E)
    bits = np.where(a == 0, 0, bits)
    bits = bits | np.where(np.signbit(v), 0x80, 0)
    return bits.astype(np.uint8)


def weight_f32(tensor_index, n_out, k_in, base_seed=1234):
    rng = np.random.Generator(np.random.PCG64(base_seed + tensor_index))
    w = rng.standard_normal((n_out, k_in), dtype=np.float32)
    w *= np.float32(WEIGHT_STD)
    return w


def quantize_fp8_rows(w_f32, rows_per_block=1024):
    """Per-output-row FP8 quantisation: returns (q bits [N][K] uint8, s [N] f32)."""
    amax = np.max(np.abs(w_f32), axis=1).astype(np.float32)
    s = (amax / np.float32(448.0)).astype(np.float32)
    s = np.where(s == 0, np.float32(1.0), s).astype(np.float32)
    q = np.empty(w_f32.shape, dtype=np.uint8)
    for r0 in range(0, w_f32.shape[0], rows_per_block):   # bounded temporaries
        blk = w_f32[r0:r0 + rows_per_block].astype(np.float64) / s[r0:r0 + rows_per_block].astype(np.float64)[:, None]
        q[r0:r0 + rows_per_block] = f32_to_e4m3_rne(blk)
    return q, s


def weight(tensor_index, n_out, k_in, dtype, base_seed=1234):
    """Stored weight for one tensor: (array, scales or None)."""
    w = weight_f32(tensor_index, n_out, k_in, base_seed)
    if dtype == "f32":
        return w, None
    if dtype == "bf16":
        return f32_to_bf16_rne(w), None
    if dtype == "fp8":
        return quantize_fp8_rows(w)
    raise ValueError(dtype)


def activations(m, k, dtype, seed=5678):
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal((m, k), dtype=np.float32)
    if dtype == "f32":
        return x
    if dtype == "bf16":
        return f32_to_bf16_rne(x)
    raise ValueError(dtype)


# --------------------------------------------------------------------------
# Workload shapes (random-weight stand-ins for the paper's models).
# Each entry is (layer, kind, n_out, k_in, dtype) in nn.Linear orientation.
# --------------------------------------------------------------------------

def ffn_block_shapes(d_model, d_ffn, dtype, layer=0):
    return [(layer, "gate", d_ffn, d_model, dtype),
            (layer, "up", d_ffn, d_model, dtype),
            (layer, "down", d_model, d_ffn, dtype)]


def decoder_layer_shapes(d_model, d_ffn, d_kv, dtype, layer=0, head_dim=0):
    """q/k/v/o carry ``head_dim`` as a sixth entry when it is given (> 0)."""
    hd = (head_dim,) if head_dim else ()
    return [(layer, "q", d_model, d_model, dtype) + hd,
            (layer, "k", d_kv, d_model, dtype) + hd,
            (layer, "v", d_kv, d_model, dtype) + hd,
            (layer, "o", d_model, d_model, dtype) + hd] + ffn_block_shapes(d_model, d_ffn, dtype, layer)


# FP32 FFN block, d_model 512, d_ffn 1024, 64 KiB pages over 16 MiB.
FFN512 = dict(d_model=512, d_ffn=1024, dtype="f32", page_bytes=64 << 10, pool_bytes=16 << 20, M=4)
# One Llama-3.1-8B-class decoder layer in BF16, 2 MiB pages over 8 GiB.
LAYER4096 = dict(d_model=4096, d_ffn=14336, d_kv=1024, dtype="bf16",
                 page_bytes=2 << 20, pool_bytes=8 << 30)
# 64-layer FP8 stack, d_model 5120, d_ffn 27648, BF16 head (vocab 152064), ~34 GiB pool.
STACK5120 = dict(d_model=5120, d_ffn=27648, d_kv=1024, n_layers=64, vocab=152064,
                 page_bytes=2 << 20, pool_bytes=34 << 30)


def prefill_lengths(total=8192, lo=256, hi=4096, max_seqs=16, seed=91):
    """Sequence lengths ~ U[lo, hi] drawn until their sum reaches ``total``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    while True:
        lens = []
        while sum(lens) < total:
            lens.append(int(rng.integers(lo, hi + 1)))
        lens[-1] -= sum(lens) - total
        if len(lens) <= max_seqs and lens[-1] > 0:
            return lens


def poisson_trace(n_requests, rate, prompt_lo, prompt_hi, out_lo, out_hi, vocab, seed=7):
    """Arrival times (s), prompt token ids and forced output lengths."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n_requests):
        plen = int(rng.integers(prompt_lo, prompt_hi + 1))
        olen = int(rng.integers(out_lo, out_hi + 1))
        prompt = rng.integers(0, vocab, size=plen, dtype=np.int64).astype(np.int32)
        reqs.append(dict(id=i, arrival=float(arrivals[i]), prompt=prompt, max_new=olen))
    return reqs

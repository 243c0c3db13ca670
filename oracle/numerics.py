"""Exact values of stored weights and FP64 reference results (oracle).

The paper's defence must leave inference results unchanged (Section 4.1,
paragraph on virtual-physical address decoupling; Section 6.1): a cloaked
layer has to compute what the plain layer computes.  The reference values are
therefore the plain definitions, evaluated in FP64 on the *logical*
(unshuffled) weights:

* linear:  ``y = x . W^T`` with ``W`` the nn.Linear ``[N][K]`` array;
* FFN:     ``y = (silu(x . Wg^T) * (x . Wu^T)) . Wd^T`` with
           ``silu(z) = z / (1 + exp(-z))`` (SwiGLU; the FFN shape of the
           paper's Llama/Qwen models, Section 5 setup).

Stored weights are decoded exactly from their bit patterns:

* bfloat16 is the upper half of an IEEE binary32 word;
* FP8 E4M3 follows the OCP 8-bit floating point specification (the "FN"
  variant: sign, 4 exponent bits with bias 7, 3 mantissa bits, subnormals at
  exponent 0, no infinities, S.1111.111 is NaN, largest finite 448), and a
  stored FP8 tensor means ``q * s[n]`` with one FP32 scale per output row.
"""

import numpy as np


def bf16_bits_to_f64(bits):
    bits = np.asarray(bits, dtype=np.uint16)
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def e4m3_bits_to_f64(bits):
    b = np.asarray(bits, dtype=np.uint8).astype(np.int64)
    sign = np.where(b & 0x80, -1.0, 1.0)
    e = (b >> 3) & 0xF
    m = (b & 0x7).astype(np.float64)
    normal = (1.0 + m / 8.0) * np.power(2.0, e - 7.0)
    subnormal = (m / 8.0) * 2.0 ** -6
    val = np.where(e == 0, subnormal, normal)
    val = np.where((e == 15) & ((b & 0x7) == 7), np.nan, val)
    return sign * val


def weights_f64(stored, dtype, scales=None):
    """Exact FP64 value of a stored nn.Linear array (logical order)."""
    if dtype == "f32":
        return np.asarray(stored, dtype=np.float32).astype(np.float64)
    if dtype == "bf16":
        return bf16_bits_to_f64(stored)
    if dtype == "fp8":
        w = e4m3_bits_to_f64(stored)
        s = np.asarray(scales, dtype=np.float32).astype(np.float64)
        return w * s[:, None]
    raise ValueError(dtype)


def activations_f64(x, dtype):
    """Exact FP64 value of an activation array stored as f32 or bf16 bits."""
    if dtype == "f32":
        return np.asarray(x, dtype=np.float32).astype(np.float64)
    if dtype == "bf16":
        return bf16_bits_to_f64(x)
    raise ValueError(dtype)


def linear(x64, w64):
    """y[M][N] = sum_k x[m][k] * W[n][k], in FP64."""
    return np.asarray(x64, np.float64) @ np.asarray(w64, np.float64).T


def silu(z):
    z = np.asarray(z, np.float64)
    return z / (1.0 + np.exp(-z))


def swiglu_ffn(x64, wg64, wu64, wd64):
    """SwiGLU FFN in FP64 on logical weights; returns (y, h)."""
    h = silu(linear(x64, wg64)) * linear(x64, wu64)
    return linear(h, wd64), h


def normwise_err(y, y_ref):
    """max |y - y*| / max |y*| over one result tensor (0 if both vanish)."""
    y = np.asarray(y, np.float64)
    y_ref = np.asarray(y_ref, np.float64)
    den = np.max(np.abs(y_ref)) if y_ref.size else 0.0
    num = np.max(np.abs(y - y_ref)) if y_ref.size else 0.0
    if den == 0.0:
        return 0.0 if num == 0.0 else np.inf
    return num / den


def f32_to_bf16_bits_rne(f):
    """Round binary32 values to bfloat16 (nearest, ties to even); NaN kept quiet."""
    u = np.asarray(f, dtype=np.float32).view(np.uint32).astype(np.uint64)
    is_nan = (u & 0x7FFFFFFF) > 0x7F800000
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) & 0xFFFF
    r = np.where(is_nan, ((u >> 16) | 0x40) & 0xFFFF, r)
    return r.astype(np.uint16)


# ----------------------------------------------------------------------------
# FP8 activations for the FP8 x FP8 prefill product.
#
# Reading (the paper names FP8 weights with per-channel scales but no
# activation format): each token's activation row is quantised to E4M3 with
# one FP32 scale s_m = max_k |x[m][k]| / 448 (1 for an all-zero row), the
# quotient x / s_m taken in binary32, then rounded to the nearest E4M3 value
# (ties to the even code, saturating at +-448).  The product is then
# y[m][n] = (sum_k q_x[m][k] q_w[n][k]) * s_m * s_w[n].
# ----------------------------------------------------------------------------

def _e4m3_nonneg_table():
    """Values of the non-negative finite E4M3 codes 0x00..0x7E, ascending."""
    return e4m3_bits_to_f64(np.arange(0x7F, dtype=np.uint8))


def f64_to_e4m3_bits_rne(v):
    """Nearest E4M3FN code by search over the code values: ties go to the even
    code, magnitudes above 448 saturate to 448, the sign bit is kept (also for
    zeros), NaN maps to 0x7F."""
    v = np.asarray(v, dtype=np.float64)
    table = _e4m3_nonneg_table()
    a = np.abs(v)
    hi = np.clip(np.searchsorted(table, a, side="left"), 0, 0x7E)
    lo = np.clip(hi - 1, 0, 0x7E)
    d_lo = a - table[lo]
    d_hi = table[hi] - a
    pick_hi = (d_hi < d_lo) | ((d_hi == d_lo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo)
    code = np.where(a >= table[0x7E], 0x7E, code)   # saturate
    code = np.where(a == 0, 0, code)
    code = code | np.where(np.signbit(v), 0x80, 0)
    code = np.where(np.isnan(v), 0x7F, code)
    return code.astype(np.uint8)


def quantize_rows_e4m3(x32):
    """Per-row E4M3 quantisation of binary32 activations: (codes uint8 [M][K],
    scales float32 [M])."""
    x32 = np.atleast_2d(np.asarray(x32, dtype=np.float32))
    amax = np.max(np.abs(x32), axis=1) if x32.shape[1] else np.zeros(x32.shape[0], np.float32)
    s = (amax.astype(np.float32) / np.float32(448.0)).astype(np.float32)
    s = np.where(s == 0, np.float32(1.0), s).astype(np.float32)
    quot = (x32 / s[:, None]).astype(np.float32)      # binary32 quotient
    return f64_to_e4m3_bits_rne(quot.astype(np.float64)), s


def fp8_activations_f64(q, s):
    """Exact value of quantised activation rows: decode(q) * s."""
    return e4m3_bits_to_f64(q) * np.asarray(s, np.float32).astype(np.float64)[:, None]

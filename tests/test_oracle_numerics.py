"""Pins for exact weight decoding and the FP64 linear / SwiGLU references."""

import os

import numpy as np
import pytest

from oracle import layout as L
from oracle import numerics as N
from paper_2606_18400_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_bf16_decode_known_patterns():
    bits = np.array([0x3F80, 0xC000, 0x0000, 0x8000, 0x7F80, 0xFF80, 0x0001, 0x4049], np.uint16)
    v = N.bf16_bits_to_f64(bits)
    assert v[0] == 1.0 and v[1] == -2.0 and v[2] == 0.0
    assert np.signbit(v[3]) and v[3] == 0.0
    assert v[4] == np.inf and v[5] == -np.inf
    assert v[6] == 2.0 ** -133          # smallest bf16 subnormal
    assert v[7] == 3.140625             # 0x4049 = 1.5703125 * 2


def test_e4m3_decode_spec_table():
    for line in open(os.path.join(GOLDEN, "e4m3fn_values.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        b, val = line.split()
        got = N.e4m3_bits_to_f64(np.array([int(b, 16)], np.uint8))[0]
        if val == "nan":
            assert np.isnan(got)
        else:
            assert got == float(val) and np.signbit(got) == val.startswith("-")


def test_e4m3_positive_codes_strictly_increase():
    v = N.e4m3_bits_to_f64(np.arange(0, 0x7F, dtype=np.uint8))
    assert np.all(np.diff(v) > 0) and v[-1] == 448.0


def test_fp8_weights_scale_rows():
    q = np.array([[0x38, 0x40], [0xB8, 0x00]], np.uint8)
    s = np.array([0.5, 3.0], np.float32)
    assert np.array_equal(N.weights_f64(q, "fp8", s), np.array([[0.5, 1.0], [-3.0, 0.0]]))


def test_linear_exact_on_small_integers_vs_triple_loop():
    rng = np.random.Generator(np.random.PCG64(1))
    x = rng.integers(-8, 9, (3, 7)).astype(np.float64)
    w = rng.integers(-8, 9, (5, 7)).astype(np.float64)
    y = N.linear(x, w)
    for m in range(3):
        for n in range(5):
            assert y[m, n] == sum(x[m, k] * w[n, k] for k in range(7))


def test_silu_closed_forms():
    z = np.linspace(-30, 30, 601)
    s = N.silu(z)
    assert N.silu(0.0) == 0.0
    np.testing.assert_allclose(s - N.silu(-z), z, rtol=0, atol=1e-12)   # x*sig(x) + x*sig(-x) = x
    assert abs(N.silu(40.0) - 40.0) < 1e-15 * 40 + 1e-12
    assert abs(N.silu(1.0) - 1.0 / (1.0 + np.exp(-1.0))) < 1e-16


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_ffn_invariant_under_hidden_permutation(seed):
    d, f, M = 32, 48, 5
    shapes = [L.Shape(0, "gate", f, d, "f32"), L.Shape(0, "up", f, d, "f32"),
              L.Shape(0, "down", d, f, "f32")]
    lay = L.build_layout(seed, shapes, 256, 256 * 128)
    rng = np.random.Generator(np.random.PCG64(seed))
    wg, wu, wd = (rng.standard_normal((s.n_out, s.k_in)) for s in shapes)
    x = rng.standard_normal((M, d))
    y, h = N.swiglu_ffn(x, wg, wu, wd)
    # the FFN evaluated directly on the stored (shuffled) arrays
    gs, us, ds = (L.shuffle_tensor(lay, t, w) for t, w in enumerate((wg, wu, wd)))
    ys, hs = N.swiglu_ffn(x, gs, us, ds)
    assert N.normwise_err(ys, y) <= 1e-12
    # hidden activations come out in permuted order: hs[:, j] == h[:, pi[j]]
    assert np.array_equal(hs, h[:, lay.pi[0]])
    assert lay.pi[0] != list(range(f))


def test_normwise_err():
    assert N.normwise_err([1.0, -2.0], [1.0, -2.0]) == 0.0
    assert N.normwise_err([1.0, -2.5], [1.0, -2.0]) == 0.25
    assert N.normwise_err([0.0], [0.0]) == 0.0


def test_bf16_rne_ties_and_overflow():
    f = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -9,
                  np.float32(3.4028235e38), np.nan], np.float32)
    b = N.f32_to_bf16_bits_rne(f)
    assert list(b[:5]) == [0x3F80, 0x3F80, 0x3F82, 0xBF80, 0x7F80]
    assert (int(b[5]) & 0x7F80) == 0x7F80 and (int(b[5]) & 0x7F)


def test_synth_bf16_rounding_agrees_with_oracle_rne():
    x = np.random.Generator(np.random.PCG64(0)).standard_normal(100000).astype(np.float32)
    assert np.array_equal(synth.f32_to_bf16_rne(x), N.f32_to_bf16_bits_rne(x))


def test_synth_fp8_quantiser_is_nearest_even_saturating():
    # Brute force against every finite E4M3 code (decoded by the oracle).
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], np.uint8)
    vals = N.e4m3_bits_to_f64(codes)
    rng = np.random.Generator(np.random.PCG64(2))
    xs = np.concatenate([rng.standard_normal(4000) * 100, rng.standard_normal(2000) * 0.01,
                         vals, (vals[:-1] + vals[1:]) / 2, [500.0, -1e6, 0.0]])
    q = synth.f32_to_e4m3_rne(xs)
    got = N.e4m3_bits_to_f64(q)
    for x, g, qb in zip(xs, got, q):
        if abs(x) >= 448:
            assert g == np.copysign(448.0, x)
            continue
        d = np.abs(vals - x)
        best = d.min()
        assert abs(g - x) == best
        ties = codes[d == best]
        if len(ties) > 1 and best > 0:   # exact tie: even mantissa wins
            assert (int(qb) & 1) == 0


# ---------------------------------------------------------------- decoder pieces

def test_rmsnorm_closed_form():
    from oracle import model as M
    v = np.array([[3.0, 4.0], [1.0, -1.0]])
    out = M.rmsnorm(v, 1.0, 0.0)
    np.testing.assert_allclose(out[0], [3 / np.sqrt(12.5), 4 / np.sqrt(12.5)], rtol=1e-15)
    np.testing.assert_allclose(out[1], [1.0, -1.0], rtol=1e-15)


def test_rope_is_a_rotation_and_relative():
    from oracle import model as M
    rng = np.random.Generator(np.random.PCG64(1))
    q = rng.standard_normal((5, 16))
    k = rng.standard_normal((5, 16))
    pos = np.array([0, 3, 7, 100, 4097])
    rq = M.rope(q, pos, 500000.0)
    np.testing.assert_allclose(np.linalg.norm(rq, axis=1), np.linalg.norm(q, axis=1), rtol=1e-13)
    np.testing.assert_allclose(rq[0], q[0], rtol=0, atol=0)          # position 0 is the identity
    # scores depend only on the distance: <R(a)q, R(b)k> = <R(a+s)q, R(b+s)k>
    a, b = np.array([10] * 5), np.array([3] * 5)
    s1 = np.sum(M.rope(q, a, 1e4) * M.rope(k, b, 1e4), axis=1)
    s2 = np.sum(M.rope(q, a + 57, 1e4) * M.rope(k, b + 57, 1e4), axis=1)
    np.testing.assert_allclose(s1, s2, rtol=1e-10, atol=1e-12)
    # 2-D case written out: angle = pos * theta^0 for d = 2
    r = M.rope(np.array([[1.0, 0.0]]), np.array([0.5]), 10.0)
    np.testing.assert_allclose(r[0], [np.cos(0.5), np.sin(0.5)], rtol=1e-15)


def test_causal_attention_brute_force():
    from oracle import model as M
    rng = np.random.Generator(np.random.PCG64(2))
    H, Hkv, T, d = 4, 2, 6, 8
    q, k, v = rng.standard_normal((H, T, d)), rng.standard_normal((Hkv, T, d)), rng.standard_normal((Hkv, T, d))
    out = M.causal_attention(q, k, v)
    for h in range(H):
        for t in range(T):
            kv = h // 2
            s = np.array([q[h, t] @ k[kv, j] / np.sqrt(d) for j in range(t + 1)])
            p = np.exp(s - s.max())
            p /= p.sum()
            want = sum(p[j] * v[kv, j] for j in range(t + 1))
            np.testing.assert_allclose(out[t, h * d:(h + 1) * d], want, rtol=1e-12, atol=1e-12)
    # the first token attends only to itself
    np.testing.assert_allclose(out[0, :d], v[0, 0], rtol=1e-13)


# ---------------------------------------------------------------- FP8 activations

def _nearest_e4m3_bruteforce(v):
    """Exact-rational nearest search over all 256 codes (ties: even code)."""
    from fractions import Fraction
    best = None
    target = Fraction(abs(v))
    for code in range(0x7F):
        val = Fraction(float(N.e4m3_bits_to_f64(np.array([code], np.uint8))[0]))
        d = abs(val - target)
        if best is None or d < best[0] or (d == best[0] and code % 2 == 0):
            best = (d, code)
    code = best[1]
    if abs(v) > 448:
        code = 0x7E
    return code | (0x80 if np.signbit(v) else 0)


def test_e4m3_encode_known_values_and_ties():
    cases = {1.0: 0x38, 0.5: 0x30, 448.0: 0x7E, 500.0: 0x7E, 1e9: 0x7E, 2.0 ** -9: 0x01,
             1.5 * 2.0 ** -9: 0x02,          # tie 1 / 2 -> even
             0.5 * 2.0 ** -9: 0x00,          # tie 0 / 1 -> even (zero)
             1.0625: 0x38,                    # tie 1.0 / 1.125 -> even
             1.1875: 0x3A,                    # tie 1.125 / 1.25 -> even
             432.0: 0x7E,                     # tie 416 / 448 -> even (0x7E)
             2.0 ** -6: 0x08, 7 * 2.0 ** -9: 0x07, 15 * 2.0 ** -10: 0x08,   # tie 7 / 8 sub->normal
             -1.0: 0xB8}
    got = N.f64_to_e4m3_bits_rne(np.array(list(cases)))
    assert list(got) == list(cases.values())
    assert list(N.f64_to_e4m3_bits_rne(np.array([0.0, -0.0]))) == [0x00, 0x80]
    assert N.f64_to_e4m3_bits_rne(np.array([np.nan]))[0] == 0x7F


def test_e4m3_encode_roundtrips_every_finite_code():
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], np.uint8)
    vals = N.e4m3_bits_to_f64(codes)
    assert np.array_equal(N.f64_to_e4m3_bits_rne(vals), codes)


def test_e4m3_encode_matches_bruteforce_on_random_values():
    rng = np.random.Generator(np.random.PCG64(41))
    v = np.concatenate([rng.standard_normal(300) * 40, rng.standard_normal(100) * 1e-2,
                        rng.uniform(-520, 520, 100)])
    got = N.f64_to_e4m3_bits_rne(v)
    want = [_nearest_e4m3_bruteforce(float(x)) for x in v]
    assert list(got) == want


def test_quantize_rows_scale_and_error_bounds():
    rng = np.random.Generator(np.random.PCG64(42))
    x = rng.standard_normal((7, 333)).astype(np.float32)
    x[3] = 0.0
    x[5, 17] = -9.5                          # a negative row maximum
    q, s = N.quantize_rows_e4m3(x)
    assert q.dtype == np.uint8 and s.dtype == np.float32
    assert s[3] == 1.0 and np.all(q[3] == 0)
    for m in range(7):
        if m == 3:
            continue
        k = int(np.argmax(np.abs(x[m])))
        assert q[m, k] & 0x7F == 0x7E        # the row maximum lands on +-448
        assert s[m] == np.float32(np.max(np.abs(x[m])) / np.float32(448.0))
    assert q[5, 17] == 0xFE
    # each dequantised element is within half an E4M3 step (relative 2^-4) or
    # half the subnormal step of its value
    deq = N.fp8_activations_f64(q, s)
    step = np.maximum(np.abs(x.astype(np.float64)) * 2.0 ** -4, 2.0 ** -10 * s[:, None].astype(np.float64))
    assert np.all(np.abs(deq - x) <= step * (1 + 1e-9))


def test_fp8_product_reduces_to_exact_integers():
    # codes of small integers are exact, and with unit scales the product is
    # plain integer arithmetic
    xq = N.f64_to_e4m3_bits_rne(np.array([[1.0, 2.0, -3.0, 4.0]]))
    wq = N.f64_to_e4m3_bits_rne(np.array([[5.0, -6.0, 7.0, 8.0], [1.0, 1.0, 1.0, 1.0]]))
    x = N.fp8_activations_f64(xq, np.array([0.5], np.float32))
    w = N.weights_f64(wq, "fp8", np.array([2.0, 0.25], np.float32))
    y = N.linear(x, w)
    assert y[0, 0] == (5 - 12 - 21 + 32) * 0.5 * 2.0
    assert y[0, 1] == (1 + 2 - 3 + 4) * 0.5 * 0.25

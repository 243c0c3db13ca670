"""Pins for the oracle's decoy fill of free pages.

Checked against things other than the decoy code itself: the sequential
SplitMix64 stream of ``oracle.prng`` (pure Python integers), a pure-Python
piece sum, the moments of the Irwin-Hall(12) law the sum follows, the E4M3 and
bf16 encoders' own pins, and the layout's page bookkeeping.
"""

import numpy as np
import pytest

from oracle import decoy as OD
from oracle import layout as OL
from oracle import numerics as ON
from oracle import prng
from oracle import remap as OR


@pytest.mark.parametrize("seed,v", [(1, 0), (0xDEC0, 17), ((1 << 64) - 1, (1 << 32) - 1)])
def test_counter_words_are_the_sequential_stream(seed, v):
    g = prng.substream(seed, 7, v)
    want = [g.next_u64() for _ in range(40)]
    assert [int(x) for x in OD.stream_words(seed, v, 40)] == want


def test_mix64_vectorised_equals_integer_definition():
    rng = np.random.Generator(np.random.PCG64(3))
    z = rng.integers(0, 1 << 63, 200, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    assert [int(x) for x in OD.mix64_np(z)] == [prng.mix64(int(x)) for x in z]


def test_centred_sums_by_shifting_the_words():
    seed, v, n = 99, 5, 50
    g = prng.substream(seed, 7, v)
    want = []
    for _ in range(n):
        s = 0
        for _ in range(3):
            w = g.next_u64()
            s += sum((w >> (16 * i)) & 0xFFFF for i in range(4))
        want.append(2 * s - 786420)
    assert list(OD.centred_sums(seed, v, n)) == want


def test_moments_follow_irwin_hall_12():
    # sum of twelve U{0..65535}: var(S) = 12 * (65536^2 - 1) / 12; C = 2S - 786420
    c = OD.centred_sums(2024, 3, 1 << 19).astype(np.float64)
    sd = 2.0 * np.sqrt(65536.0 ** 2 - 1)
    assert abs(c.mean()) < 4 * sd / np.sqrt(c.size)
    assert abs(c.std() / sd - 1) < 0.005
    # excess kurtosis of Irwin-Hall(n) is -6 / (5 n) = -0.1
    k = np.mean((c / c.std()) ** 4) - 3
    assert abs(k + 0.1) < 0.03
    assert np.all(c % 2 == 0) and np.max(np.abs(c)) <= 786420


def test_bf16_f32_and_fp8_pages():
    B = 1 << 16
    f = OD.decoy_page(7, 40, B, "f32").view(np.float32)
    c = OD.centred_sums(7, 40, B // 4)
    assert np.array_equal(f, (c * 5).astype(np.float64) * 2.0 ** -25)       # exact in binary32
    assert abs(f.std() - 5 / 256) < 5e-4
    b = OD.decoy_page(7, 40, B, "bf16").view(np.uint16)
    cb = OD.centred_sums(7, 40, B // 2)
    assert np.array_equal(b, ON.f32_to_bf16_bits_rne(((cb * 5) * 2.0 ** -25).astype(np.float32)))
    q = OD.decoy_page(7, 40, B, "fp8")
    vals = ON.e4m3_bits_to_f64(q)
    cq = OD.centred_sums(7, 40, B)
    exact = cq * 3 * 2.0 ** -12
    # nearest code: no E4M3 value lies strictly closer than the chosen one
    assert np.all(np.abs(vals - np.clip(exact, -448, 448)) <= np.abs(exact) * 2.0 ** -4 + 2.0 ** -10)
    assert 85 < vals.std() < 105 and abs(vals.mean()) < 2
    assert np.mean(np.abs(vals) == 448) < 1e-4


def test_dtype_rule():
    S = OL.Shape
    lay = OL.build_layout(1, [S(0, "gate", 64, 64, "bf16"), S(1, "gate", 64, 128, "fp8")], 1024, 1024 * 64)
    assert OD.decoy_dtype(lay) == "fp8"                      # 8192 B each: tie goes to fp8
    lay = OL.build_layout(1, [S(0, "gate", 64, 64, "bf16"), S(1, "gate", 64, 64, "fp8")], 1024, 1024 * 64)
    assert OD.decoy_dtype(lay) == "bf16"
    lay = OL.build_layout(1, [S(0, "gate", 64, 64, "f32")], 1024, 1024 * 64)
    assert OD.decoy_dtype(lay) == "f32"
    assert OD.decoy_dtype(OL.build_layout(1, [], 1024, 1024 * 8)) == "bf16"


def test_fill_touches_exactly_the_free_pages_and_follows_remap():
    shapes = [OL.Shape(0, "gate", 40, 200, "bf16"), OL.Shape(0, "up", 40, 200, "bf16"),
              OL.Shape(0, "down", 200, 40, "bf16")]
    B, P = 1024, 64
    lay = OL.build_layout(11, shapes, B, B * P)
    rng = np.random.Generator(np.random.PCG64(1))
    ws = [rng.integers(0, 1 << 16, (s.n_out, s.k_in), dtype=np.uint16) for s in shapes]
    plain = OL.pack(lay, ws)
    pool = OD.fill_decoys(lay, plain.copy(), 555)
    free = {lay.phi[v] for v in range(lay.V, lay.P)}
    for p in range(P):
        same = np.array_equal(pool[p * B:(p + 1) * B], plain[p * B:(p + 1) * B])
        assert same == (p not in free), p
        if p in free:
            assert np.count_nonzero(pool[p * B:(p + 1) * B]) > B // 2
    for t in range(len(shapes)):
        assert np.array_equal(OL.unpack(lay, pool, t), ws[t])
    # a remap moves decoys with their pages: refilling under the new map changes nothing
    pool2, phi2 = OR.remap(pool, lay.phi, 4242, B)
    lay2 = OL.Layout(**{**lay.__dict__, "phi": phi2})
    assert np.array_equal(OD.fill_decoys(lay2, pool2.copy(), 555), pool2)
    # another decoy seed, other bytes; the layout seed plays no part
    other = OD.fill_decoys(lay, plain.copy(), 556)
    assert not np.array_equal(other, pool)
    lay_b = OL.build_layout(12, shapes, B, B * P)
    v = lay.V
    assert np.array_equal(OD.decoy_page(555, v, B, "bf16"),
                          OD.fill_decoys(lay_b, OL.pack(lay_b, ws), 555)[lay_b.phi[v] * B:(lay_b.phi[v] + 1) * B])

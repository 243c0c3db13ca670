"""Pins for the oracle's attention-head permutation (intra-layer shuffle of q/k/v/o).

The paper names intra-layer shuffling without a mechanism (abstract); the
reading extends the FFN hidden-neuron permutation to attention: key/value head
groups, query heads inside a group and value dimensions inside a head are
permuted.  What fixes it independently of the code under test: the attention
function must not change (checked in FP64 through the decoder definition on
stored weights), rotary dimensions must stay in place, every map must be a
bijection, and layouts without head sizes must not change at all.
"""

import numpy as np
import pytest

from oracle import layout as L
from oracle import model as OM
from oracle import prng


def attn_shapes(d_model, n_q, n_kv, hd, layers=1, dtype="f32", head_dim=None, ffn=24):
    hd_tag = hd if head_dim is None else head_dim
    out = []
    for l in range(layers):
        out += [L.Shape(l, "q", n_q * hd, d_model, dtype, hd_tag),
                L.Shape(l, "k", n_kv * hd, d_model, dtype, hd_tag),
                L.Shape(l, "v", n_kv * hd, d_model, dtype, hd_tag),
                L.Shape(l, "o", d_model, n_q * hd, dtype, hd_tag),
                L.Shape(l, "gate", ffn, d_model, dtype), L.Shape(l, "up", ffn, d_model, dtype),
                L.Shape(l, "down", d_model, ffn, dtype)]
    return out


GEOMS = [(64, 8, 2, 8), (48, 4, 4, 12), (32, 4, 1, 8), (96, 6, 3, 16)]   # d_model, Hq, Hkv, hd


@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("seed", [3, 0xFEED, (1 << 64) - 5])
def test_head_maps_are_bijections_and_keep_rotary_dims(geom, seed):
    D, Hq, Hkv, hd = geom
    G = Hq // Hkv
    lay = L.build_layout(seed, attn_shapes(D, Hq, Hkv, hd, layers=2), 4096, 4096 * 128)
    for l in range(2):
        t = {k: 7 * l + i for i, k in enumerate(("q", "k", "v", "o"))}
        q, k, v = (lay.row_perm(t[x]) for x in ("q", "k", "v"))
        o = lay.col_perm(t["o"])
        assert sorted(q) == list(range(Hq * hd)) and sorted(o) == list(range(Hq * hd))
        assert sorted(k) == list(range(Hkv * hd)) and sorted(v) == list(range(Hkv * hd))
        assert lay.col_perm(t["q"]) is None and lay.row_perm(t["o"]) is None
        for j in range(Hq * hd):
            # rotary pairs (i, i + hd/2) are defined inside a head: q keeps its dims
            assert q[j] % hd == j % hd
            # the query head in stored slot j // hd reads stored kv head (j // hd) // G,
            # which must hold the logical kv head of its logical query head
            assert (q[j] // hd) // G == k[((j // hd) // G) * hd] // hd
            # o's column follows the query head and the value dimension
            assert o[j] // hd == q[j] // hd
            assert o[j] % hd == v[((j // hd) // G) * hd + j % hd] % hd
        for j in range(Hkv * hd):
            assert k[j] % hd == j % hd
            assert k[j] // hd == v[j] // hd


def test_head_draw_order_and_nontrivial():
    D, Hq, Hkv, hd = 64, 8, 2, 8
    lay = L.build_layout(11, attn_shapes(D, Hq, Hkv, hd), 4096, 4096 * 128)
    a = lay.heads[0]
    g = prng.substream(11, 6, 0)
    assert a["rho"] == prng.fisher_yates(Hkv, g)
    assert a["theta"] == [prng.fisher_yates(4, g) for _ in range(Hkv)]
    assert a["chi"] == prng.fisher_yates(hd, g)
    assert lay.row_perm(0) != list(range(Hq * hd))
    assert lay.row_perm(2) != list(range(Hkv * hd))


def test_identity_layout_keeps_heads_in_place():
    lay = L.build_layout(5, attn_shapes(64, 8, 2, 8), 4096, 4096 * 128, identity=True)
    assert lay.row_perm(0) == list(range(64)) and lay.col_perm(3) == list(range(64))
    assert lay.row_perm(2) == list(range(16))


def test_zero_head_dim_leaves_every_draw_unchanged():
    a = L.build_layout(21, attn_shapes(64, 8, 2, 8), 4096, 4096 * 128)
    b = L.build_layout(21, attn_shapes(64, 8, 2, 8, head_dim=0), 4096, 4096 * 128)
    assert (a.sigma, a.pi, a.phi, a.vbase) == (b.sigma, b.pi, b.phi, b.vbase)
    assert b.heads == {} and all(b.row_perm(t) is None for t in range(4))
    w = np.arange(64 * 64, dtype=np.float32).reshape(64, 64)
    assert np.array_equal(L.shuffle_tensor(b, 0, w), w)


def _weights(shapes, rng):
    return [rng.standard_normal((s.n_out, s.k_in)) for s in shapes]


def _decoder(shapes, ws, D, Hq, Hkv, hd, vocab, rng):
    w = {(s.layer, s.kind): x for s, x in zip(shapes, ws)}
    w[(-1, "embed")] = rng.standard_normal((vocab, D))
    w[(-1, "head")] = rng.standard_normal((vocab, D))
    cfg = dict(d_model=D, n_heads=Hq, n_kv_heads=Hkv, head_dim=hd, d_ffn=24, vocab=vocab,
               n_layers=max(s.layer for s in shapes) + 1, theta=10000.0, eps=1e-5)
    return cfg, w


@pytest.mark.parametrize("geom", GEOMS)
def test_decoder_cannot_see_the_permutation(geom):
    # The FP64 decoder run directly on the stored (permuted) arrays, i.e. with
    # attention in stored head order and the FFN in stored hidden order, gives
    # the logits of the logical model.
    D, Hq, Hkv, hd = geom
    rng = np.random.Generator(np.random.PCG64(sum(geom)))
    shapes = attn_shapes(D, Hq, Hkv, hd, layers=2)
    lay = L.build_layout(0xC10A4, shapes, 4096, 4096 * 128)
    ws = _weights(shapes, rng)
    cfg, w = _decoder(shapes, ws, D, Hq, Hkv, hd, 40, rng)
    stored = dict(w)
    for t, s in enumerate(shapes):
        stored[(s.layer, s.kind)] = L.shuffle_tensor(lay, t, ws[t])
    toks = [3, 17, 5, 39, 0, 22]
    ref = OM.DecoderFP64(cfg, w).forward(toks)
    got = OM.DecoderFP64(cfg, stored).forward(toks)
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))
    # and a plausible mistake is visible: o left in logical column order
    bad = dict(stored)
    bad[(0, "o")] = w[(0, "o")]
    assert np.max(np.abs(OM.DecoderFP64(cfg, bad).forward(toks) - ref)) > 1e-3


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_pack_unpack_round_trip_with_heads(dtype):
    shapes = attn_shapes(64, 8, 2, 8, layers=2, dtype=dtype)
    lay = L.build_layout(9, shapes, 4096, 4096 * 128)
    rng = np.random.Generator(np.random.PCG64(4))
    st = L.STORAGE_DTYPE[dtype]
    ws = [rng.integers(0, 1 << 16, (s.n_out, s.k_in)).astype(st) if dtype != "f32"
          else rng.standard_normal((s.n_out, s.k_in)).astype(np.float32) for s in shapes]
    pool = L.pack(lay, ws)
    for t in range(len(shapes)):
        assert np.array_equal(L.unpack(lay, pool, t).view(np.uint8), np.ascontiguousarray(ws[t]).view(np.uint8))


def test_scales_follow_q_k_v_rows():
    shapes = attn_shapes(64, 8, 2, 8, dtype="fp8")
    lay = L.build_layout(13, shapes, 4096, 4096 * 128)
    for t, s in enumerate(shapes[:4]):
        sc = np.arange(s.n_out, dtype=np.float32)
        got = L.shuffle_scales(lay, t, sc)
        rp = lay.row_perm(t)
        assert np.array_equal(got, sc if rp is None else sc[rp])
    assert np.array_equal(L.shuffle_scales(lay, 3, np.arange(64, dtype=np.float32)), np.arange(64))


def test_head_layout_errors():
    base = attn_shapes(64, 8, 2, 8)
    with pytest.raises(ValueError):                         # k without a head size
        L.build_layout(1, [base[0], L.Shape(0, "k", 16, 64, "f32"), base[2], base[3]], 4096, 4096 * 128)
    with pytest.raises(ValueError):                         # missing v
        L.build_layout(1, [base[0], base[1], base[3]], 4096, 4096 * 128)
    with pytest.raises(ValueError):                         # head sizes disagree
        L.build_layout(1, [base[0], L.Shape(0, "k", 16, 64, "f32", 4), base[2], base[3]], 4096, 4096 * 128)
    with pytest.raises(ValueError):                         # 3 query heads over 2 kv heads
        L.build_layout(1, attn_shapes(64, 3, 2, 8), 4096, 4096 * 128)
    with pytest.raises(ValueError):                         # o's K is not q's N
        L.build_layout(1, base[:3] + [L.Shape(0, "o", 64, 56, "f32", 8)], 4096, 4096 * 128)
    with pytest.raises(ValueError):                         # head size on an FFN tensor
        L.Shape(0, "gate", 8, 8, "f32", 8)
    neg = [L.Shape(-2, s.kind, s.n_out, s.k_in, s.dtype, s.head_dim) for s in base[:4]]
    with pytest.raises(ValueError):
        L.build_layout(1, neg, 4096, 4096 * 128)

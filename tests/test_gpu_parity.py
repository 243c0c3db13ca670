"""GPU parity of the cloaked path against the CPU oracle (MI355X, via the C-ABI).

Bit-exact: pool bytes after upload, read-back, remap, one-hot probes through
the GEMV and the cloaked-vs-native comparison of tensors whose K is not
permuted.  Normwise tolerance against FP64 (max|y-y*| / max|y*|): 1e-5 for
f32, 1e-2 for bf16, 5e-2 for FP8.
"""

import numpy as np
import pytest

from cloak_cases import (TOL, act_dtype, decoder_shapes, from_device, make_weights, oracle_layout, to_device_x,
                         values_f64, w64)
from oracle import layout as OL
from oracle import numerics as ON
from oracle import remap as OR
from paper_2606_18400_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    import torch
    assert torch.cuda.is_available()
    from paper_2606_18400_amd import cloak
    return cloak


def pool_bytes_of(cw):
    return cw.pool.cpu().numpy()


# rows of 272 elements (544 B bf16, 1088 B f32, 272 B fp8) and hidden sizes 80/48:
# no row is a multiple of 1 KiB, so 1 KiB wave loads cross page boundaries
RAGGED = [(0, "q", 40, 272, None), (0, "gate", 80, 272, None), (0, "up", 80, 272, None),
          (0, "down", 272, 80, None), (1, "gate", 48, 272, None), (1, "up", 48, 272, None),
          (1, "down", 272, 48, None), (-1, "head", 50, 272, None)]


def ragged_shapes(dtype):
    return [(l, k, n, kk, dtype) for (l, k, n, kk, _) in RAGGED]


# a head-permuted attention block on the same 272-wide rows: 8 query heads of
# 12 over 2 kv heads
def ragged_heads(dtype, layer=3):
    return [(layer, "q", 96, 272, dtype, 12), (layer, "k", 24, 272, dtype, 12), (layer, "v", 24, 272, dtype, 12),
            (layer, "o", 272, 96, dtype, 12)]


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("page_bytes", [1024, 65536])
def test_upload_pool_bytes_and_readback_bit_exact(C, dtype, page_bytes):
    shapes = ragged_shapes(dtype) + ragged_heads(dtype)
    pool = page_bytes * (1024 if page_bytes == 1024 else 32)
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, page_bytes, pool, seed=7)
    cw.load(ws, scs)
    lay = oracle_layout(7, shapes, page_bytes, pool)
    assert np.array_equal(pool_bytes_of(cw), OL.pack(lay, ws))
    for t, w in enumerate(ws):
        back = np.zeros_like(w)
        C.cloak_unload(cw.layout, cw.pool, t, back)
        assert np.array_equal(back.view(np.uint8), w.view(np.uint8))
    cw.close()


def test_upload_order_is_kept_by_the_library(C):
    """cloak_load refuses a first upload out of the tensor order; cloak_load_all
    sends every tensor in that order and gives the oracle's pool bytes; a
    tensor already uploaded may be sent again."""
    import torch
    shapes = decoder_shapes(512, 1024, 128, "bf16", layers=2)
    B, P = 65536, 256
    ws, scs = make_weights(shapes)
    lay_c = C.cloak_layout_build(11, shapes, B, B * P)
    C.cloak_layout_to_device(lay_c)
    pool = torch.empty(B * P, dtype=torch.uint8, device="cuda")
    C.cloak_pool_init(lay_c, pool)
    sigma = list(C.cloak_query(lay_c, "SIGMA"))
    t_bad = next(t for t in range(len(shapes)) if t != sigma[0])
    with pytest.raises(C.CloakError) as e:
        C.cloak_load(lay_c, pool, t_bad, ws[t_bad])
    assert e.value.code == C.CLOAK_ESTATE
    torch.cuda.synchronize()
    assert not pool.any().item(), "a refused upload must not write the pool"
    C.cloak_load_all(lay_c, pool, ws)
    lay = oracle_layout(11, shapes, B, B * P)
    assert np.array_equal(pool.cpu().numpy(), OL.pack(lay, ws))
    C.cloak_load(lay_c, pool, t_bad, ws[t_bad])     # a second upload is allowed in any order
    assert np.array_equal(pool.cpu().numpy(), OL.pack(lay, ws))
    C.cloak_layout_free(lay_c)


@pytest.mark.parametrize("uniform", [False, True])
def test_remap_on_device_matches_oracle_and_keeps_results(C, uniform):
    import torch
    shapes = decoder_shapes(512, 1024, 128, "bf16", layers=2)
    B, P = 65536, 257   # odd pool: one page keeps its place in every matching remap
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, B, B * P, seed=3, flags=C.CLOAK_REMAP_UNIFORM if uniform else 0)
    cw.load(ws, scs)
    lay = oracle_layout(3, shapes, B, B * P)
    pool, phi = OL.pack(lay, ws), lay.phi
    x = to_device_x(synth.activations(5, 512, "bf16"))
    before = [cw.linear(t, x).clone() for t in range(len(shapes)) if shapes[t][3] == 512]
    mlp_before = cw.mlp(0, x).clone()
    for rs in (1, 2, 99):
        cw.remap(rs)
        pool, phi = (OR.remap_uniform if uniform else OR.remap)(pool, phi, rs, B)
    torch.cuda.synchronize()
    assert list(C.cloak_query(cw.layout, "PHI")) == phi
    assert np.array_equal(pool_bytes_of(cw), pool)
    after = [cw.linear(t, x) for t in range(len(shapes)) if shapes[t][3] == 512]
    for a, b in zip(before, after):
        assert torch.equal(a.view(torch.int16), b.view(torch.int16))
    assert torch.equal(mlp_before.view(torch.int16), cw.mlp(0, x).view(torch.int16))
    cw.close()


@pytest.mark.parametrize("uniform", [False, True])
def test_incremental_remap_on_device_matches_oracle_slices(C, uniform):
    import torch
    shapes = decoder_shapes(512, 1024, 128, "bf16", layers=2)
    B, P = 65536, 257
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, B, B * P, seed=3, flags=C.CLOAK_REMAP_UNIFORM if uniform else 0)
    cw.load(ws, scs)
    lay = oracle_layout(3, shapes, B, B * P)
    x = to_device_x(synth.activations(5, 512, "bf16"))
    before = [cw.linear(t, x).clone() for t in range(len(shapes)) if shapes[t][3] == 512]
    mlp_before = cw.mlp(1, x).clone()
    cw.remap_begin(606)
    slices = OR.remap_uniform_in_slices if uniform else OR.remap_in_slices
    states = list(slices(OL.pack(lay, ws), lay.phi, 606, B, 13))
    for k, (pool_k, phi_k) in enumerate(states):
        left = cw.remap_step(13)
        # results between slices are those of the untouched layout
        after = [cw.linear(t, x) for t in range(len(shapes)) if shapes[t][3] == 512]
        for a, b in zip(before, after):
            assert torch.equal(a.view(torch.int16), b.view(torch.int16)), k
        assert torch.equal(mlp_before.view(torch.int16), cw.mlp(1, x).view(torch.int16)), k
        if k in (0, len(states) // 2, len(states) - 1):
            torch.cuda.synchronize()
            assert list(C.cloak_query(cw.layout, "PHI")) == phi_k
            assert np.array_equal(pool_bytes_of(cw), pool_k)
    assert left == 0 and C.cloak_query(cw.layout, "REMAPS") == 1
    with pytest.raises(C.CloakError) as e:
        cw.remap_step(1)
    assert e.value.code == C.CLOAK_ESTATE
    cw.close()


def test_vmm_twin_matches_software_translation(C):
    """The same layout read through the MMU (pages mapped in phi order,
    untranslated kernels) and through the in-kernel page map gives
    bit-identical results, before and after whole and sliced remaps."""
    import torch
    shapes = decoder_shapes(1024, 2816, 256, "bf16", layers=1, extra=[(-1, "head", 1000, 1024, "bf16")])
    B, P = 2 << 20, 24
    ws, scs = make_weights(shapes)
    soft = C.CloakedWeights(shapes, B, B * P, seed=61)
    try:
        hard = C.CloakedWeights(shapes, B, B * P, seed=61, vmm=True)
    except C.CloakError as e:
        soft.close()
        pytest.skip(f"no virtual memory management: {e}")
    soft.load(ws, scs)
    hard.load(ws, scs)

    def same_results(tag):
        for M in (1, 8, 300):
            for t, s in enumerate(shapes):
                x = to_device_x(synth.activations(M, s[3], "bf16", seed=t))
                a, b = soft.linear(t, x), hard.linear(t, x)
                assert torch.equal(a.view(torch.int16), b.view(torch.int16)), (tag, M, s)
            x = to_device_x(synth.activations(M, 1024, "bf16", seed=71))
            assert torch.equal(soft.mlp(0, x).view(torch.int16), hard.mlp(0, x).view(torch.int16)), (tag, M)

    same_results("loaded")
    for M in (1, 8, 300):     # the MMU-translated twin against the oracle itself
        check_linear_all(C, hard, shapes, ws, scs, M)
    for t, w in enumerate(ws):
        back = np.zeros_like(w)
        C.cloak_unload(hard.layout, hard.pool, t, back)
        assert np.array_equal(back.view(np.uint8), w.view(np.uint8))
    soft.remap(5)
    hard.remap(5)
    same_results("remapped")
    check_linear_all(C, hard, shapes, ws, scs, 8)
    soft.remap_begin(6)
    hard.remap_begin(6)
    while soft.remap_step(3):
        hard.remap_step(3)
    hard.remap_step(3)
    assert C.cloak_query(hard.layout, "REMAP_PENDING") == 0
    same_results("sliced remap")
    assert list(C.cloak_query(hard.layout, "PHI")) == list(C.cloak_query(soft.layout, "PHI"))
    soft.close()
    hard.close()


def check_linear_all(C, cw, shapes, ws, scs, M, xseed=5678):
    """Every tensor through cloak_linear and every FFN through cloak_mlp."""
    dtypes = {s[4] for s in shapes}
    worst = 0.0
    for t, s in enumerate(shapes):
        adt = act_dtype(s[4])
        x_np = synth.activations(M, s[3], adt, seed=xseed + t)
        y = from_device(cw.linear(t, to_device_x(x_np)))
        ref = ON.linear(values_f64(x_np), w64(shapes, ws, scs, t))
        err = ON.normwise_err(values_f64(y), ref)
        worst = max(worst, err)
        assert err <= TOL[s[4]], (t, s, M, err)
    layers = sorted({s[0] for s in shapes if s[1] == "gate"})
    for l in layers:
        ig = next(t for t, s in enumerate(shapes) if s[0] == l and s[1] == "gate")
        iu = next(t for t, s in enumerate(shapes) if s[0] == l and s[1] == "up")
        idn = next(t for t, s in enumerate(shapes) if s[0] == l and s[1] == "down")
        wdt = shapes[ig][4]
        x_np = synth.activations(M, shapes[ig][3], act_dtype(wdt), seed=xseed + 100 + l)
        y = from_device(cw.mlp(l, to_device_x(x_np)))
        ref, _ = ON.swiglu_ffn(values_f64(x_np), w64(shapes, ws, scs, ig), w64(shapes, ws, scs, iu),
                               w64(shapes, ws, scs, idn))
        err = ON.normwise_err(values_f64(y), ref)
        worst = max(worst, err)
        assert err <= TOL[wdt], ("mlp", l, M, err)
    return worst, dtypes


@pytest.mark.parametrize("M", [1, 4])
def test_ffn512_block_f32_vs_fp64(C, M):
    cfg = synth.FFN512
    shapes = synth.ffn_block_shapes(cfg["d_model"], cfg["d_ffn"], "f32")
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, cfg["page_bytes"], cfg["pool_bytes"], seed=1)
    cw.load(ws, scs)
    check_linear_all(C, cw, shapes, ws, scs, M)
    cw.close()


@pytest.mark.parametrize("M", [1, 2, 3, 5, 8, 13])
def test_bf16_layer_vs_fp64(C, M):
    shapes = decoder_shapes(1024, 2816, 256, "bf16", layers=1, extra=[(-1, "head", 1000, 1024, "bf16")])
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 512, seed=11)
    cw.load(ws, scs)
    check_linear_all(C, cw, shapes, ws, scs, M)
    cw.close()


@pytest.mark.parametrize("M", [1, 3, 8])
@pytest.mark.parametrize("dtype", ["bf16", "fp8", "f32"])
def test_ragged_rows_straddling_pages(C, M, dtype):
    shapes = ragged_shapes(dtype)
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 1024, 1024 * 512, seed=5)
    cw.load(ws, scs)
    check_linear_all(C, cw, shapes, ws, scs, M)
    cw.close()


# rows of 17..32 KiB chunks at one token take the 16-wave GEMV layout (the
# down projection of a 14336-wide FFN is one); M = 2 takes the 8-wave one
WIDE = {"bf16": (9216, 8960), "fp8": (27648, 27648), "f32": (4480, 4352)}


@pytest.mark.parametrize("M", [1, 2])
@pytest.mark.parametrize("dtype", ["bf16", "fp8", "f32"])
def test_long_rows_single_token(C, M, dtype):
    dff, kq = WIDE[dtype]
    shapes = [(0, "gate", dff, 256, dtype), (0, "up", dff, 256, dtype), (0, "down", 256, dff, dtype),
              (1, "q", 64, kq, dtype)]
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 1024, seed=47)
    cw.load(ws, scs)
    check_linear_all(C, cw, shapes, ws, scs, M)
    cw.close()


@pytest.mark.parametrize("M", [1, 3])
def test_fp8_two_chunk_waves(C, M):
    # one token over 6144+ FP8 rows of 2..8 KiB takes two chunks per wave
    shapes = [(0, "gate", 3072, 4096, "fp8"), (0, "up", 3072, 4096, "fp8"), (0, "down", 4096, 3072, "fp8"),
              (1, "q", 6400, 2048, "fp8"), (1, "k", 64, 2048, "fp8")]
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 1024, seed=53)
    cw.load(ws, scs)
    check_linear_all(C, cw, shapes, ws, scs, M)
    cw.close()


@pytest.mark.parametrize("M", [1, 2, 4, 8])
def test_fp8_layer_vs_fp64(C, M):
    shapes = decoder_shapes(1280, 3456, 256, "fp8", layers=1, extra=[(-1, "head", 700, 1280, "bf16")])
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 512, seed=13)
    cw.load(ws, scs)
    check_linear_all(C, cw, shapes, ws, scs, M)
    cw.close()


def plus_zero(a):
    """Signed zeros made +0: a dot product whose only nonzero input meets a -0
    weight sums -0 with the +0 products of the other terms, and the IEEE sum
    of zeros of opposite sign is +0 (FP8 weights below half the smallest
    subnormal quantise to -0 as often as to +0)."""
    a = np.array(a)
    if a.dtype == np.float32:
        return np.where(a == 0, np.float32(0), a)
    return np.where(a == 0x8000, np.uint16(0), a).astype(a.dtype)


def one_hot_expected(shapes, ws, scs, t, ks):
    """y[m][n] for x = e_{ks[m]}: the weight itself, rounded like the kernel's output."""
    s = shapes[t]
    if s[4] in ("f32", "bf16"):
        return plus_zero(np.stack([ws[t][:, k] for k in ks]))
    # FP8: acc = e4m3(q) exactly, times the f32 row scale (one f32 rounding), then bf16
    q = ON.e4m3_bits_to_f64(ws[t]).astype(np.float32)
    prod = q * scs[t].astype(np.float32)[:, None]
    return plus_zero(np.stack([ON.f32_to_bf16_bits_rne(prod[:, k]) for k in ks]))


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_one_hot_probes_are_bit_exact(C, dtype):
    shapes = ragged_shapes(dtype) + [(2, "gate", 64, 512, dtype), (2, "up", 64, 512, dtype),
                                     (2, "down", 512, 64, dtype)]
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 1024, 1024 * 1024, seed=21)
    cw.load(ws, scs)
    rng = np.random.Generator(np.random.PCG64(4))
    for t, s in enumerate(shapes):
        K = s[3]
        ks = list(rng.choice(K, size=min(8, K), replace=False))
        ks[0], ks[-1] = 0, K - 1
        if dtype == "f32":
            x = np.zeros((len(ks), K), np.float32)
            for m, k in enumerate(ks):
                x[m, k] = 1.0
        else:
            x = np.zeros((len(ks), K), np.uint16)
            for m, k in enumerate(ks):
                x[m, k] = 0x3F80
        y = plus_zero(from_device(cw.linear(t, to_device_x(x))))
        want = one_hot_expected(shapes, ws, scs, t, ks)
        assert np.array_equal(y.view(np.uint8), want.view(np.uint8)), (t, s)
    cw.close()


def test_cloaked_equals_native_twin(C):
    import torch
    shapes = decoder_shapes(1024, 2816, 256, "bf16", layers=2)
    ws, scs = make_weights(shapes)
    B, P = 65536, 1024
    cl = C.CloakedWeights(shapes, B, B * P, seed=31)
    nat = C.CloakedWeights(shapes, B, B * P, seed=31, flags=C.CLOAK_IDENTITY | C.CLOAK_NATIVE)
    idt = C.CloakedWeights(shapes, B, B * P, seed=31, flags=C.CLOAK_IDENTITY)
    for cw in (cl, nat, idt):
        cw.load(ws, scs)
    assert C.cloak_query(nat.layout, "CONTIGUITY") == 1.0
    assert C.cloak_query(cl.layout, "CONTIGUITY") < 0.05
    for M in (1, 8):
        for t, s in enumerate(shapes):
            x = to_device_x(synth.activations(M, s[3], "bf16", seed=t))
            a, b, c = cl.linear(t, x), nat.linear(t, x), idt.linear(t, x)
            assert torch.equal(b.view(torch.int16), c.view(torch.int16))
            if s[1] == "down":
                err = ON.normwise_err(values_f64(from_device(a)), values_f64(from_device(b)))
                assert err <= 1e-2
            else:
                assert torch.equal(a.view(torch.int16), b.view(torch.int16)), s
        x = to_device_x(synth.activations(M, 1024, "bf16", seed=77))
        err = ON.normwise_err(values_f64(from_device(cl.mlp(1, x))), values_f64(from_device(nat.mlp(1, x))))
        assert err <= 1e-2
    for cw in (cl, nat, idt):
        cw.close()


def test_fused_qkv_equals_separate(C):
    import torch
    shapes = decoder_shapes(1024, 2816, 256, "bf16", layers=1)
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 512, seed=2)
    cw.load(ws, scs)
    x = to_device_x(synth.activations(3, 1024, "bf16"))
    fused = cw.linear_fused([0, 1, 2], x)
    sep = torch.cat([cw.linear(t, x) for t in (0, 1, 2)], dim=1)
    assert torch.equal(fused.view(torch.int16), sep.view(torch.int16))
    # gate and up fused: the scatter through pi applies per tensor
    gu = cw.linear_fused([4, 5], x)
    assert torch.equal(gu.view(torch.int16), torch.cat([cw.linear(4, x), cw.linear(5, x)], 1).view(torch.int16))
    cw.close()


def test_empty_batch_and_argument_errors(C):
    import torch
    shapes = decoder_shapes(512, 1024, 128, "bf16", layers=1)
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 128, seed=4)
    cw.load(ws, scs)
    y = torch.full((1, 512), 7, dtype=torch.int16, device="cuda")
    C.cloak_linear(cw.layout, cw.pool, 0, y, 0, y)     # M = 0: nothing written
    torch.cuda.synchronize()
    assert int(y.min()) == 7 and int(y.max()) == 7
    x = to_device_x(synth.activations(2, 512, "bf16"))
    out = torch.empty((2, 512), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(C.CloakError) as e:
        C.cloak_mlp(cw.layout, cw.pool, 0, x, 2, out, out, 16)   # workspace too small
    assert e.value.code == C.CLOAK_EINVAL
    with pytest.raises(C.CloakError) as e:
        C.cloak_linear_fused(cw.layout, cw.pool, [0, 6], x, 2, out)   # K differs
    assert e.value.code == C.CLOAK_ESHAPE
    with pytest.raises(C.CloakError) as e:
        C.cloak_linear(cw.layout, cw.pool.data_ptr() + 16, 0, x, 2, out)   # misaligned pool
    assert e.value.code == C.CLOAK_EINVAL
    cw.close()
    nat = C.CloakedWeights(shapes, 65536, 65536 * 128, seed=4, flags=C.CLOAK_IDENTITY | C.CLOAK_NATIVE)
    with pytest.raises(C.CloakError) as e:
        nat.remap(1)
    assert e.value.code == C.CLOAK_ESTATE
    nat.close()


# ---------------------------------------------------------------- attention-head permutation

@pytest.mark.parametrize("M", [1, 3, 17, 64, 300])
@pytest.mark.parametrize("dtype", ["bf16", "fp8", "f32"])
def test_head_permuted_layer_vs_fp64(C, dtype, M):
    # q/k/v rows permuted by head (scattered back by the kernels), o's columns
    # permuted (activations gathered); GEMV, skinny MFMA and 256x256 MFMA paths
    if dtype == "f32" and M > 17:
        pytest.skip("f32 weights run the GEMV at every batch size; covered by M <= 17")
    shapes = decoder_shapes(1024, 2816, 256, dtype, layers=1, head_dim=128)
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 1024, seed=41)
    cw.load(ws, scs)
    lay = oracle_layout(41, shapes, 65536, 65536 * 1024)
    assert lay.row_perm(0) != list(range(1024)) and lay.col_perm(3) != list(range(1024))
    check_linear_all(C, cw, shapes, ws, scs, M)
    cw.close()


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_head_permuted_one_hot_bit_exact(C, dtype):
    # the scatter of q/k/v rows and the gather of o's activations are exact:
    # a one-hot x returns the logical weight column itself
    shapes = ragged_heads(dtype, layer=0)
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 1024, 1024 * 256, seed=43)
    cw.load(ws, scs)
    for t, s in enumerate(shapes):
        K = s[3]
        ks = [0, 5, 13, K // 2, K - 1]
        if dtype == "f32":
            x = np.zeros((len(ks), K), np.float32)
            for m, k in enumerate(ks):
                x[m, k] = 1.0
        else:
            x = np.zeros((len(ks), K), np.uint16)
            for m, k in enumerate(ks):
                x[m, k] = 0x3F80
        y = plus_zero(from_device(cw.linear(t, to_device_x(x))))
        assert np.array_equal(y.view(np.uint8), one_hot_expected(shapes, ws, scs, t, ks).view(np.uint8)), (t, s)
    cw.close()


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
@pytest.mark.parametrize("M", [1, 3, 40, 300])
def test_linear_stored_is_the_permuted_logical_result(C, M, dtype):
    # stored-order calls do the same products: q/k/v results are the logical
    # ones with columns in stored row order; o fed stored-order x equals o
    # fed logical x through the gather (bit for bit; FP8 at 300 tokens quantises
    # the activations per token, which a column permutation does not change)
    import torch
    shapes = decoder_shapes(1024, 2816, 256, dtype, layers=1, head_dim=128)
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 512, seed=47)
    cw.load(ws, scs)
    L = cw.layout
    x = to_device_x(synth.activations(M, 1024, "bf16", seed=M))
    need = C.cloak_linear_fused_ws_bytes(L, [0, 1, 2], M) + C.cloak_ws_bytes(L, C.CLOAK_OP_LINEAR, 3, M) + 256
    ws_t = torch.empty(need, dtype=torch.uint8, device="cuda")
    y_st = torch.empty((M, 1536), dtype=torch.bfloat16, device="cuda")
    C.cloak_linear_stored(L, cw.pool, [0, 1, 2], x, M, y_st, ws_t, need)
    y_lg = cw.linear_fused([0, 1, 2], x)
    perm = np.concatenate([C.cloak_query(L, "ROW_PERM", 0), 1024 + C.cloak_query(L, "ROW_PERM", 1),
                           1280 + C.cloak_query(L, "ROW_PERM", 2)])
    assert torch.equal(y_st.view(torch.int16), y_lg[:, torch.from_numpy(perm).long().cuda()].view(torch.int16))
    cp = torch.from_numpy(C.cloak_query(L, "COL_PERM", 3).astype(np.int64)).cuda()
    o_st = torch.empty((M, 1024), dtype=torch.bfloat16, device="cuda")
    C.cloak_linear_stored(L, cw.pool, [3], x[:, cp].contiguous(), M, o_st, ws_t, need)
    assert torch.equal(o_st.view(torch.int16), cw.linear(3, x).view(torch.int16))
    cw.close()


def test_head_permuted_qkv_equals_native(C):
    # q/k/v keep K in place: scattered results are bit-identical to the
    # contiguous comparator; fused q/k/v equals the three separate calls
    import torch
    shapes = decoder_shapes(1024, 2816, 256, "bf16", layers=1, head_dim=128)
    ws, scs = make_weights(shapes)
    B, P = 65536, 512
    cl = C.CloakedWeights(shapes, B, B * P, seed=45)
    nat = C.CloakedWeights(shapes, B, B * P, seed=45, flags=C.CLOAK_IDENTITY | C.CLOAK_NATIVE)
    for cw in (cl, nat):
        cw.load(ws, scs)
    for M in (1, 8, 40, 300):
        x = to_device_x(synth.activations(M, 1024, "bf16", seed=M))
        fused = cl.linear_fused([0, 1, 2], x)
        sep = torch.cat([cl.linear(t, x) for t in (0, 1, 2)], dim=1)
        assert torch.equal(fused.view(torch.int16), sep.view(torch.int16))
        assert torch.equal(fused.view(torch.int16), nat.linear_fused([0, 1, 2], x).view(torch.int16)), M
        err = ON.normwise_err(values_f64(from_device(cl.linear(3, x))), values_f64(from_device(nat.linear(3, x))))
        assert err <= 1e-2
    for cw in (cl, nat):
        cw.close()


# ---------------------------------------------------------------- cryptographic layout streams

def test_csprng_layout_on_device(C):
    # draws from counter-mode SHA-256: same kernels, other placement
    shapes = ragged_shapes("bf16") + ragged_heads("bf16")
    B, P = 1024, 1024
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, B, B * P, seed=77, flags=C.CLOAK_CSPRNG)
    cw.load(ws, scs)
    lay = OL.build_layout(77, [OL.Shape(*s) for s in shapes], B, B * P, csprng=True)
    assert np.array_equal(pool_bytes_of(cw), OL.pack(lay, ws))
    check_linear_all(C, cw, shapes, ws, scs, 3)
    pool2, phi2 = OR.remap(pool_bytes_of(cw), lay.phi, 5, B, csprng=True)
    cw.remap(5)
    assert np.array_equal(pool_bytes_of(cw), pool2)
    assert list(C.cloak_query(cw.layout, "PHI")) == phi2
    cw.close()


# ---------------------------------------------------------------- masked device page map

@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_masked_map_table_and_results(C, dtype):
    # the device table holds phi XOR the keyed mask, re-keyed by every upload;
    # results are bit-identical to the plain map (same pages, same kernels)
    import torch
    shapes = decoder_shapes(1024, 2816, 256, dtype, layers=1, head_dim=128,
                            extra=[(-1, "head", 1000, 1024, dtype)])
    B, P = 65536, 512
    ws, scs = make_weights(shapes)
    plain = C.CloakedWeights(shapes, B, B * P, seed=51)
    mask = C.CloakedWeights(shapes, B, B * P, seed=51, flags=C.CLOAK_MASKED_MAP)
    for cw in (plain, mask):
        cw.load(ws, scs)
    keys = OL.map_keys(51)
    lay = oracle_layout(51, shapes, B, B * P)
    k = next(keys)
    assert C.cloak_query(mask.layout, "MAP_KEY") == k and C.cloak_query(plain.layout, "MAP_KEY") == 0
    assert list(C.cloak_device_map_read(mask.layout)) == OL.masked_map(lay.phi, k)
    assert list(C.cloak_device_map_read(plain.layout)) == lay.phi

    def same_results():
        for M in (1, 3, 40, 300):
            for t, s in enumerate(shapes):
                x = to_device_x(synth.activations(M, s[3], "bf16", seed=t + M))
                assert torch.equal(mask.linear(t, x).view(torch.int16), plain.linear(t, x).view(torch.int16)), (t, M)
            x = to_device_x(synth.activations(M, 1024, "bf16", seed=M))
            assert torch.equal(mask.mlp(0, x).view(torch.int16), plain.mlp(0, x).view(torch.int16))

    same_results()
    # a remap in three slices: every slice uploads the map under the next key
    phi = lay.phi
    slices = list(OR.remap_in_slices(pool_bytes_of(plain), phi, 808, B, (P // 2 + 2) // 3))
    for cw in (plain, mask):
        cw.remap_begin(808)
    for pool_i, phi_i in slices:
        for cw in (plain, mask):
            C.cloak_remap_step(cw.layout, cw.pool, (P // 2 + 2) // 3)
        k = next(keys)
        assert C.cloak_query(mask.layout, "MAP_KEY") == k
        assert list(C.cloak_device_map_read(mask.layout)) == OL.masked_map(phi_i, k)
        assert np.array_equal(pool_bytes_of(mask), pool_i)
        same_results()
    for cw in (plain, mask):
        cw.close()


# ---------------------------------------------------------------- decoy fill of free pages

@pytest.mark.parametrize("dtype,page_bytes", [("f32", 1024), ("bf16", 1024), ("fp8", 1024), ("bf16", 65536),
                                              ("fp8", 65536)])
def test_decoy_pool_bit_exact_and_results_unchanged(C, dtype, page_bytes):
    import torch
    from oracle import decoy as OD
    shapes = ragged_shapes(dtype) + ragged_heads(dtype)
    pool = page_bytes * (1024 if page_bytes == 1024 else 48)
    ws, scs = make_weights(shapes)
    plain = C.CloakedWeights(shapes, page_bytes, pool, seed=7)
    dec = C.CloakedWeights(shapes, page_bytes, pool, seed=7, decoy=0xD1CE)
    for cw in (plain, dec):
        cw.load(ws, scs)
    lay = oracle_layout(7, shapes, page_bytes, pool)
    assert lay.P - lay.V >= 10
    assert np.array_equal(pool_bytes_of(dec), OD.fill_decoys(lay, OL.pack(lay, ws), 0xD1CE))
    for M in (1, 40):
        for t, s in enumerate(shapes):
            x = to_device_x(synth.activations(M, s[3], act_dtype(dtype), seed=t))
            a, b = dec.linear(t, x), plain.linear(t, x)
            assert torch.equal(a.view(torch.int8), b.view(torch.int8)), (t, s, M)
    # a remap carries the decoys with their pages (whole-pool bytes vs the oracle)
    pool2, phi2 = OR.remap(pool_bytes_of(dec), lay.phi, 99, page_bytes)
    dec.remap(99)
    assert np.array_equal(pool_bytes_of(dec), pool2)
    assert list(C.cloak_query(dec.layout, "PHI")) == phi2
    # decoys written again after the remap land on the same bytes
    C.cloak_pool_decoy(dec.layout, dec.pool, 0xD1CE)
    assert np.array_equal(pool_bytes_of(dec), pool2)
    for cw in (plain, dec):
        cw.close()


def test_decoy_full_size_pages_sampled(C):
    # 2 MiB pages over a 1 GiB pool holding one 4096/14336 BF16 layer (208
    # pages): the 304 free pages carry decoys; sampled pages checked whole
    import time
    import torch
    from oracle import decoy as OD
    shapes = decoder_shapes(4096, 14336, 1024, "bf16", layers=1)
    B, P = 2 << 20, 512
    cw = C.CloakedWeights(shapes, B, B * P, seed=3)
    lay = oracle_layout(3, shapes, B, B * P)
    assert lay.V == 208
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    C.cloak_pool_decoy(cw.layout, cw.pool, 12345)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"decoy fill: {(P - lay.V) * B / dt / 1e9:.1f} GB/s over {P - lay.V} pages")
    rng = np.random.Generator(np.random.PCG64(8))
    for v in [lay.V, P - 1] + list(rng.choice(np.arange(lay.V + 1, P - 1), 4, replace=False)):
        p = lay.phi[v]
        got = cw.pool[p * B:(p + 1) * B].cpu().numpy()
        assert np.array_equal(got, OD.decoy_page(12345, int(v), B, "bf16")), v
    # tensor pages stay zero (nothing loaded)
    p = lay.phi[0]
    assert int(cw.pool[p * B:(p + 1) * B].count_nonzero()) == 0
    cw.close()


# ---------------------------------------------------------------- prefill GEMM (MFMA)

@pytest.mark.parametrize("M", [17, 32, 64, 100, 200, 256, 300, 600])
def test_prefill_gemm_vs_fp64(C, M):
    # 5..256 tokens: skinny split-K MFMA GEMM; above: the 256x256 MFMA GEMM
    # K = 1024 / 2816 (multiples of 64): the BF16 MFMA GEMM path; N = 1000 and
    # d_ffn 2816 leave ragged row tiles, M leaves ragged token tiles
    shapes = decoder_shapes(1024, 2816, 256, "bf16", layers=1, extra=[(-1, "head", 1000, 1024, "bf16")])
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 512, seed=17)
    cw.load(ws, scs)
    check_linear_all(C, cw, shapes, ws, scs, M)
    cw.close()


@pytest.mark.parametrize("M", [40, 200, 300])
def test_prefill_gemm_one_hot_bit_exact(C, M):
    # 40 and 200 tokens: skinny split-K kernel; 300: the 256x256 GEMM
    import torch
    shapes = decoder_shapes(1024, 2816, 256, "bf16", layers=1)
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 512, seed=19)
    cw.load(ws, scs)
    rng = np.random.Generator(np.random.PCG64(8))
    for t, s in enumerate(shapes):
        K = s[3]
        ks = list(rng.choice(K, size=M, replace=False))
        ks[0], ks[-1] = 0, K - 1
        x = np.zeros((len(ks), K), np.uint16)
        for m, k in enumerate(ks):
            x[m, k] = 0x3F80
        xd = to_device_x(x)
        need = C.cloak_ws_bytes(cw.layout, C.CLOAK_OP_LINEAR, t, len(ks))
        ws_buf = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        y = torch.empty((len(ks), s[2]), dtype=torch.bfloat16, device="cuda")
        C.cloak_linear(cw.layout, cw.pool, t, xd, len(ks), y, ws_buf, ws_buf.numel())
        want = plus_zero(np.stack([ws[t][:, k] for k in ks]))
        assert np.array_equal(plus_zero(from_device(y)), want), (t, s)
    cw.close()


@pytest.mark.parametrize("M", [48, 333])
def test_prefill_gemm_cloaked_equals_native(C, M):
    import torch
    shapes = decoder_shapes(1024, 2816, 256, "bf16", layers=1)
    ws, scs = make_weights(shapes)
    B, P = 65536, 512
    cl = C.CloakedWeights(shapes, B, B * P, seed=23)
    nat = C.CloakedWeights(shapes, B, B * P, seed=23, flags=C.CLOAK_IDENTITY | C.CLOAK_NATIVE)
    cl.load(ws, scs)
    nat.load(ws, scs)
    for t, s in enumerate(shapes):
        if s[1] == "down":
            continue
        x = to_device_x(synth.activations(M, s[3], "bf16", seed=t))
        assert torch.equal(cl.linear(t, x).view(torch.int16), nat.linear(t, x).view(torch.int16)), s
    x = to_device_x(synth.activations(M, 1024, "bf16", seed=99))
    err = ON.normwise_err(values_f64(from_device(cl.mlp(0, x))), values_f64(from_device(nat.mlp(0, x))))
    assert err <= 1e-2
    cl.close()
    nat.close()


@pytest.mark.parametrize("M", [5, 17, 64, 128, 256, 300])
def test_fp8_mfma_paths_vs_fp64(C, M):
    # FP8 weights through the MFMA paths: up to 64 tokens the skinny split-K
    # kernel widens them to BF16 exactly in LDS (row scales applied after the
    # contraction); from 65 tokens, FP8 x FP8 on quantised activations (the
    # skinny direct-to-LDS tiles, then the 256x256 GEMM).  K = 1280 / 3456,
    # d_ffn 3456 and the 700-row head leave ragged row tiles
    shapes = decoder_shapes(1280, 3456, 256, "fp8", layers=1, extra=[(-1, "head", 700, 1280, "fp8")])
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 512, seed=29)
    cw.load(ws, scs)
    check_linear_all(C, cw, shapes, ws, scs, M)
    cw.close()


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
@pytest.mark.parametrize("M", [129, 256])
def test_skinny_256_token_tile_ragged(C, dtype, M):
    # 129..256 tokens: the 8-wave tile over 128 weight rows (64 hidden units
    # of SwiGLU per tile).  d_ffn 2848 leaves the last SwiGLU tile half full
    # (and sends the down projection, K = 2848, to the GEMV); 129 tokens pad
    # 127 of the 256 token rows.
    shapes = decoder_shapes(1024, 2848, 256, dtype, layers=1, extra=[(-1, "head", 1000, 1024, dtype)])
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 512, seed=31)
    cw.load(ws, scs)
    check_linear_all(C, cw, shapes, ws, scs, M)
    cw.close()


def one_hot_expected_a8(shapes, ws, scs, t, ks):
    """x = e_k through FP8 x FP8: the row quantises to code 448 with scale
    fl(1/448); the kernel forms ((448 q_w) * s_x) * s_w in binary32."""
    sx = np.float32(1.0) / np.float32(448.0)
    q = ON.e4m3_bits_to_f64(ws[t]).astype(np.float32)
    acc = np.float32(448.0) * q
    prod = (acc * sx).astype(np.float32) * scs[t].astype(np.float32)[:, None]
    return plus_zero(np.stack([ON.f32_to_bf16_bits_rne(prod[:, k]) for k in ks]))


@pytest.mark.parametrize("M", [40, 200, 300])
def test_fp8_mfma_one_hot_bit_exact(C, M):
    import torch
    shapes = decoder_shapes(1280, 3456, 256, "fp8", layers=1)
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 512, seed=37)
    cw.load(ws, scs)
    rng = np.random.Generator(np.random.PCG64(9))
    for t, s in enumerate(shapes):
        K = s[3]
        ks = list(rng.choice(K, size=M, replace=False))
        ks[0], ks[-1] = 0, K - 1
        x = np.zeros((M, K), np.uint16)
        for m, k in enumerate(ks):
            x[m, k] = 0x3F80
        need = C.cloak_ws_bytes(cw.layout, C.CLOAK_OP_LINEAR, t, M)
        ws_buf = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        y = torch.empty((M, s[2]), dtype=torch.bfloat16, device="cuda")
        C.cloak_linear(cw.layout, cw.pool, t, to_device_x(x), M, y, ws_buf, ws_buf.numel())
        want = one_hot_expected(shapes, ws, scs, t, ks) if M <= 64 else one_hot_expected_a8(shapes, ws, scs, t, ks)
        assert np.array_equal(plus_zero(from_device(y)), want), (t, s)
    cw.close()


def test_quantize_fp8_codes_and_scales_bit_exact(C):
    import torch
    rng = np.random.Generator(np.random.PCG64(51))
    for M, K, ld in [(9, 1280, 1280), (5, 333, 400), (3, 27648, 27648), (1, 8, 8)]:
        x32 = (rng.standard_normal((M, ld)) * rng.uniform(0.01, 50, (M, 1))).astype(np.float32)
        x32[M // 2] = 0.0                         # an all-zero row
        x32[0, :min(K, 16)] = [2.0 ** -12, -448.0, 1e-30, 3.0, -0.0, 96.0, 1.0, 0.5, 7.0, 6.5, 0.0, 1.0,
                               2.0, 2.25, -2.5, 2.75][:min(K, 16)]
        xb = synth.f32_to_bf16_rne(x32)
        q = torch.empty((M, K), dtype=torch.uint8, device="cuda")
        sc = torch.empty(M, dtype=torch.float32, device="cuda")
        C.cloak_quantize_fp8(to_device_x(xb)[:, :K], M, q, sc)
        wq, ws_ = ON.quantize_rows_e4m3(synth.bf16_to_f32(xb[:, :K]))
        assert np.array_equal(q.cpu().numpy(), wq), (M, K)
        assert np.array_equal(sc.cpu().numpy().view(np.uint32), ws_.view(np.uint32)), (M, K)


@pytest.mark.parametrize("M", [65, 128, 200, 256, 257, 600])
def test_fp8_x_fp8_gemm_vs_oracle(C, M):
    # from 65 tokens FP8 weights run FP8 x FP8 MFMA on per-token quantised
    # activations (65..256: the skinny split-K direct-to-LDS tiles; above:
    # the 256x256 GEMM): against the oracle's product of the same quantised
    # activations the only differences are FP32 summation order and the bf16
    # output rounding (1e-2); against unquantised FP64 the FP8 bar (5e-2)
    shapes = decoder_shapes(1280, 3456, 256, "fp8", layers=1)
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, 65536, 65536 * 512, seed=43)
    cw.load(ws, scs)
    worst_q, worst_u = 0.0, 0.0
    for t, s in enumerate(shapes):
        x_np = synth.activations(M, s[3], "bf16", seed=900 + t)
        y = values_f64(from_device(cw.linear(t, to_device_x(x_np))))
        # (a down projection quantises after its gather through pi: a row's
        # scale and each element's code do not depend on the column order)
        xq = ON.fp8_activations_f64(*ON.quantize_rows_e4m3(synth.bf16_to_f32(x_np)))
        w = w64(shapes, ws, scs, t)
        eq = ON.normwise_err(y, ON.linear(xq, w))
        eu = ON.normwise_err(y, ON.linear(values_f64(x_np), w))
        worst_q, worst_u = max(worst_q, eq), max(worst_u, eu)
        assert eq <= 1e-2, (t, s, eq)
        assert eu <= TOL["fp8"], (t, s, eu)
    x_np = synth.activations(M, 1280, "bf16", seed=990)
    y = values_f64(from_device(cw.mlp(0, to_device_x(x_np))))
    ref, _ = ON.swiglu_ffn(values_f64(x_np), w64(shapes, ws, scs, 4), w64(shapes, ws, scs, 5), w64(shapes, ws, scs, 6))
    eu = ON.normwise_err(y, ref)
    assert eu <= TOL["fp8"], eu
    print(f"fp8 x fp8 M={M}: vs quantised-activation oracle {worst_q:.2e}, vs FP64 {worst_u:.2e}, mlp {eu:.2e}")
    cw.close()


def test_decode_full_layer4096_bench_calls(C):
    """The bench's decode step at full size (4096/14336/1024 BF16 layer, 2 MiB
    pages over an 8 GiB pool) at every batch it reports, through the same
    calls (fused q/k/v, o, cloak_swiglu then cloak_down with one workspace),
    against FP64 on every output."""
    import torch
    cfg = synth.LAYER4096
    d, f, kv = cfg["d_model"], cfg["d_ffn"], cfg["d_kv"]
    shapes = decoder_shapes(d, f, kv, "bf16", layers=1)
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, cfg["page_bytes"], cfg["pool_bytes"], seed=1)
    cw.load(ws, scs)
    L = cw.layout
    W = [w64(shapes, ws, scs, t) for t in range(len(shapes))]
    # 100 and 128 tokens run the 4-stage LDS-ring tile with K slices sized to
    # one pass over the CUs, 256 the 3-stage ring on 8 waves
    for M in (1, 8, 32, 64, 100, 128, 256):
        x_np = synth.activations(M, d, "bf16", seed=100 + M)
        x, x64 = to_device_x(x_np), values_f64(x_np)
        need = max(C.cloak_linear_fused_ws_bytes(L, [0, 1, 2], M), C.cloak_ws_bytes(L, C.CLOAK_OP_LINEAR, 3, M),
                   C.cloak_ws_bytes(L, C.CLOAK_OP_SWIGLU, 0, M), C.cloak_ws_bytes(L, C.CLOAK_OP_DOWN, 0, M))
        wsb = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        qkv = torch.empty((M, d + 2 * kv), dtype=torch.bfloat16, device="cuda")
        o = torch.empty((M, d), dtype=torch.bfloat16, device="cuda")
        h = torch.empty((M, f), dtype=torch.bfloat16, device="cuda")
        y = torch.empty((M, d), dtype=torch.bfloat16, device="cuda")
        C.cloak_linear_fused(L, cw.pool, [0, 1, 2], x, M, qkv, wsb, wsb.numel())
        C.cloak_linear(L, cw.pool, 3, x, M, o, wsb, wsb.numel())
        C.cloak_swiglu(L, cw.pool, 0, x, M, h, wsb, wsb.numel())
        C.cloak_down(L, cw.pool, 0, h, M, y, wsb, wsb.numel())
        ref_qkv = np.concatenate([ON.linear(x64, W[t]) for t in (0, 1, 2)], axis=1)
        assert ON.normwise_err(values_f64(from_device(qkv)), ref_qkv) <= 1e-2, M
        assert ON.normwise_err(values_f64(from_device(o)), ON.linear(x64, W[3])) <= 1e-2, M
        ref_y, _ = ON.swiglu_ffn(x64, W[4], W[5], W[6])
        assert ON.normwise_err(values_f64(from_device(y)), ref_y) <= 1e-2, M
    cw.close()
    torch.cuda.empty_cache()


def test_fp8_stack_layer5120_full_size_sampled(C):
    """One layer of the 64-layer FP8 stack at full size (5120/27648/1024 E4M3
    with row scales) and the 152064 x 5120 BF16 head, 2 MiB pages, at decode
    batches 1, 64 and 256, against FP64 on sampled tokens."""
    import torch
    cfg = synth.STACK5120
    d, f, kv, V = cfg["d_model"], cfg["d_ffn"], cfg["d_kv"], cfg["vocab"]
    shapes = decoder_shapes(d, f, kv, "fp8", layers=1, extra=[(-1, "head", V, d, "bf16")])
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, cfg["page_bytes"], 4 << 30, seed=9)
    cw.load(ws, scs)
    rng = np.random.Generator(np.random.PCG64(17))
    W = {t: w64(shapes, ws, scs, t) for t in (0, 3, 4, 5, 6, 7)}
    for M in (1, 64, 256):
        x_np = synth.activations(M, d, "bf16", seed=200 + M)
        x = to_device_x(x_np)
        rows = np.unique(np.concatenate([[0, M - 1], rng.choice(M, size=min(M, 10), replace=False)]))
        x64 = values_f64(x_np[rows])
        for t in (0, 3, 7):        # q, o and the head
            y = from_device(cw.linear(t, x))[rows]
            tol = TOL[shapes[t][4]]
            assert ON.normwise_err(values_f64(y), ON.linear(x64, W[t])) <= tol, (M, t)
        y = from_device(cw.mlp(0, x))[rows]
        ref, _ = ON.swiglu_ffn(x64, W[4], W[5], W[6])
        assert ON.normwise_err(values_f64(y), ref) <= TOL["fp8"], M
    # prefill: 8192 tokens through FP8 x FP8 MFMA on per-token E4M3
    # activations, the configuration the stack's prefill figure is taken on;
    # quantisation is per row, so the sampled rows' codes are the oracle's own
    M = 8192
    x_np = synth.activations(M, d, "bf16", seed=8192)
    x = to_device_x(x_np)
    rows = np.unique(np.concatenate([[0, M - 1], rng.choice(M, size=24, replace=False)]))
    x64 = values_f64(x_np[rows])
    xq = ON.fp8_activations_f64(*ON.quantize_rows_e4m3(synth.bf16_to_f32(x_np[rows])))
    for t in (0, 3):
        y = values_f64(from_device(cw.linear(t, x))[rows])
        assert ON.normwise_err(y, ON.linear(xq, W[t])) <= 1e-2, ("a8", t)
        assert ON.normwise_err(y, ON.linear(x64, W[t])) <= TOL["fp8"], ("a8", t)
    y = values_f64(from_device(cw.mlp(0, x))[rows])
    ref, _ = ON.swiglu_ffn(x64, W[4], W[5], W[6])
    assert ON.normwise_err(y, ref) <= TOL["fp8"], "a8 mlp"
    del W
    cw.close()
    torch.cuda.empty_cache()


def test_prefill_full_layer4096_sampled_tokens(C):
    """The 4096/14336 layer at M = 8192 prefill tokens, 2 MiB pages over an
    8 GiB pool, checked against FP64 on 48 sampled tokens."""
    import torch
    cfg = synth.LAYER4096
    shapes = decoder_shapes(cfg["d_model"], cfg["d_ffn"], cfg["d_kv"], "bf16", layers=1)
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, cfg["page_bytes"], cfg["pool_bytes"], seed=1)
    cw.load(ws, scs)
    M = 8192
    x_np = synth.activations(M, cfg["d_model"], "bf16")
    x = to_device_x(x_np)
    rng = np.random.Generator(np.random.PCG64(3))
    rows = np.sort(rng.choice(M, size=48, replace=False))
    rows[0], rows[-1] = 0, M - 1
    x64 = values_f64(x_np[rows])
    for t in (0, 1, 2, 3):   # q, k, v and o (K = 4096)
        y = from_device(cw.linear(t, x))[rows]
        err = ON.normwise_err(values_f64(y), ON.linear(x64, w64(shapes, ws, scs, t)))
        assert err <= 1e-2, (t, err)
    # the fused q/k/v call the bench times
    y = from_device(cw.linear_fused([0, 1, 2], x))[rows]
    ref = np.concatenate([ON.linear(x64, w64(shapes, ws, scs, t)) for t in (0, 1, 2)], axis=1)
    err = ON.normwise_err(values_f64(y), ref)
    assert err <= 1e-2, ("qkv", err)
    y = from_device(cw.mlp(0, x))[rows]
    ref, _ = ON.swiglu_ffn(x64, w64(shapes, ws, scs, 4), w64(shapes, ws, scs, 5), w64(shapes, ws, scs, 6))
    err = ON.normwise_err(values_f64(y), ref)
    assert err <= 1e-2, err
    cw.close()
    torch.cuda.empty_cache()


def test_stream_read_calibration_runs_and_checks_arguments(C):
    import torch
    buf = torch.ones(1 << 20, dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    C.cloak_stream_read(buf, buf.numel(), out)
    torch.cuda.synchronize()
    assert int(out.item()) == 0          # the fold of all-ones words is not the sentinel
    for nbytes, off in [(1000, 0), ((1 << 20) - 16, 8)]:   # not a multiple of 16; misaligned
        with pytest.raises(C.CloakError):
            C.cloak_stream_read(buf[off:], nbytes, out)

"""The C-ABI library on the CPU: exports, layout and host images vs the oracle.

No device is touched: these calls are host-only by contract (include/cloak.h).
"""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import layout as OL
from oracle import remap as OR
from paper_2606_18400_amd import cloak as C
from paper_2606_18400_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "cloak.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cloak_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = header_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(C.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(C.EXPORTED)


def oracle_shapes(shapes):
    return [OL.Shape(*s) for s in shapes]


def small_model(dtype="bf16", layers=2, d=512, ffn=768, dkv=128, vocab=1000, head_dim=0):
    shapes = []
    for l in range(layers):
        shapes += synth.decoder_layer_shapes(d, ffn, dkv, dtype, layer=l, head_dim=head_dim)
    shapes += [(-1, "embed", vocab, d, dtype), (-1, "head", vocab, d, dtype)]
    return shapes


def compare_layout(lay_c, lay_o):
    assert C.cloak_query(lay_c, "P") == lay_o.P
    assert C.cloak_query(lay_c, "V") == lay_o.V
    assert list(C.cloak_query(lay_c, "SIGMA")) == lay_o.sigma
    assert list(C.cloak_query(lay_c, "PHI")) == lay_o.phi
    assert list(C.cloak_query(lay_c, "VBASE")) == lay_o.vbase
    assert list(C.cloak_query(lay_c, "NPAGES")) == lay_o.npages
    for l, pi in lay_o.pi.items():
        assert list(C.cloak_query(lay_c, "PI", l)) == pi
    for t in range(lay_o.T):
        assert list(C.cloak_query(lay_c, "UPLOAD_ORDER", t)) == OL.upload_order(lay_o, t)
        s = lay_o.shapes[t]
        rp, cp = lay_o.row_perm(t), lay_o.col_perm(t)
        assert list(C.cloak_query(lay_c, "ROW_PERM", t)) == (rp if rp is not None else list(range(s.n_out)))
        assert list(C.cloak_query(lay_c, "COL_PERM", t)) == (cp if cp is not None else list(range(s.k_in)))
        assert list(C.cloak_query(lay_c, "SHAPE", t)) == [s.n_out, s.k_in, C.DTYPES[s.dtype], s.head_dim]
    assert C.cloak_query(lay_c, "CONTIGUITY") == pytest.approx(OL.contiguity(lay_o), abs=0)


@pytest.mark.parametrize("seed", [1, 0xC10A4, (1 << 64) - 1])
@pytest.mark.parametrize("flags", [0, C.CLOAK_IDENTITY, C.CLOAK_CSPRNG])
def test_layout_matches_oracle(seed, flags):
    shapes = small_model(head_dim=64)
    lay_c = C.cloak_layout_build(seed, shapes, 64 << 10, 64 << 20, flags)
    try:
        lay_o = OL.build_layout(seed, oracle_shapes(shapes), 64 << 10, 64 << 20,
                                identity=bool(flags & C.CLOAK_IDENTITY), csprng=bool(flags & C.CLOAK_CSPRNG))
        compare_layout(lay_c, lay_o)
    finally:
        C.cloak_layout_free(lay_c)


@pytest.mark.parametrize("seed", [1, 0xC10A4, (1 << 64) - 1])
@pytest.mark.parametrize("flags", [0, C.CLOAK_IDENTITY])
@pytest.mark.parametrize("geom", [(512, 128, 64), (512, 512, 128), (512, 64, 64)])   # d, d_kv, head_dim
def test_head_permuted_layout_matches_oracle(seed, flags, geom):
    d, dkv, hd = geom
    shapes = small_model(d=d, dkv=dkv, head_dim=hd)
    lay_c = C.cloak_layout_build(seed, shapes, 64 << 10, 64 << 20, flags)
    try:
        lay_o = OL.build_layout(seed, oracle_shapes(shapes), 64 << 10, 64 << 20, identity=bool(flags))
        assert lay_o.heads and set(lay_o.heads) == {0, 1}
        compare_layout(lay_c, lay_o)
        # head size 0 on the same shapes draws the same sigma, pi and phi
        plain = C.cloak_layout_build(seed, small_model(d=d, dkv=dkv), 64 << 10, 64 << 20, flags)
        assert list(C.cloak_query(plain, "PHI")) == lay_o.phi
        assert list(C.cloak_query(plain, "ROW_PERM", 0)) == list(range(d))
        C.cloak_layout_free(plain)
    finally:
        C.cloak_layout_free(lay_c)


def test_head_permuted_layout_errors():
    good = synth.decoder_layer_shapes(256, 512, 64, "bf16", head_dim=32)
    for bad, code in [
        ([s for s in good if s[1] != "v"], C.CLOAK_ESHAPE),                       # v missing
        ([s[:5] if s[1] == "k" else s for s in good], C.CLOAK_ESHAPE),            # k without head size
        ([s[:5] + (16,) if s[1] == "k" else s for s in good], C.CLOAK_ESHAPE),    # head sizes disagree
        ([s + (32,) if s[1] == "gate" else s for s in good], C.CLOAK_EINVAL),     # head size on gate
        ([(s[0], s[1], 96, *s[3:]) if s[1] == "k" else s for s in good], C.CLOAK_ESHAPE),  # 8 q over 3 kv
        ([(-1,) + s[1:] if s[1] in "qkvo" else s for s in good], C.CLOAK_ESHAPE),  # negative layer
    ]:
        with pytest.raises(C.CloakError) as e:
            C.cloak_layout_build(1, bad, 64 << 10, 64 << 20)
        assert e.value.code == code, bad


def test_layout_matches_oracle_on_ffn512_block():
    cfg = synth.FFN512
    shapes = synth.ffn_block_shapes(cfg["d_model"], cfg["d_ffn"], cfg["dtype"])
    for seed in (1, 2, 3):
        lay_c = C.cloak_layout_build(seed, shapes, cfg["page_bytes"], cfg["pool_bytes"])
        lay_o = OL.build_layout(seed, oracle_shapes(shapes), cfg["page_bytes"], cfg["pool_bytes"])
        compare_layout(lay_c, lay_o)
        assert lay_o.V == 96 and lay_o.P == 256
        C.cloak_layout_free(lay_c)


def test_layout_matches_oracle_on_layer4096_pool():
    cfg = synth.LAYER4096
    shapes = []
    for copy in range(16):
        shapes += synth.decoder_layer_shapes(cfg["d_model"], cfg["d_ffn"], cfg["d_kv"], "bf16", layer=copy)
    lay_c = C.cloak_layout_build(1, shapes, cfg["page_bytes"], cfg["pool_bytes"])
    lay_o = OL.build_layout(1, oracle_shapes(shapes), cfg["page_bytes"], cfg["pool_bytes"])
    assert lay_o.V == 16 * 208 and lay_o.P == 4096
    compare_layout(lay_c, lay_o)
    C.cloak_layout_free(lay_c)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("seed", [3, 4])
def test_pack_host_matches_oracle_pool_bytes(dtype, seed):
    # 1 KiB pages, rows that straddle pages (K*elt not a multiple of 1 KiB);
    # layer 2's attention is head-permuted (6 query heads over 2 kv heads of 12)
    shapes = [(0, "q", 40, 264, dtype), (0, "gate", 72, 264, dtype), (0, "up", 72, 264, dtype),
              (0, "down", 264, 72, dtype), (1, "gate", 48, 264, dtype), (1, "up", 48, 264, dtype),
              (1, "down", 264, 48, dtype), (-1, "head", 50, 264, dtype),
              (2, "q", 72, 264, dtype, 12), (2, "k", 24, 264, dtype, 12), (2, "v", 24, 264, dtype, 12),
              (2, "o", 264, 72, dtype, 12)]
    P, B = 1024, 1024
    rng = np.random.Generator(np.random.PCG64(seed))
    ws = [rng.integers(0, 256, (s[2], s[3] * {"f32": 4, "bf16": 2, "fp8": 1}[dtype]), dtype=np.uint8)
          .view(C.STORAGE[dtype]) for s in shapes]
    lay_c = C.cloak_layout_build(seed, shapes, B, P * B)
    lay_o = OL.build_layout(seed, oracle_shapes(shapes), B, P * B)
    img = np.zeros(P * B, np.uint8)
    for t, w in enumerate(ws):
        C.cloak_pack_host(lay_c, t, w, img)
    want = OL.pack(lay_o, ws)
    assert np.array_equal(img, want)
    C.cloak_layout_free(lay_c)


@pytest.mark.parametrize("remap_seed", [1, 2, 12345])
@pytest.mark.parametrize("csprng", [False, True])
def test_remap_host_matches_oracle(remap_seed, csprng):
    shapes = small_model("bf16", layers=1, d=128, ffn=256, dkv=32, vocab=100)
    P, B = 1025, 1024   # odd P: one page stays put
    ws = [synth.weight(t, s[2], s[3], "bf16")[0] for t, s in enumerate(shapes)]
    lay_c = C.cloak_layout_build(9, shapes, B, P * B, C.CLOAK_CSPRNG if csprng else 0)
    lay_o = OL.build_layout(9, oracle_shapes(shapes), B, P * B, csprng=csprng)
    img = np.zeros(P * B, np.uint8)
    for t, w in enumerate(ws):
        C.cloak_pack_host(lay_c, t, w, img)
    pool_o = OL.pack(lay_o, ws)
    C.cloak_remap_host(lay_c, img, remap_seed)
    pool_o2, phi_o2 = OR.remap(pool_o, lay_o.phi, remap_seed, B, csprng=csprng)
    assert list(C.cloak_query(lay_c, "PHI")) == phi_o2
    assert np.array_equal(img, pool_o2)
    assert C.cloak_query(lay_c, "REMAPS") == 1
    C.cloak_layout_free(lay_c)


@pytest.mark.parametrize("slice_pairs", [1, 37, 0])
def test_incremental_remap_host_matches_oracle_slices(slice_pairs):
    shapes = small_model("bf16", layers=1, d=128, ffn=256, dkv=32, vocab=100)
    P, B = 513, 1024   # odd P: one page stays put
    ws = [synth.weight(t, s[2], s[3], "bf16")[0] for t, s in enumerate(shapes)]
    lay_c = C.cloak_layout_build(9, shapes, B, P * B)
    lay_o = OL.build_layout(9, oracle_shapes(shapes), B, P * B)
    img = np.zeros(P * B, np.uint8)
    for t, w in enumerate(ws):
        C.cloak_pack_host(lay_c, t, w, img)
    pool_o = OL.pack(lay_o, ws)
    C.cloak_remap_begin(lay_c, 4242)
    assert C.cloak_query(lay_c, "REMAP_PENDING") == P // 2
    expect_error(C.CLOAK_ESTATE, C.cloak_remap_begin, lay_c, 1)          # one remap at a time
    expect_error(C.CLOAK_ESTATE, C.cloak_remap_host, lay_c, img, 1)
    states = list(OR.remap_in_slices(pool_o, lay_o.phi, 4242, B, slice_pairs if slice_pairs > 0 else P))
    for k, (pool_k, phi_k) in enumerate(states):
        left = C.cloak_remap_step_host(lay_c, img, slice_pairs)
        assert left == C.cloak_query(lay_c, "REMAP_PENDING")
        assert list(C.cloak_query(lay_c, "PHI")) == phi_k
        assert np.array_equal(img, pool_k)
        assert C.cloak_query(lay_c, "REMAPS") == (1 if left == 0 else 0)
    assert left == 0
    expect_error(C.CLOAK_ESTATE, C.cloak_remap_step_host, lay_c, img, 1)  # nothing in progress
    C.cloak_layout_free(lay_c)


@pytest.mark.parametrize("remap_seed", [1, 7, 99991])
@pytest.mark.parametrize("csprng", [False, True])
@pytest.mark.parametrize("P", [1, 2, 3, 1025])
def test_uniform_remap_host_matches_oracle(remap_seed, csprng, P):
    # P = 1..3: degenerate pools (nothing or one pair to move; rho may be the identity)
    B = 1024
    shapes = small_model("bf16", layers=1, d=128, ffn=256, dkv=32, vocab=100) if P > 3 else [(0, "q", 8, 64, "bf16")]
    ws = [synth.weight(t, s[2], s[3], "bf16")[0] for t, s in enumerate(shapes)]
    flags = C.CLOAK_REMAP_UNIFORM | (C.CLOAK_CSPRNG if csprng else 0)
    lay_c = C.cloak_layout_build(9, shapes, B, P * B, flags)
    lay_o = OL.build_layout(9, oracle_shapes(shapes), B, P * B, csprng=csprng)
    img = np.zeros(P * B, np.uint8)
    for t, w in enumerate(ws):
        C.cloak_pack_host(lay_c, t, w, img)
    pool_o = OL.pack(lay_o, ws)
    phi_o = lay_o.phi
    for k in range(2):   # two remaps in a row: the second starts from a scattered map
        C.cloak_remap_host(lay_c, img, remap_seed + k)
        pool_o, phi_o = OR.remap_uniform(pool_o, phi_o, remap_seed + k, B, csprng=csprng)
        assert list(C.cloak_query(lay_c, "PHI")) == phi_o
        assert np.array_equal(img, pool_o)
        assert C.cloak_query(lay_c, "REMAPS") == k + 1


@pytest.mark.parametrize("slice_pairs", [1, 37, 0])
def test_incremental_uniform_remap_host_matches_oracle_slices(slice_pairs):
    shapes = small_model("bf16", layers=1, d=128, ffn=256, dkv=32, vocab=100)
    P, B = 513, 1024
    ws = [synth.weight(t, s[2], s[3], "bf16")[0] for t, s in enumerate(shapes)]
    lay_c = C.cloak_layout_build(9, shapes, B, P * B, C.CLOAK_REMAP_UNIFORM)
    lay_o = OL.build_layout(9, oracle_shapes(shapes), B, P * B)
    img = np.zeros(P * B, np.uint8)
    for t, w in enumerate(ws):
        C.cloak_pack_host(lay_c, t, w, img)
    pool_o = OL.pack(lay_o, ws)
    one, two = OR.uniform_passes(4242, P)
    C.cloak_remap_begin(lay_c, 4242)
    assert C.cloak_query(lay_c, "REMAP_PENDING") == len(one) + len(two)
    if slice_pairs > 0:
        states = list(OR.remap_uniform_in_slices(pool_o, lay_o.phi, 4242, B, slice_pairs))
    else:   # one call runs both passes
        states = [OR.remap_uniform(pool_o, lay_o.phi, 4242, B)]
    for pool_k, phi_k in states:
        left = C.cloak_remap_step_host(lay_c, img, slice_pairs)
        assert left == C.cloak_query(lay_c, "REMAP_PENDING")
        assert list(C.cloak_query(lay_c, "PHI")) == phi_k
        assert np.array_equal(img, pool_k)
    assert left == 0 and C.cloak_query(lay_c, "REMAPS") == 1
    C.cloak_layout_free(lay_c)


def expect_error(code, fn, *args):
    with pytest.raises(C.CloakError) as e:
        fn(*args)
    assert e.value.code == code
    assert C.cloak_last_error()


def test_error_codes_without_device():
    good = [(0, "q", 8, 512, "bf16")]
    expect_error(C.CLOAK_EINVAL, C.cloak_layout_build, 1, good, 3000, 3000 * 8)       # not a power of two
    expect_error(C.CLOAK_EINVAL, C.cloak_layout_build, 1, good, 512, 512 * 8)         # below 1 KiB
    expect_error(C.CLOAK_EINVAL, C.cloak_layout_build, 1, good, 1024, 1024 * 8 + 1)   # pool not whole pages
    expect_error(C.CLOAK_ENOMEM, C.cloak_layout_build, 1, [(0, "q", 4096, 512, "bf16")], 1024, 1024 * 8)
    expect_error(C.CLOAK_ESHAPE, C.cloak_layout_build, 1, good + good, 1024, 1024 * 64)
    expect_error(C.CLOAK_ESHAPE, C.cloak_layout_build, 1,
                 [(0, "gate", 64, 512, "bf16"), (0, "down", 512, 48, "bf16")], 1024, 1024 * 256)
    expect_error(C.CLOAK_EINVAL, C.cloak_layout_build, 1, good, 1024, 1024 * 64, C.CLOAK_NATIVE)
    expect_error(C.CLOAK_EINVAL, C.cloak_layout_build, 1, [(0, "q", 0, 512, "bf16")], 1024, 1024 * 64)
    L = C.cloak_layout_build(1, good, 1024, 1024 * 64)
    try:
        # device calls before cloak_layout_to_device are refused before any launch
        expect_error(C.CLOAK_ESTATE, C.cloak_linear, L, 256, 0, 256, 1, 256, None, 0, 0)
        expect_error(C.CLOAK_ESTATE, C.cloak_remap, L, 256, 1, 0)
        expect_error(C.CLOAK_EINVAL, C.cloak_query, L, 99, 0)
        expect_error(C.CLOAK_EINVAL, C.cloak_query, L, "PI", 5)
        img = np.zeros(10, np.uint8)
        expect_error(C.CLOAK_EINVAL, C.cloak_pack_host, L, 0, np.zeros((8, 512), np.uint16), img)
        expect_error(C.CLOAK_EINVAL, C.cloak_pack_host, L, 3, np.zeros((8, 512), np.uint16),
                     np.zeros(1024 * 64, np.uint8))
    finally:
        C.cloak_layout_free(L)
    N = C.cloak_layout_build(1, good, 1024, 1024 * 64, C.CLOAK_IDENTITY | C.CLOAK_NATIVE)
    expect_error(C.CLOAK_ESTATE, C.cloak_remap_host, N, np.zeros(1024 * 64, np.uint8), 1)
    expect_error(C.CLOAK_ESTATE, C.cloak_remap_begin, N, 1)
    C.cloak_layout_free(N)


def test_first_uploads_must_follow_the_tensor_order():
    # a caller that sends tensors in their architectural order is refused before
    # any page crosses the bus (the check comes before the device checks)
    shapes = small_model("bf16", layers=2, d=128, ffn=256, dkv=32, vocab=100)
    L = C.cloak_layout_build(9, shapes, 1024, 1024 * 1024)
    try:
        sigma = list(C.cloak_query(L, "SIGMA"))
        assert sigma != list(range(len(shapes)))
        first_canonical = next(t for t in range(len(shapes)) if t != sigma[0])
        with pytest.raises(C.CloakError) as e:
            C.cloak_load(L, 256, first_canonical, np.zeros((shapes[first_canonical][2], shapes[first_canonical][3]),
                                                           np.uint16), stream=0)
        assert e.value.code == C.CLOAK_ESTATE and "tensor order" in C.cloak_last_error()
        # the tensor sigma names first passes the order check (and then needs a device)
        with pytest.raises(C.CloakError) as e:
            C.cloak_load(L, 256, sigma[0], np.zeros((shapes[sigma[0]][2], shapes[sigma[0]][3]), np.uint16), stream=0)
        assert e.value.code == C.CLOAK_ESTATE and "tensor order" not in C.cloak_last_error()
    finally:
        C.cloak_layout_free(L)


def test_mlp_workspace_is_exported_under_its_name():
    shapes = small_model("bf16", layers=2, d=512, ffn=768, dkv=128, vocab=100)
    L = C.cloak_layout_build(2, shapes, 1 << 16, 1 << 26)
    try:
        for M in (0, 1, 4, 5, 64, 256, 300):
            assert C.cloak_mlp_ws_bytes(L, 1, M) == C.cloak_ws_bytes(L, C.CLOAK_OP_MLP, 1, M)
        assert C.cloak_mlp_ws_bytes(L, 1, 1) > 0
        with pytest.raises(C.CloakError):
            C.cloak_mlp_ws_bytes(L, 7, 4)      # no such layer
    finally:
        C.cloak_layout_free(L)


def test_identity_layout_is_contiguous():
    shapes = small_model("f32", layers=1, d=256, ffn=512, dkv=64, vocab=300)
    L = C.cloak_layout_build(5, shapes, 1024, 1024 * 4096, C.CLOAK_IDENTITY)
    assert C.cloak_query(L, "CONTIGUITY") == 1.0
    assert list(C.cloak_query(L, "SIGMA")) == list(range(len(shapes)))
    C.cloak_layout_free(L)


@pytest.mark.parametrize("dtype,page_bytes", [("f32", 1024), ("bf16", 1024), ("fp8", 1024), ("bf16", 4096),
                                              ("mixed", 2048)])
def test_decoy_host_image_matches_oracle(dtype, page_bytes):
    from oracle import decoy as OD
    if dtype == "mixed":
        # fp8 holds the most bytes: decoys are E4M3 codes
        shapes = [(0, "gate", 64, 256, "bf16"), (0, "up", 64, 256, "bf16"), (0, "down", 256, 64, "bf16"),
                  (1, "gate", 256, 256, "fp8"), (1, "up", 256, 256, "fp8")]
    else:
        shapes = [(0, "gate", 72, 264, dtype), (0, "up", 72, 264, dtype), (0, "down", 264, 72, dtype),
                  (1, "q", 96, 264, dtype, 12), (1, "k", 24, 264, dtype, 12), (1, "v", 24, 264, dtype, 12),
                  (1, "o", 264, 96, dtype, 12)]
    P = 640
    lay_c = C.cloak_layout_build(17, shapes, page_bytes, P * page_bytes)
    lay_o = OL.build_layout(17, oracle_shapes(shapes), page_bytes, P * page_bytes)
    rng = np.random.Generator(np.random.PCG64(2))
    ws = [rng.integers(0, 256, (s[2], s[3] * {"f32": 4, "bf16": 2, "fp8": 1}[s[4]]), dtype=np.uint8)
          .view(C.STORAGE[s[4]]) for s in shapes]
    img = np.zeros(P * page_bytes, np.uint8)
    for t, w in enumerate(ws):
        C.cloak_pack_host(lay_c, t, w, img)
    C.cloak_pool_decoy_host(lay_c, img, 0xDEC0DE)
    want = OD.fill_decoys(lay_o, OL.pack(lay_o, ws), 0xDEC0DE)
    assert lay_o.P - lay_o.V > 50
    assert np.array_equal(img, want)
    C.cloak_layout_free(lay_c)


def test_hardening_flags_on_the_host():
    shapes = small_model(head_dim=64)
    for flags in (C.CLOAK_MASKED_MAP, C.CLOAK_CSPRNG | C.CLOAK_MASKED_MAP):
        lay = C.cloak_layout_build(3, shapes, 64 << 10, 64 << 20, flags)
        assert C.cloak_query(lay, "MAP_KEY") == 0          # no device map yet
        o = OL.build_layout(3, oracle_shapes(shapes), 64 << 10, 64 << 20,
                            csprng=bool(flags & C.CLOAK_CSPRNG))
        assert list(C.cloak_query(lay, "PHI")) == o.phi      # masking never touches the host map
        C.cloak_layout_free(lay)
    with pytest.raises(C.CloakError):
        C.cloak_layout_build(3, shapes, 64 << 10, 64 << 20, 32)   # unknown flag

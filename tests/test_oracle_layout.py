"""Pins for the oracle's layout: bijections, brute-force placement, round trips."""

import numpy as np
import pytest

from oracle import layout as L
from oracle import prng


def tiny_shapes(dtype="bf16", layers=2, d=16, ffn=24):
    shapes = []
    for l in range(layers):
        shapes += [L.Shape(l, "q", d, d, dtype), L.Shape(l, "o", d, d, dtype),
                   L.Shape(l, "gate", ffn, d, dtype), L.Shape(l, "up", ffn, d, dtype),
                   L.Shape(l, "down", d, ffn, dtype)]
    shapes.append(L.Shape(-1, "head", 40, d, dtype))
    return shapes


def random_weights(shapes, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for s in shapes:
        if s.dtype == "f32":
            out.append(rng.standard_normal((s.n_out, s.k_in)).astype(np.float32))
        elif s.dtype == "bf16":
            out.append(rng.integers(0, 1 << 16, (s.n_out, s.k_in), dtype=np.uint16))
        else:
            out.append(rng.integers(0, 256, (s.n_out, s.k_in), dtype=np.uint8))
    return out


@pytest.mark.parametrize("seed", [1, 0xC10A4, (1 << 64) - 1])
def test_permutations_are_bijections(seed):
    shapes = tiny_shapes()
    lay = L.build_layout(seed, shapes, 64, 64 * 256)
    assert sorted(lay.sigma) == list(range(lay.T))
    assert sorted(lay.phi) == list(range(lay.P))
    for l, p in lay.pi.items():
        assert sorted(p) == list(range(24))
    assert set(lay.pi) == {0, 1}


def test_virtual_pages_follow_sigma_without_overlap():
    shapes = tiny_shapes()
    lay = L.build_layout(7, shapes, 64, 64 * 256)
    # brute force: walk the stream page by page and record the owner
    owner = [None] * lay.V
    for t in range(lay.T):
        assert lay.npages[t] == -(-shapes[t].nbytes // 64)
        for i in range(lay.npages[t]):
            assert owner[lay.vbase[t] + i] is None
            owner[lay.vbase[t] + i] = t
    assert None not in owner
    order = []
    for t in owner:
        if not order or order[-1] != t:
            order.append(t)
    assert order == lay.sigma
    assert lay.V == sum(lay.npages)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_pack_matches_element_by_element_definition(dtype):
    shapes = tiny_shapes(dtype)
    B = 64
    lay = L.build_layout(3, shapes, B, B * 256)
    ws = random_weights(shapes, 5)
    pool = L.pack(lay, ws)
    elt = L.ELT_BYTES[dtype]
    for t, s in enumerate(shapes):
        w_bytes = np.ascontiguousarray(ws[t]).view(np.uint8).reshape(s.n_out, s.k_in * elt)
        inv = None
        if s.layer in lay.pi:
            inv = {p: j for j, p in enumerate(lay.pi[s.layer])}
        for n in range(s.n_out):
            for k in range(s.k_in):
                # stored coordinates of logical element (n, k)
                if s.kind in ("gate", "up"):
                    j, c = inv[n], k
                elif s.kind == "down":
                    j, c = n, inv[k]
                else:
                    j, c = n, k
                off = (j * s.k_in + c) * elt
                for b in range(elt):
                    v = lay.vbase[t] + (off + b) // B
                    phys = lay.phi[v] * B + (off + b) % B
                    assert pool[phys] == w_bytes[n, k * elt + b]


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_unpack_inverts_pack_bit_exactly(dtype, seed):
    shapes = tiny_shapes(dtype)
    lay = L.build_layout(seed, shapes, 128, 128 * 128)
    ws = random_weights(shapes, seed)
    pool = L.pack(lay, ws)
    for t in range(lay.T):
        back = L.unpack(lay, pool, t)
        assert back.dtype == ws[t].dtype
        assert np.array_equal(back.view(np.uint8), ws[t].view(np.uint8))


def test_free_pages_and_padding_are_zero():
    shapes = tiny_shapes("bf16", d=16, ffn=20)  # 20*16*2 = 640 B: ragged last page
    B = 256
    lay = L.build_layout(11, shapes, B, B * 64)
    ws = random_weights(shapes, 1)
    pool = L.pack(lay, ws)
    used = set(lay.phi[v] for v in range(lay.V))
    for p in range(lay.P):
        if p not in used:
            assert not pool[p * B:(p + 1) * B].any()
    for t, s in enumerate(shapes):
        tail = lay.npages[t] * B - s.nbytes
        last = lay.phi[lay.vbase[t] + lay.npages[t] - 1]
        if tail:
            assert not pool[(last + 1) * B - tail:(last + 1) * B].any()


def test_identity_layout_is_plain_concatenation():
    shapes = tiny_shapes("f32")
    B = 64
    lay = L.build_layout(5, shapes, B, B * 256, identity=True)
    ws = random_weights(shapes, 2)
    pool = L.pack(lay, ws)
    cursor = 0
    for t, s in enumerate(shapes):
        raw = ws[t].view(np.uint8).reshape(-1)
        assert np.array_equal(pool[cursor:cursor + raw.size], raw)
        cursor += lay.npages[t] * B
    assert L.contiguity(lay) == 1.0


def test_shuffle_direction_gather_convention():
    shapes = [L.Shape(0, "gate", 5, 2, "f32"), L.Shape(0, "down", 2, 5, "f32")]
    lay = L.build_layout(4, shapes, 64, 64 * 8)
    pi = lay.pi[0]
    g = np.arange(10, dtype=np.float32).reshape(5, 2)
    d = np.arange(10, dtype=np.float32).reshape(2, 5)
    gs = L.shuffle_tensor(lay, 0, g)
    ds = L.shuffle_tensor(lay, 1, d)
    for j in range(5):
        assert list(gs[j]) == list(g[pi[j]])
        assert list(ds[:, j]) == list(d[:, pi[j]])


def test_upload_order_is_a_permutation_of_each_tensor():
    shapes = tiny_shapes()
    lay = L.build_layout(9, shapes, 64, 64 * 256)
    for t in range(lay.T):
        assert sorted(L.upload_order(lay, t)) == list(range(lay.npages[t]))


def test_contiguity_of_uniform_map_is_one_over_P():
    # For a uniform phi, P(phi[v+1] == phi[v] + 1) = (P-1)/P * 1/(P-1) = 1/P.
    shapes = [L.Shape(0, "q", 64, 64, "f32")]  # 16 KiB over 256-B pages: 64 pages
    P = 128
    vals = [L.contiguity(L.build_layout(s, shapes, 256, 256 * P)) for s in range(400)]
    assert abs(np.mean(vals) - 1.0 / P) < 3 * np.sqrt(1.0 / P / (63 * 400)) + 1e-4


def test_layout_errors():
    with pytest.raises(MemoryError):
        L.build_layout(1, tiny_shapes(), 64, 64 * 8)
    bad = [L.Shape(0, "gate", 24, 16, "bf16"), L.Shape(0, "down", 16, 20, "bf16")]
    with pytest.raises(ValueError):
        L.build_layout(1, bad, 64, 64 * 64)
    with pytest.raises(ValueError):
        L.build_layout(1, tiny_shapes(), 64, 64 * 256 + 1)


def test_seed_reproducible_and_seed_sensitive():
    shapes = tiny_shapes()
    a = L.build_layout(123, shapes, 64, 64 * 256)
    b = L.build_layout(123, shapes, 64, 64 * 256)
    c = L.build_layout(124, shapes, 64, 64 * 256)
    assert a.phi == b.phi and a.sigma == b.sigma and a.pi == b.pi
    assert a.phi != c.phi


def test_hidden_perm_uses_its_own_substream():
    shapes = tiny_shapes(layers=3)
    lay = L.build_layout(77, shapes, 64, 64 * 512)
    for l in range(3):
        assert lay.pi[l] == prng.fisher_yates(24, prng.substream(77, 2, l))
    assert lay.phi == prng.fisher_yates(512, prng.substream(77, 3, 0))
    assert lay.sigma == prng.fisher_yates(len(shapes), prng.substream(77, 1, 0))


def test_csprng_layout_is_valid_and_differs():
    shapes = tiny_shapes()
    a = L.build_layout(5, shapes, 64, 64 * 256, csprng=True)
    b = L.build_layout(5, shapes, 64, 64 * 256)
    assert sorted(a.phi) == list(range(a.P)) and sorted(a.sigma) == list(range(a.T))
    assert all(sorted(p) == list(range(24)) for p in a.pi.values())
    assert a.phi != b.phi and a.pi != b.pi
    assert a.phi == prng.fisher_yates(a.P, prng.substream_csprng(5, 3, 0))
    assert L.upload_order(a, 0) == prng.fisher_yates(a.npages[0], prng.substream_csprng(5, 4, 0))


def test_masked_map_hides_phi_and_unmasks_exactly():
    import hashlib
    import struct
    lay = L.build_layout(31, tiny_shapes(), 64, 64 * 4096)
    keys = L.map_keys(31)
    k0, k1 = next(keys), next(keys)
    # keys: words of SHA-256(seed || 8 || 0 || block), as the stream defines
    d = hashlib.sha256(struct.pack("<QIIQ", 31, 8, 0, 0)).digest()
    assert (k0, k1) == struct.unpack_from("<QQ", d, 0)
    t0 = L.masked_map(lay.phi, k0)
    # unmasking with the key restores phi; another key does not
    assert [t0[v] ^ L.map_mask(k0, v) for v in range(lay.P)] == lay.phi
    assert [t0[v] ^ L.map_mask(k1, v) for v in range(lay.P)] != lay.phi
    # entries spread over all 32 bits (phi < 4096 occupies 12): no high bit is constant
    t = np.array(t0, dtype=np.uint64)
    for bit in range(12, 32):
        frac = np.mean((t >> np.uint64(bit)) & np.uint64(1))
        assert 0.45 < frac < 0.55, bit
    # successive uploads differ entry by entry almost everywhere
    t1 = L.masked_map(lay.phi, k1)
    assert np.mean(np.array(t0) != np.array(t1)) > 0.99

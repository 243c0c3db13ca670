"""Pins for the oracle's remap: involution, zero-scratch moves, gather invariance."""

import numpy as np
import pytest

from oracle import layout as L
from oracle import prng
from oracle import remap as R
from test_oracle_layout import random_weights, tiny_shapes


@pytest.mark.parametrize("P", [1, 2, 7, 64, 257])
def test_matching_is_an_involution(P):
    tau = R.matching(42, P)
    assert sorted(tau) == list(range(P))
    assert all(tau[tau[p]] == p for p in range(P))
    fixed = sum(tau[p] == p for p in range(P))
    assert fixed == P % 2


def test_matching_pairs_consecutive_draws():
    P = 10
    s = prng.fisher_yates(P, prng.substream(5, prng.TAG_REMAP, 0))
    tau = R.matching(5, P)
    for i in range(P // 2):
        assert tau[s[2 * i]] == s[2 * i + 1]


@pytest.mark.parametrize("remap_seed", [1, 2, 3])
def test_remap_preserves_every_tensor(remap_seed):
    shapes = tiny_shapes("bf16")
    lay = L.build_layout(8, shapes, 64, 64 * 256)
    ws = random_weights(shapes, 3)
    pool = L.pack(lay, ws)
    pool2, phi2 = R.remap(pool, lay.phi, remap_seed, 64)
    assert sorted(phi2) == list(range(lay.P))
    lay2 = L.Layout(**{**lay.__dict__, "phi": phi2})
    for t in range(lay.T):
        assert np.array_equal(L.unpack(lay2, pool2, t), ws[t])
    # bytes are only moved: the multiset of pages is unchanged
    B = 64
    pages = sorted(bytes(pool[p * B:(p + 1) * B]) for p in range(lay.P))
    pages2 = sorted(bytes(pool2[p * B:(p + 1) * B]) for p in range(lay.P))
    assert pages == pages2


def test_remap_moves_each_page_to_its_partner_brute_force():
    P, B = 16, 8
    pool = np.arange(P * B, dtype=np.uint64).astype(np.uint8)
    phi = list(range(P))
    tau = R.matching(9, P)
    out, phi2 = R.remap(pool, phi, 9, B)
    for p in range(P):
        for i in range(B):
            assert out[tau[p] * B + i] == pool[p * B + i]
    assert phi2 == tau


def test_two_remaps_compose():
    shapes = tiny_shapes("f32")
    lay = L.build_layout(2, shapes, 128, 128 * 128)
    ws = random_weights(shapes, 4)
    pool = L.pack(lay, ws)
    p1, f1 = R.remap(pool, lay.phi, 1, 128)
    p2, f2 = R.remap(p1, f1, 2, 128)
    t1, t2 = R.matching(1, lay.P), R.matching(2, lay.P)
    assert f2 == [t2[t1[v]] for v in lay.phi]
    lay2 = L.Layout(**{**lay.__dict__, "phi": f2})
    for t in range(lay.T):
        assert np.array_equal(L.unpack(lay2, p2, t), ws[t])


@pytest.mark.parametrize("slice_pairs", [1, 5, 1000])
def test_remap_in_slices_keeps_every_tensor_between_slices(slice_pairs):
    shapes = tiny_shapes("bf16")
    lay = L.build_layout(8, shapes, 64, 64 * 257)       # odd pool: one page stays
    ws = random_weights(shapes, 4)
    pool = L.pack(lay, ws)
    states = list(R.remap_in_slices(pool, lay.phi, 77, 64, slice_pairs))
    assert len(states) == -(-(257 // 2) // slice_pairs)
    for pool_i, phi_i in states:
        assert sorted(phi_i) == list(range(lay.P))
        lay_i = L.Layout(**{**lay.__dict__, "phi": phi_i})
        for t in range(lay.T):
            assert np.array_equal(L.unpack(lay_i, pool_i, t), ws[t])
    # all slices together are the whole remap
    full_pool, full_phi = R.remap(pool, lay.phi, 77, 64)
    assert np.array_equal(states[-1][0], full_pool) and states[-1][1] == full_phi


def test_remap_slices_touch_only_their_pairs():
    P, B = 12, 4
    pool = np.arange(P * B, dtype=np.uint64).astype(np.uint8)
    todo = R.pairs(3, P)
    assert all(a < b for a, b in todo) and [a for a, _ in todo] == sorted(a for a, _ in todo)
    first = next(R.remap_in_slices(pool, list(range(P)), 3, B, 2))
    moved = {p for pr in todo[:2] for p in pr}
    for p in range(P):
        same = np.array_equal(first[0][p * B:(p + 1) * B], pool[p * B:(p + 1) * B])
        assert same == (p not in moved)


# ---------------------------------------------------------------- uniform remap

def test_uniform_draw_is_fisher_yates_on_its_own_substream():
    P = 11
    want = prng.fisher_yates(P, prng.substream(77, prng.TAG_REMAP, 1))
    assert R.uniform_draw(77, P) == want
    assert R.uniform_draw(77, P) != prng.fisher_yates(P, prng.substream(77, prng.TAG_REMAP, 0))


def test_uniform_remap_moves_each_page_to_rho_brute_force():
    P, B = 13, 8
    pool = (np.arange(P * B) * 7 % 251).astype(np.uint8)
    phi = prng.fisher_yates(P, prng.substream(3, prng.TAG_PAGE_MAP, 0))
    rho = R.uniform_draw(21, P)
    out, phi2 = R.remap_uniform(pool, phi, 21, B)
    for p in range(P):
        for i in range(B):
            assert out[rho[p] * B + i] == pool[p * B + i]
    for v in range(P):
        assert phi2[v] == rho[phi[v]]


@pytest.mark.parametrize("remap_seed", [1, 2, 3])
def test_uniform_remap_preserves_every_tensor(remap_seed):
    shapes = tiny_shapes("bf16")
    lay = L.build_layout(8, shapes, 64, 64 * 256)
    ws = random_weights(shapes, 3)
    pool = L.pack(lay, ws)
    pool2, phi2 = R.remap_uniform(pool, lay.phi, remap_seed, 64)
    assert sorted(phi2) == list(range(lay.P))
    lay2 = L.Layout(**{**lay.__dict__, "phi": phi2})
    for t in range(lay.T):
        assert np.array_equal(L.unpack(lay2, pool2, t), ws[t])


def test_uniform_remap_is_uniform_whatever_the_map():
    # chi-square of phi' over all 24 maps of a 4-page pool, from a fixed
    # non-identity phi: every map equally likely (23 degrees of freedom; the
    # 0.999 quantile is 49.7), and on average one page keeps its place
    import itertools
    phi = [2, 0, 3, 1]
    index = {p: i for i, p in enumerate(itertools.permutations(range(4)))}
    counts = np.zeros(24)
    fixed = 0
    n = 4800
    for s in range(n):
        _, phi2 = R.remap_uniform(np.zeros(4, np.uint8), phi, 1000 + s, 1)
        counts[index[tuple(phi2)]] += 1
        fixed += sum(phi2[v] == phi[v] for v in range(4))
    chi2 = float(np.sum((counts - n / 24) ** 2 / (n / 24)))
    assert chi2 < 49.7, chi2
    assert abs(fixed / n - 1.0) < 0.1


@pytest.mark.parametrize("P", [1, 2, 3, 5, 16, 257])
@pytest.mark.parametrize("seed", [4, 5])
def test_two_passes_of_disjoint_swaps_realise_rho(P, seed):
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    rho = R.uniform_draw(seed, P)
    one, two = R.uniform_passes(seed, P)
    where = list(range(P))        # where[item] = page holding it; item p starts on page p
    at = list(range(P))           # at[page] = item on it
    for pas in (one, two):
        touched = [x for pr in pas for x in pr]
        assert len(touched) == len(set(touched)), "a pass must be disjoint transpositions"
        assert pas == sorted(pas) and all(a < b for a, b in pas)
        for a, b in pas:
            ia, ib = at[a], at[b]
            at[a], at[b] = ib, ia
            where[ia], where[ib] = b, a
    assert where == rho
    # the fewest transpositions that realise rho: P minus its number of cycles
    g = coo_matrix((np.ones(P), (np.arange(P), np.array(rho))), shape=(P, P))
    ncyc, _ = connected_components(g, directed=True, connection="weak")
    assert len(one) + len(two) == P - ncyc


def test_uniform_slices_keep_every_tensor_and_end_at_the_whole_remap():
    shapes = tiny_shapes("f32")
    lay = L.build_layout(5, shapes, 64, 64 * 257)
    ws = random_weights(shapes, 4)
    pool = L.pack(lay, ws)
    one, two = R.uniform_passes(31, lay.P)
    states = list(R.remap_uniform_in_slices(pool, lay.phi, 31, 64, 10))
    assert len(states) == -(-len(one) // 10) + -(-len(two) // 10)
    for pool_k, phi_k in states:
        assert sorted(phi_k) == list(range(lay.P))
        lay_k = L.Layout(**{**lay.__dict__, "phi": phi_k})
        for t in range(lay.T):
            assert np.array_equal(L.unpack(lay_k, pool_k, t), ws[t])
    whole_pool, whole_phi = R.remap_uniform(pool, lay.phi, 31, 64)
    assert np.array_equal(states[-1][0], whole_pool) and states[-1][1] == whole_phi


def test_planted_pass_mistake_is_visible():
    # swapping the order of the two passes gives rho^-1 on cycles longer than 2
    rho = R.uniform_draw(8, 64)
    one, two = R.uniform_passes(8, 64)
    where, at = list(range(64)), list(range(64))
    for pas in (two, one):
        for a, b in pas:
            ia, ib = at[a], at[b]
            at[a], at[b] = ib, ia
            where[ia], where[ib] = b, a
    assert where != rho

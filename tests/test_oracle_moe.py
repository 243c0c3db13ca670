"""Pins for the oracle's MoE layer: reductions to the dense SwiGLU FFN (itself
pinned), linearity in the router weights, slot-order invariance, dropped
invalid slots, and an independent dense formulation through a one-hot
dispatch matrix."""

import numpy as np
import pytest

from oracle import moe as OM
from oracle import numerics as N


def experts(E, d, F, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [(rng.standard_normal((F, d)) * 0.1, rng.standard_normal((F, d)) * 0.1,
             rng.standard_normal((d, F)) * 0.1) for _ in range(E)]


def test_single_expert_weight_one_is_the_dense_ffn():
    ex = experts(5, 16, 24)
    x = np.random.Generator(np.random.PCG64(1)).standard_normal((3, 16))
    for e in range(5):
        y = OM.moe_ffn(x, np.full((3, 1), e), np.ones((3, 1)), ex)
        ref, _ = N.swiglu_ffn(x, *ex[e])
        assert np.allclose(y, ref, rtol=1e-13, atol=1e-13)


def test_linear_in_weights_and_invariant_to_slot_order():
    ex = experts(8, 16, 24, seed=2)
    rng = np.random.Generator(np.random.PCG64(3))
    x = rng.standard_normal((4, 16))
    ids = rng.integers(0, 8, (4, 3))
    w = rng.standard_normal((4, 3))
    y = OM.moe_ffn(x, ids, w, ex)
    assert np.allclose(OM.moe_ffn(x, ids, 2.5 * w, ex), 2.5 * y, rtol=1e-12, atol=1e-12)
    perm = [2, 0, 1]
    assert np.allclose(OM.moe_ffn(x, ids[:, perm], w[:, perm], ex), y, rtol=1e-12, atol=1e-12)
    # two slots naming the same expert add up
    same = OM.moe_ffn(x, np.stack([ids[:, 0], ids[:, 0]], 1), np.stack([w[:, 0], w[:, 0]], 1), ex)
    assert np.allclose(same, 2 * OM.moe_ffn(x, ids[:, :1], w[:, :1], ex), rtol=1e-12, atol=1e-12)


def test_invalid_slots_contribute_nothing():
    ex = experts(4, 8, 8, seed=4)
    x = np.ones((2, 8))
    ids = np.array([[1, -1], [4, 2]])
    w = np.array([[0.5, 9.0], [9.0, 0.25]])
    y = OM.moe_ffn(x, ids, w, ex)
    want = OM.moe_ffn(x, np.array([[1], [2]]), np.array([[0.5], [0.25]]), ex)
    assert np.allclose(y, want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("seed", [5, 6])
def test_dense_dispatch_formulation(seed):
    # y = sum_e diag(D[:, e]) FFN_e(X), D[m][e] = sum of the weights of token m's slots naming e
    E, d, F, M, k = 6, 12, 20, 7, 2
    ex = experts(E, d, F, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 10))
    x = rng.standard_normal((M, d))
    ids = rng.integers(0, E, (M, k))
    w = rng.random((M, k))
    D = np.zeros((M, E))
    for m in range(M):
        for j in range(k):
            D[m, ids[m, j]] += w[m, j]
    want = sum(D[:, e:e + 1] * N.swiglu_ffn(x, *ex[e])[0] for e in range(E))
    assert np.allclose(OM.moe_ffn(x, ids, w, ex), want, rtol=1e-12, atol=1e-12)

"""Pins for the oracle's generator, bounded draw and Fisher-Yates permutation."""

import itertools
import os

import numpy as np
import pytest

from oracle import prng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class Scripted:
    """Stand-in generator that returns a fixed list of 64-bit outputs."""

    def __init__(self, values):
        self.values = list(values)

    def next_u64(self):
        return self.values.pop(0)


def test_splitmix64_published_vectors():
    want = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if l.strip() and not l.startswith("#")]
    g = prng.SplitMix64(0)
    assert [g.next_u64() for _ in want] == want


def _unxorshift(z, s):
    x = z
    for _ in range(64 // s + 1):
        x = z ^ (x >> s)
    return x & prng.MASK64


def test_mix64_is_the_published_bijection():
    # Invert each step independently: xor-shift right is inverted by
    # iteration, odd multipliers by their inverse modulo 2**64.
    inv1 = pow(0xBF58476D1CE4E5B9, -1, 1 << 64)
    inv2 = pow(0x94D049BB133111EB, -1, 1 << 64)
    rng = np.random.Generator(np.random.PCG64(3))
    for z in [0, 1, prng.MASK64] + [int(v) for v in rng.integers(0, 2**63, 200, dtype=np.int64)]:
        y = prng.mix64(z)
        y = _unxorshift(y, 31)
        y = (y * inv2) & prng.MASK64
        y = _unxorshift(y, 27)
        y = (y * inv1) & prng.MASK64
        y = _unxorshift(y, 30)
        assert y == z


def test_substreams_are_distinct():
    firsts = set()
    for tag in range(1, 6):
        for idx in range(50):
            firsts.add(prng.substream(1, tag, idx).next_u64())
    assert len(firsts) == 250
    with pytest.raises(ValueError):
        prng.substream(1, 2, 1 << 32)


def test_bounded_rejects_biased_low_outputs():
    # 2**64 mod 3 == 1: the single output 0 must be rejected.
    assert prng.bounded(Scripted([0, 5]), 3) == 2
    # 2**64 mod 10 == 6: outputs 0..5 rejected, 6 accepted (6 mod 10).
    assert prng.bounded(Scripted([0, 3, 5, 6]), 10) == 6
    # powers of two reject nothing
    assert prng.bounded(Scripted([0]), 8) == 0
    assert prng.bounded(Scripted([prng.MASK64]), 1) == 0


def test_bounded_is_uniform_chi2():
    g = prng.SplitMix64(12345)
    n, draws = 7, 70000
    counts = np.bincount([prng.bounded(g, n) for _ in range(draws)], minlength=n)
    expected = draws / n
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    assert chi2 < 22.46  # p = 0.001 for 6 degrees of freedom


def test_fisher_yates_scripted_walk():
    # n = 4, draws for i = 3, 2, 1: 6 mod 4 = 2, 7 mod 3 = 1, 5 mod 2 = 1.
    # Worked by hand: [0,1,2,3] -> swap(3,2) -> [0,1,3,2] -> swap(2,1) ->
    # [0,3,1,2] -> swap(1,1) -> [0,3,1,2].
    assert prng.fisher_yates(4, Scripted([6, 7, 5])) == [0, 3, 1, 2]


def test_fisher_yates_reaches_every_permutation_once():
    # Each draw sequence (j3, j2, j1) in [0,4) x [0,3) x [0,2) must give a
    # different permutation: the algorithm is a bijection onto S_4.
    perms = set()
    for j3, j2, j1 in itertools.product(range(4), range(3), range(2)):
        perms.add(tuple(prng.fisher_yates(4, Scripted([j3, j2 + 3, j1]))))
    assert perms == set(itertools.permutations(range(4)))


def test_fisher_yates_uniform_chi2():
    counts = {}
    seeds = 6000
    for s in range(seeds):
        p = tuple(prng.fisher_yates(3, prng.substream(s, 1, 0)))
        counts[p] = counts.get(p, 0) + 1
    assert len(counts) == 6
    exp = seeds / 6
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < 20.52  # p = 0.001 for 5 degrees of freedom


@pytest.mark.parametrize("n", [0, 1, 2, 17, 1000])
def test_fisher_yates_is_permutation(n):
    p = prng.fisher_yates(n, prng.substream(99, 2, 3))
    assert sorted(p) == list(range(n))


# ---------------------------------------------------------------- counter-mode SHA-256 streams

def test_sha256_primitive_known_answers():
    # FIPS 180-4 example messages: the empty string and "abc"
    import hashlib
    assert hashlib.sha256(b"").hexdigest() == \
        "e3b0c44298fc1c149afbf4c8996fb92427ae41e4649b934ca495991b7852b855"
    assert hashlib.sha256(b"abc").hexdigest() == \
        "ba7816bf8f01cfea414140de5dae2223b00361a396177a9cb410ff61f20015ad"


def test_csprng_words_follow_the_counter_construction():
    import hashlib
    import struct
    g = prng.substream_csprng(0x0123456789ABCDEF, 3, 7)
    words = [g.next_u64() for _ in range(9)]
    for j, w in enumerate(words):
        msg = (0x0123456789ABCDEF).to_bytes(8, "little") + (3).to_bytes(4, "little") + \
            (7).to_bytes(4, "little") + (j // 4).to_bytes(8, "little")
        block = hashlib.sha256(msg).digest()
        assert w == struct.unpack_from("<Q", block, 8 * (j % 4))[0]
    # distinct (tag, idx) give unrelated streams; the seed is masked to 64 bits
    assert words[0] != prng.substream_csprng(0x0123456789ABCDEF, 3, 8).next_u64()
    assert prng.substream_csprng(-1, 1, 0).next_u64() == prng.substream_csprng((1 << 64) - 1, 1, 0).next_u64()


def test_csprng_permutations_are_uniform_on_small_n():
    # all 24 permutations of 4 items, chi-square over 4800 sub-streams
    from collections import Counter
    cnt = Counter(tuple(prng.fisher_yates(4, prng.substream_csprng(s, 2, 0))) for s in range(4800))
    assert len(cnt) == 24
    chi2 = sum((c - 200) ** 2 / 200 for c in cnt.values())
    assert chi2 < 49.7      # 23 degrees of freedom, p = 0.001

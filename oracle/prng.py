"""Seeded randomness behind every layout decision (oracle).

The paper seeds a pseudo-random generator from the operating system's entropy
source before deployment, then enumerates virtual addresses, computes a random
permutation and allocates physical pages from it, all before any weight
transfer (Section 5, Implementation Details).  It does not name the generator
or the permutation algorithm.

Readings taken here (listed with the other readings in the design notes):

* Generator: SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast Splittable
  Pseudorandom Number Generators", OOPSLA 2014): a 64-bit Weyl-sequence state
  advanced by the golden-ratio increment, each output passed through a
  bijective 64-bit finaliser (xor-shift 30, multiply, xor-shift 27, multiply,
  xor-shift 31, "variant 13" constants).
* Independent sub-streams: ``state0 = mix64(seed XOR mix64((tag << 32) | idx))``
  with tags 1 tensor order, 2 hidden permutation of layer ``idx``, 3 page map,
  4 upload order of tensor ``idx``, 5 remap matching (keyed by the remap seed),
  6 attention-head permutation of layer ``idx``.
* Bounded draw: rejection of the ``2**64 mod n`` lowest outputs, then
  ``r mod n`` -- exactly uniform on ``[0, n)``.
* Permutation: Fisher-Yates in Durstenfeld's in-place form, walking ``i`` from
  ``n-1`` down to ``1`` and swapping ``a[i]`` with ``a[bounded(i+1)]``.

Cryptographic alternative (layouts built with the CSPRNG flag): the same
sub-streams, but word ``j`` of sub-stream (seed, tag, idx) is bytes
``8*(j % 4) .. 8*(j % 4) + 7`` (little-endian) of
``SHA-256(seed_le64 || tag_le32 || idx_le32 || (j // 4)_le64)`` -- SHA-256
(FIPS 180-4) in counter mode, so that no output reveals the seed or another
output.  Bounded draws and Fisher-Yates are unchanged.

Pure Python integers, no vectorisation: this is the definition written out.
"""

import hashlib
import struct

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15  # 2**64 / golden ratio, odd

TAG_TENSOR_ORDER = 1
TAG_HIDDEN_PERM = 2
TAG_PAGE_MAP = 3
TAG_UPLOAD_ORDER = 4
TAG_REMAP = 5
TAG_HEAD_PERM = 6


def mix64(z: int) -> int:
    """SplitMix64 output finaliser (a bijection on 64-bit words)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


class SplitMix64:
    """One SplitMix64 stream: advance the Weyl state, return its mix."""

    def __init__(self, state: int):
        self.state = state & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + GOLDEN_GAMMA) & MASK64
        return mix64(self.state)


def substream(seed: int, tag: int, idx: int) -> SplitMix64:
    """Independent stream for (seed, purpose tag, index)."""
    if not (0 <= idx < (1 << 32)):
        raise ValueError("sub-stream index must fit in 32 bits")
    return SplitMix64(mix64((seed & MASK64) ^ mix64((tag << 32) | idx)))


class Sha256Ctr:
    """Counter-mode SHA-256 word stream for (seed, tag, idx)."""

    def __init__(self, seed: int, tag: int, idx: int):
        self.prefix = struct.pack("<QII", seed & MASK64, tag, idx)
        self.j = 0
        self.block = b""

    def next_u64(self) -> int:
        if self.j % 4 == 0:
            self.block = hashlib.sha256(self.prefix + struct.pack("<Q", self.j // 4)).digest()
        w = int.from_bytes(self.block[8 * (self.j % 4):8 * (self.j % 4) + 8], "little")
        self.j += 1
        return w


def substream_csprng(seed: int, tag: int, idx: int) -> Sha256Ctr:
    if not (0 <= idx < (1 << 32)):
        raise ValueError("sub-stream index must fit in 32 bits")
    return Sha256Ctr(seed, tag, idx)


def bounded(rng, n: int) -> int:
    """Uniform integer in [0, n) by rejection of the biased low outputs."""
    if n <= 0:
        raise ValueError("bounded(n) needs n >= 1")
    threshold = (1 << 64) % n
    while True:
        r = rng.next_u64()
        if r >= threshold:
            return r % n


def fisher_yates(n: int, rng) -> list:
    """Uniform permutation of range(n) (gather convention: slot j holds a[j])."""
    a = list(range(n))
    for i in range(n - 1, 0, -1):
        j = bounded(rng, i + 1)
        a[i], a[j] = a[j], a[i]
    return a

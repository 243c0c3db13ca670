"""Decoy contents of the free pages (oracle).

The paper leaves the pages of the pool that hold no weights unspecified
(Section 4.2 only requires the page map to scatter tensors over the pool).
Zero-filled free pages tell an observer which pages carry weights, so the
hardened layout fills them with weight-like bytes.  Reading (written out
identically in include/cloak.h):

* Decoys are keyed by their own ``decoy_seed``, never by the layout seed:
  SplitMix64 is invertible, and decoy bytes derived from the layout seed would
  hand it to whoever reads a free page.
* Free virtual page ``v`` (``V <= v < P``) uses the SplitMix64 stream of
  sub-stream(decoy_seed, tag 7, idx v); element ``e`` of the page takes
  outputs ``3e, 3e+1, 3e+2`` of that stream (``r_j = mix64(s0 + (j+1)*gamma)``).
* ``S`` = sum of the twelve 16-bit pieces of those three words (an
  Irwin-Hall(12) draw, 0..786420), ``C = 2S - 786420`` (mean 0, standard
  deviation ~2**17).
* Element value, exact in binary32 (``|C|*5 < 2**24``): f32 and bf16 decoys
  ``C*5 * 2**-25`` (sd ~0.0195, then bf16 nearest-even); fp8 decoys
  ``C*3 * 2**-12`` (sd ~96, like per-row scaled E4M3 weight codes), then E4M3
  nearest-even, saturating at 448.
* Element type: the storage type holding the most tensor bytes in the layout
  (ties: fp8, then bf16, then f32; bf16 for an empty layout).
"""

import numpy as np

from . import layout as OL
from . import numerics as ON
from . import prng

TAG_DECOY = 7
_MASK = np.uint64((1 << 64) - 1)


def mix64_np(z):
    """SplitMix64 finaliser on a uint64 array (NumPy wraps products mod 2**64)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def stream_words(decoy_seed, v, count):
    """Outputs 0..count-1 of the SplitMix64 stream (decoy_seed, tag 7, idx v)."""
    s0 = np.uint64(prng.substream(decoy_seed, TAG_DECOY, v).state)
    j = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64_np(s0 + j * np.uint64(prng.GOLDEN_GAMMA))


def centred_sums(decoy_seed, v, n_elems):
    """C = 2*S - 786420 per element, S the sum of twelve 16-bit pieces."""
    w = stream_words(decoy_seed, v, 3 * n_elems).reshape(n_elems, 3)
    pieces = w.view(np.uint16).reshape(n_elems, 12).astype(np.int64)   # little-endian 16-bit pieces
    return 2 * pieces.sum(axis=1) - 786420


def decoy_dtype(layout):
    total = {"fp8": 0, "bf16": 0, "f32": 0}
    for s in layout.shapes:
        total[s.dtype] += s.nbytes
    if not any(total.values()):
        return "bf16"
    return max(("fp8", "bf16", "f32"), key=lambda d: (total[d], -("fp8", "bf16", "f32").index(d)))


def decoy_page(decoy_seed, v, page_bytes, dtype):
    """The bytes of free virtual page v."""
    n = page_bytes // OL.ELT_BYTES[dtype]
    c = centred_sums(decoy_seed, v, n)
    if dtype == "fp8":
        vals = (c * 3).astype(np.float32) * np.float32(2.0 ** -12)
        return ON.f64_to_e4m3_bits_rne(vals.astype(np.float64)).view(np.uint8)
    vals = (c * 5).astype(np.float32) * np.float32(2.0 ** -25)
    if dtype == "f32":
        return vals.view(np.uint8)
    return ON.f32_to_bf16_bits_rne(vals).view(np.uint8)


def fill_decoys(layout, pool, decoy_seed):
    """Write the decoy of every free virtual page to its physical page (in place)."""
    B = layout.page_bytes
    dt = decoy_dtype(layout)
    for v in range(layout.V, layout.P):
        p = layout.phi[v]
        pool[p * B:(p + 1) * B] = decoy_page(decoy_seed, v, B, dt)
    return pool

"""In-place re-randomisation of physical page placement (oracle).

The paper re-randomises the virtual-to-physical page mapping periodically,
with no extra memory footprint, paying only synchronisation points that the
operator amortises by choosing the cadence (Section 4.2, "Physical page
remapping"; Section 5.2; Figure 7).  It does not say how the pages move.

Reading: a seeded random perfect matching ``tau`` of the pool's pages.  Draw
``s`` = Fisher-Yates(P, tag 5) from the remap seed and pair ``s[2i]`` with
``s[2i+1]`` for ``i < P // 2`` (with odd ``P`` the last page stays put).  Each
pair swaps contents, so the move needs no scratch page: the page that held
physical page ``p`` now sits at ``tau[p]``, and the map becomes
``phi' = tau o phi``.
"""

import numpy as np

from . import prng


def matching(remap_seed, P, csprng=False):
    """tau as an array: tau[p] is the page that p swaps with (an involution).
    ``csprng`` draws the words from counter-mode SHA-256 (layouts built so)."""
    sub = prng.substream_csprng if csprng else prng.substream
    s = prng.fisher_yates(P, sub(remap_seed, prng.TAG_REMAP, 0))
    tau = list(range(P))
    for i in range(P // 2):
        a, b = s[2 * i], s[2 * i + 1]
        tau[a], tau[b] = b, a
    return tau


def remap(pool, phi, remap_seed, page_bytes, csprng=False):
    """Return (pool', phi') after one remap; the inputs are not modified."""
    P = len(phi)
    tau = matching(remap_seed, P, csprng)
    B = page_bytes
    out = np.empty_like(pool)
    for p in range(P):
        q = tau[p]
        out[q * B:(q + 1) * B] = pool[p * B:(p + 1) * B]
    phi2 = [tau[phi[v]] for v in range(P)]
    return out, phi2


# ----------------------------------------------------------------------------
# Incremental remap.  The paper amortises the remap's synchronisation cost by
# choosing when it runs (Section 4.2; Figure 7 sweeps the cadence).  Reading
# for spreading one remap over several serving steps: the pairs of tau, taken
# in ascending order of their lower page, are applied in consecutive slices;
# after each slice the moved pages' entries of phi are updated, so between
# slices the pool and phi are a consistent layout (the pairs are disjoint
# transpositions, so the slices commute and together equal tau).
# ----------------------------------------------------------------------------

def pairs(remap_seed, P, csprng=False):
    """Pairs (p, tau[p]) with p < tau[p], ascending in p."""
    tau = matching(remap_seed, P, csprng)
    return [(p, tau[p]) for p in range(P) if tau[p] > p]


def remap_in_slices(pool, phi, remap_seed, page_bytes, slice_pairs, csprng=False):
    """Yield (pool_i, phi_i) after each slice of at most slice_pairs pairs."""
    if slice_pairs < 1:
        raise ValueError("slice_pairs must be positive")
    B = page_bytes
    pool = pool.copy()
    phi = list(phi)
    where = {phi[v]: v for v in range(len(phi))}   # physical page -> virtual page
    todo = pairs(remap_seed, len(phi), csprng)
    for i0 in range(0, len(todo), slice_pairs):
        for a, b in todo[i0:i0 + slice_pairs]:
            pa = pool[a * B:(a + 1) * B].copy()
            pool[a * B:(a + 1) * B] = pool[b * B:(b + 1) * B]
            pool[b * B:(b + 1) * B] = pa
            va, vb = where[a], where[b]
            phi[va], phi[vb] = b, a
            where[a], where[b] = vb, va
        yield pool.copy(), list(phi)

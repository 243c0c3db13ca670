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


def matching(remap_seed, P):
    """tau as an array: tau[p] is the page that p swaps with (an involution)."""
    s = prng.fisher_yates(P, prng.substream(remap_seed, prng.TAG_REMAP, 0))
    tau = list(range(P))
    for i in range(P // 2):
        a, b = s[2 * i], s[2 * i + 1]
        tau[a], tau[b] = b, a
    return tau


def remap(pool, phi, remap_seed, page_bytes):
    """Return (pool', phi') after one remap; the inputs are not modified."""
    P = len(phi)
    tau = matching(remap_seed, P)
    B = page_bytes
    out = np.empty_like(pool)
    for p in range(P):
        q = tau[p]
        out[q * B:(q + 1) * B] = pool[p * B:(p + 1) * B]
    phi2 = [tau[phi[v]] for v in range(P)]
    return out, phi2

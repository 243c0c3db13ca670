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


# ----------------------------------------------------------------------------
# Uniform remap (layouts built with the uniform-remap flag).  One matching
# re-draw leaves phi' = tau o phi confined to involutions of phi: no page ever
# stays where it is, and a page's new place gives away its partner's.  The
# uniform reading draws a fresh permutation rho of all pool pages and moves
# the contents of physical page p to physical page rho[p], so the new map
# phi' = rho o phi is a uniform draw whatever phi was (Section 4.2 asks for
# the map to be re-randomised, with no extra memory).
#
# rho = Fisher-Yates(P) on sub-stream (remap_seed, tag 5, idx 1).
#
# In place it runs as two passes of disjoint page-pair swaps (no scratch
# page).  Each cycle of rho is listed from its smallest page c_0, with
# c_{i+1} = rho[c_i], length k.  The shift i -> i+1 (mod k) is the
# reflection i -> -i followed by the reflection i -> 1-i:
#   pass 1 swaps c_i with c_{k-i} for 1 <= i < k-i,
#   pass 2 swaps c_i with c_{(1-i) mod k} for the pairs with i < (1-i) mod k,
#          i.e. (c_0, c_1), (c_2, c_{k-1}), (c_3, c_{k-2}), ...
# Within a pass the pairs are taken in ascending order of their lower page.
# ----------------------------------------------------------------------------

def uniform_draw(remap_seed, P, csprng=False):
    """rho as a list: the contents of physical page p move to page rho[p]."""
    sub = prng.substream_csprng if csprng else prng.substream
    return prng.fisher_yates(P, sub(remap_seed, prng.TAG_REMAP, 1))


def remap_uniform(pool, phi, remap_seed, page_bytes, csprng=False):
    """Return (pool', phi') after one uniform remap (the definition: every
    page's contents land on rho[p] at once); inputs are not modified."""
    P = len(phi)
    rho = uniform_draw(remap_seed, P, csprng)
    B = page_bytes
    out = np.empty_like(pool)
    for p in range(P):
        out[rho[p] * B:(rho[p] + 1) * B] = pool[p * B:(p + 1) * B]
    return out, [rho[phi[v]] for v in range(P)]


def cycles(perm):
    """Cycles of a permutation, each listed from its smallest element."""
    seen = [False] * len(perm)
    out = []
    for start in range(len(perm)):
        if seen[start]:
            continue
        c, p = [], start
        while not seen[p]:
            seen[p] = True
            c.append(p)
            p = perm[p]
        out.append(c)
    return out


def uniform_passes(remap_seed, P, csprng=False):
    """(pass1, pass2): lists of page pairs (lo, hi), each ascending in lo."""
    rho = uniform_draw(remap_seed, P, csprng)
    one, two = [], []
    for c in cycles(rho):
        k = len(c)
        for i in range(k):
            j = (k - i) % k
            if i < j:
                one.append((min(c[i], c[j]), max(c[i], c[j])))
            j = (1 - i) % k
            if i < j:
                two.append((min(c[i], c[j]), max(c[i], c[j])))
    return sorted(one), sorted(two)


def remap_uniform_in_slices(pool, phi, remap_seed, page_bytes, slice_pairs, csprng=False):
    """Yield (pool_i, phi_i) after each slice: pass 1's pairs, then pass 2's,
    in slices of at most slice_pairs pairs that never span both passes."""
    if slice_pairs < 1:
        raise ValueError("slice_pairs must be positive")
    B = page_bytes
    pool = pool.copy()
    phi = list(phi)
    where = {phi[v]: v for v in range(len(phi))}
    for todo in uniform_passes(remap_seed, len(phi), csprng):
        for i0 in range(0, len(todo), slice_pairs):
            for a, b in todo[i0:i0 + slice_pairs]:
                pa = pool[a * B:(a + 1) * B].copy()
                pool[a * B:(a + 1) * B] = pool[b * B:(b + 1) * B]
                pool[b * B:(b + 1) * B] = pa
                va, vb = where[a], where[b]
                phi[va], phi[vb] = b, a
                where[a], where[b] = vb, va
            yield pool.copy(), list(phi)

"""Cloaked weight layout: shuffles, virtual pages, page map, pack/unpack (oracle).

What the paper fixes (CloakLM, arXiv 2606.18400):

* Inter-layer randomisation (Section 4.2, paragraph on virtual address
  shuffling; Table 1a): tensors cross the bus and take their virtual
  addresses in a seeded order unrelated to the model's layer order, so
  neighbouring address ranges say nothing about neighbouring layers.
* Intra-layer shuffling is named in the abstract without a mechanism.
  Reading: a seeded permutation of each FFN's hidden neurons -- rows of gate
  and up, columns of down -- which leaves the FFN function unchanged.  The
  same reading extends to attention when q/k/v/o carry a head size: whole
  key/value head groups are permuted, the query heads inside a group are
  permuted, and the value dimensions inside a head are permuted, all in ways
  the attention function cannot see (query/key dimensions stay in place: the
  rotary embedding pairs them by position inside the head).
* Page scattering (Section 4.2, paragraph on physical page remapping;
  Table 1b): the pages of a tensor land on physical pages of a pool that are
  neither adjacent nor in order.  Pages are 2 MB in the paper; any power of two works.
* Everything is drawn from the seeded generator before any weight is
  transferred (Section 5, Implementation Details).

Conventions (readings, shared by the library only through this written
definition, never through code):

* A tensor is stored as the nn.Linear array ``W[N][K]`` (output channel ``n``
  is row ``n``, K contiguous).  Element sizes: f32 4, bf16 2, fp8-e4m3 1.
* Tensor index ``t`` is the caller's order (layer-major).  ``sigma`` =
  Fisher-Yates(T, tag 1): tensor ``sigma[i]`` is placed i-th in the virtual
  page stream, each tensor starting on a fresh page.
* ``pi[l]`` = Fisher-Yates(d_ffn, tag 2, idx l).  Shuffled storage is
  ``gate_s[j] = gate[pi[j]]``, ``up_s[j] = up[pi[j]]``, ``down_s[:, j] =
  down[:, pi[j]]`` (gather convention: slot ``j`` holds item ``pi[j]``).
* Attention heads of layer ``l`` (only when its q/k/v/o carry a head size
  ``hd``; ``Hq = q.n_out / hd`` query heads, ``Hkv = k.n_out / hd`` key/value
  heads, ``G = Hq / Hkv``): one stream ``g`` = sub-stream(tag 6, idx l) draws,
  in this order, ``rho`` = Fisher-Yates(Hkv, g), then ``theta[c]`` =
  Fisher-Yates(G, g) for c = 0..Hkv-1, then ``chi`` = Fisher-Yates(hd, g).
  Stored key/value head ``c`` holds logical head ``rho[c]``; stored query
  head ``c*G + i`` holds logical query head ``rho[c]*G + theta[c][i]``; value
  dimension ``d`` of a stored head holds logical dimension ``chi[d]``.  Rows of
  q and k keep their dimension order, rows of v and columns of o take ``chi``.
* ``phi`` = Fisher-Yates(P, tag 3) over all ``P = pool_bytes / page_bytes``
  pages: virtual page ``v`` lives at physical page ``phi[v]``; virtual pages
  ``V..P-1`` are the free pages, which hold zeros.
* Upload order of tensor ``t``'s pages: Fisher-Yates(npages_t, tag 4, idx t).
* With ``identity=True`` every permutation is the identity: the plain
  contiguous, layer-ordered layout used as the uncloaked comparator.
* With ``csprng=True`` every sub-stream above draws its words from counter-mode
  SHA-256 instead of SplitMix64 (``prng.substream_csprng``).
"""

import numpy as np

from . import prng

KINDS = ("q", "k", "v", "o", "gate", "up", "down", "embed", "head")
ATTN_KINDS = ("q", "k", "v", "o")
ELT_BYTES = {"f32": 4, "bf16": 2, "fp8": 1}
STORAGE_DTYPE = {"f32": np.float32, "bf16": np.uint16, "fp8": np.uint8}
FFN_ROW_PERMUTED = ("gate", "up")   # hidden dim is N: rows permuted
FFN_COL_PERMUTED = ("down",)        # hidden dim is K: columns permuted


class Shape:
    """One weight tensor: (layer, kind, n_out, k_in, dtype[, head_dim]).

    ``head_dim`` (q/k/v/o only) asks for the attention-head permutation; 0
    leaves attention unpermuted.
    """

    def __init__(self, layer, kind, n_out, k_in, dtype, head_dim=0):
        if kind not in KINDS:
            raise ValueError(f"unknown kind {kind}")
        if dtype not in ELT_BYTES:
            raise ValueError(f"unknown dtype {dtype}")
        if head_dim and kind not in ATTN_KINDS:
            raise ValueError("only q/k/v/o carry a head size")
        self.layer, self.kind = int(layer), kind
        self.n_out, self.k_in, self.dtype = int(n_out), int(k_in), dtype
        self.head_dim = int(head_dim)

    @property
    def nbytes(self):
        return self.n_out * self.k_in * ELT_BYTES[self.dtype]

    def __repr__(self):
        hd = f",hd={self.head_dim}" if self.head_dim else ""
        return f"Shape({self.layer},{self.kind},{self.n_out},{self.k_in},{self.dtype}{hd})"


class Layout:
    """Plain record of every layout decision (all lists of Python ints)."""

    def __init__(self, **kw):
        self.__dict__.update(kw)

    def hidden_dim_of(self, t):
        s = self.shapes[t]
        if s.kind in FFN_ROW_PERMUTED:
            return s.n_out
        if s.kind in FFN_COL_PERMUTED:
            return s.k_in
        return None

    def row_perm(self, t):
        """Stored row j of tensor t holds logical row p[j] (None: unpermuted)."""
        s = self.shapes[t]
        if s.kind in FFN_ROW_PERMUTED:
            return list(self.pi[s.layer])
        if s.kind in ("q", "k", "v") and s.layer in self.heads:
            a = self.heads[s.layer]
            hd, G = a["head_dim"], a["group"]
            out = []
            if s.kind == "q":
                for c in range(a["n_kv"]):
                    for i in range(G):
                        h = a["rho"][c] * G + a["theta"][c][i]
                        out += [h * hd + d for d in range(hd)]
            else:
                dims = a["chi"] if s.kind == "v" else list(range(hd))
                for c in range(a["n_kv"]):
                    out += [a["rho"][c] * hd + dims[d] for d in range(hd)]
            return out
        return None

    def col_perm(self, t):
        """Stored column j of tensor t holds logical column p[j] (None: unpermuted)."""
        s = self.shapes[t]
        if s.kind in FFN_COL_PERMUTED:
            return list(self.pi[s.layer])
        if s.kind == "o" and s.layer in self.heads:
            a = self.heads[s.layer]
            hd, G = a["head_dim"], a["group"]
            out = []
            for c in range(a["n_kv"]):
                for i in range(G):
                    h = a["rho"][c] * G + a["theta"][c][i]
                    out += [h * hd + a["chi"][d] for d in range(hd)]
            return out
        return None


def build_layout(seed, shapes, page_bytes, pool_bytes, identity=False, csprng=False):
    """Draw sigma, pi_l, the virtual page assignment and phi."""
    sub = prng.substream_csprng if csprng else prng.substream
    if page_bytes <= 0 or pool_bytes % page_bytes != 0:
        raise ValueError("pool_bytes must be a positive multiple of page_bytes")
    T = len(shapes)
    P = pool_bytes // page_bytes

    # Inter-layer shuffle: the order tensors occupy the virtual page stream.
    sigma = list(range(T)) if identity else prng.fisher_yates(
        T, sub(seed, prng.TAG_TENSOR_ORDER, 0))

    # Intra-layer shuffle: one hidden-neuron permutation per FFN layer.
    d_ffn = {}
    seen = set()
    for s in shapes:
        if (s.layer, s.kind) in seen:
            raise ValueError(f"duplicate tensor {s}")
        seen.add((s.layer, s.kind))
        h = s.n_out if s.kind in FFN_ROW_PERMUTED else (
            s.k_in if s.kind in FFN_COL_PERMUTED else None)
        if h is None:
            continue
        if d_ffn.setdefault(s.layer, h) != h:
            raise ValueError(f"inconsistent hidden size in layer {s.layer}")
    pi = {}
    for layer, h in sorted(d_ffn.items()):
        pi[layer] = list(range(h)) if identity else prng.fisher_yates(
            h, sub(seed, prng.TAG_HIDDEN_PERM, layer))

    heads = {layer: _draw_heads(sub, seed, layer, four, identity)
             for layer, four in sorted(_attention_groups(shapes).items())}

    # Virtual pages: tensors in sigma order, each starting on a fresh page.
    npages = [-(-s.nbytes // page_bytes) for s in shapes]
    vbase = [0] * T
    cursor = 0
    for i in range(T):
        t = sigma[i]
        vbase[t] = cursor
        cursor += npages[t]
    V = cursor
    if V > P:
        raise MemoryError(f"layout needs {V} pages, pool has {P}")

    # Physical placement: a bijection over every page of the pool.
    phi = list(range(P)) if identity else prng.fisher_yates(
        P, sub(seed, prng.TAG_PAGE_MAP, 0))

    return Layout(seed=seed, shapes=list(shapes), page_bytes=page_bytes,
                  pool_bytes=pool_bytes, P=P, V=V, T=T, sigma=sigma, pi=pi, heads=heads,
                  npages=npages, vbase=vbase, phi=phi, identity=identity, csprng=csprng)


def _attention_groups(shapes):
    """Layers whose q/k/v/o carry a head size -> {kind: Shape}, validated."""
    groups = {}
    for s in shapes:
        if s.head_dim:
            groups.setdefault(s.layer, {})[s.kind] = s
    for layer, four in groups.items():
        if layer < 0:
            raise ValueError("attention-head permutation needs a layer index >= 0")
        if set(four) != set(ATTN_KINDS):
            raise ValueError(f"layer {layer}: q, k, v and o must all carry the head size")
        hd = four["q"].head_dim
        q, k, v, o = (four[x] for x in ATTN_KINDS)
        if any(x.head_dim != hd for x in (k, v, o)):
            raise ValueError(f"layer {layer}: head sizes disagree")
        if (q.n_out % hd or k.n_out % hd or k.n_out != v.n_out or o.k_in != q.n_out
                or not (q.k_in == k.k_in == v.k_in) or (q.n_out // hd) % (k.n_out // hd)):
            raise ValueError(f"layer {layer}: q/k/v/o sizes do not form whole heads")
    return groups


def _draw_heads(sub, seed, layer, four, identity):
    hd = four["q"].head_dim
    n_kv = four["k"].n_out // hd
    G = four["q"].n_out // hd // n_kv
    if identity:
        rho, theta, chi = list(range(n_kv)), [list(range(G)) for _ in range(n_kv)], list(range(hd))
    else:
        g = sub(seed, prng.TAG_HEAD_PERM, layer)
        rho = prng.fisher_yates(n_kv, g)
        theta = [prng.fisher_yates(G, g) for _ in range(n_kv)]
        chi = prng.fisher_yates(hd, g)
    return dict(head_dim=hd, n_kv=n_kv, group=G, rho=rho, theta=theta, chi=chi)


def upload_order(layout, t):
    """Seeded order in which tensor t's virtual pages cross the bus."""
    n = layout.npages[t]
    if layout.identity:
        return list(range(n))
    sub = prng.substream_csprng if getattr(layout, "csprng", False) else prng.substream
    return prng.fisher_yates(n, sub(layout.seed, prng.TAG_UPLOAD_ORDER, t))


def shuffle_tensor(layout, t, w):
    """Logical nn.Linear array -> stored (hidden-neuron / head permuted) array."""
    s = layout.shapes[t]
    w = np.asarray(w)
    assert w.shape == (s.n_out, s.k_in)
    rp, cp = layout.row_perm(t), layout.col_perm(t)
    if rp is not None:
        w = w[np.asarray(rp), :]
    if cp is not None:
        w = w[:, np.asarray(cp)]
    return w


def unshuffle_tensor(layout, t, ws):
    """Inverse of shuffle_tensor (scatter back through the permutations)."""
    rp, cp = layout.row_perm(t), layout.col_perm(t)
    out = np.array(ws, copy=True)
    if cp is not None:
        tmp = np.empty_like(out)
        tmp[:, np.asarray(cp)] = out
        out = tmp
    if rp is not None:
        tmp = np.empty_like(out)
        tmp[np.asarray(rp), :] = out
        out = tmp
    return out


def shuffle_scales(layout, t, scales):
    """Per-output-channel scales follow the rows they belong to."""
    scales = np.asarray(scales, dtype=np.float32)
    rp = layout.row_perm(t)
    return scales if rp is None else scales[np.asarray(rp)]


def tensor_stream(layout, t, w):
    """Virtual byte stream of tensor t: shuffled rows, row-major, zero padded."""
    s = layout.shapes[t]
    ws = np.ascontiguousarray(shuffle_tensor(layout, t, w).astype(STORAGE_DTYPE[s.dtype]))
    raw = ws.view(np.uint8).reshape(-1)
    out = np.zeros(layout.npages[t] * layout.page_bytes, dtype=np.uint8)
    out[: raw.size] = raw
    return out


def pack(layout, weights):
    """Pool image: virtual page v of every tensor copied to physical page phi[v].

    ``weights[t]`` is the logical array of tensor t (or None to leave its
    pages zero).  Free pages are zero.
    """
    B = layout.page_bytes
    pool = np.zeros(layout.P * B, dtype=np.uint8)
    for t, w in enumerate(weights):
        if w is None:
            continue
        stream = tensor_stream(layout, t, w)
        for i in range(layout.npages[t]):
            p = layout.phi[layout.vbase[t] + i]
            pool[p * B:(p + 1) * B] = stream[i * B:(i + 1) * B]
    return pool


def unpack(layout, pool, t):
    """Read tensor t back from a pool image and undo the hidden shuffle."""
    s = layout.shapes[t]
    B = layout.page_bytes
    pages = [pool[layout.phi[layout.vbase[t] + i] * B:(layout.phi[layout.vbase[t] + i] + 1) * B]
             for i in range(layout.npages[t])]
    stream = np.concatenate(pages) if pages else np.zeros(0, np.uint8)
    raw = np.ascontiguousarray(stream[: s.nbytes])
    ws = raw.view(STORAGE_DTYPE[s.dtype]).reshape(s.n_out, s.k_in)
    return unshuffle_tensor(layout, t, ws)


def virtual_to_physical(layout, t, byte_offset):
    """Physical pool byte holding byte ``byte_offset`` of tensor t's stream."""
    B = layout.page_bytes
    v = layout.vbase[t] + byte_offset // B
    return layout.phi[v] * B + byte_offset % B


# ----------------------------------------------------------------------------
# Masked device page map.  The paper's page tables are the GPU's own; here the
# map is a table in device memory that every translating kernel reads, so a
# hardened layout stores it masked.  Reading: the k-th upload of the map uses
# key_k = the k-th nonzero word of the counter-mode SHA-256 stream (seed,
# tag 8, idx 0) and stores entry v as phi[v] XOR m(key_k, v); the key travels
# in the kernels' arguments only.  m: with k0 the low and k1 the high 32 bits
# of the key (k1 made odd), h = v XOR k0, h = (h XOR h>>16) * k1,
# h = (h XOR h>>15) * 0x2C1B3C6D, m = (h XOR h>>16) XOR k0, all mod 2**32.
# ----------------------------------------------------------------------------

TAG_MAP_KEY = 8


def map_keys(seed):
    """Keys of successive uploads of the device map (zero words skipped)."""
    g = prng.substream_csprng(seed, TAG_MAP_KEY, 0)
    while True:
        k = g.next_u64()
        if k:
            yield k


def map_mask(key, v):
    M = 0xFFFFFFFF
    k0, k1 = key & M, ((key >> 32) & M) | 1
    h = (v & M) ^ k0
    h = ((h ^ (h >> 16)) * k1) & M
    h = ((h ^ (h >> 15)) * 0x2C1B3C6D) & M
    return (h ^ (h >> 16)) ^ k0


def masked_map(phi, key):
    """Device table entries (as uint32) for page map phi under key."""
    return [(phi[v] ^ map_mask(key, v)) & 0xFFFFFFFF for v in range(len(phi))]


def contiguity(layout):
    """Share of in-tensor page successions that stay physically adjacent.

    The paper reports the percentage of virtual ranges backed by contiguous
    physical pages (Table 2).  Reading: over every pair of consecutive
    virtual pages inside one tensor, the fraction whose physical pages are
    also consecutive.  Returns a fraction in [0, 1] (1.0 if no pairs).
    """
    hits = total = 0
    for t in range(layout.T):
        for i in range(layout.npages[t] - 1):
            total += 1
            a = layout.phi[layout.vbase[t] + i]
            b = layout.phi[layout.vbase[t] + i + 1]
            hits += (b == a + 1)
    return 1.0 if total == 0 else hits / total

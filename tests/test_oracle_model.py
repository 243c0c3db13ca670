"""Pins of the FP64 reference decoder's composition (oracle/model.py).

The pieces (rmsnorm, rope, causal attention, SwiGLU) are pinned in
test_oracle_numerics.py; these tests pin how DecoderFP64.forward puts them
together -- the residual adds, which norm gain feeds which block, the final
norm before the head, the causal prefix and the GQA head grouping -- with
closed forms on weights chosen so the answer is known, a hand-derived 2-wide
case, and an independent token-by-token decoder with a KV cache written with
scalar loops.  A dropped residual, a norm in the wrong place, the head applied
before the final norm, a wrong kv-head mapping or a mask off by one fails at
least one of them.
"""

import math

import numpy as np
import pytest

from oracle import model as OM


def _cfg(D, H, Hkv, hd, F, vocab, layers, theta=10000.0, eps=1e-5):
    return dict(d_model=D, n_heads=H, n_kv_heads=Hkv, head_dim=hd, d_ffn=F, vocab=vocab, n_layers=layers,
                theta=theta, eps=eps)


def _random_model(cfg, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    D, H, Hkv, hd, F, V = (cfg[k] for k in ("d_model", "n_heads", "n_kv_heads", "head_dim", "d_ffn", "vocab"))
    w = {}
    for l in range(cfg["n_layers"]):
        w[(l, "q")] = rng.standard_normal((H * hd, D)) * 0.5
        w[(l, "k")] = rng.standard_normal((Hkv * hd, D)) * 0.5
        w[(l, "v")] = rng.standard_normal((Hkv * hd, D)) * 0.5
        w[(l, "o")] = rng.standard_normal((D, H * hd)) * 0.5
        w[(l, "gate")] = rng.standard_normal((F, D)) * 0.5
        w[(l, "up")] = rng.standard_normal((F, D)) * 0.5
        w[(l, "down")] = rng.standard_normal((D, F)) * 0.5
    w[(-1, "embed")] = rng.standard_normal((V, D))
    w[(-1, "head")] = rng.standard_normal((V, D))
    g = {}
    for l in range(cfg["n_layers"]):
        g[("attn", l)] = 0.5 + rng.random(D)
        g[("mlp", l)] = 0.5 + rng.random(D)
    g[("final", -1)] = 0.5 + rng.random(D)
    return w, g


def _norm_rows(x, gain, eps):
    """Row-wise x / sqrt(sum(x^2)/d + eps) * gain, one row at a time."""
    out = np.empty_like(x)
    for i in range(x.shape[0]):
        ms = sum(float(v) * float(v) for v in x[i]) / x.shape[1]
        out[i] = x[i] / math.sqrt(ms + eps) * gain
    return out


def test_zero_o_and_down_keep_the_embedding_in_the_residual():
    # With o and down zero, neither block adds anything: the residual stream
    # stays E[token] through every layer, and the logits are the final norm
    # (with its own gain, not a block's) of the embedding times the head.
    cfg = _cfg(16, 4, 2, 4, 12, 23, layers=2)
    w, g = _random_model(cfg, 11)
    for l in range(2):
        w[(l, "o")] = np.zeros_like(w[(l, "o")])
        w[(l, "down")] = np.zeros_like(w[(l, "down")])
    toks = [5, 0, 22, 5, 9]
    got = OM.DecoderFP64(cfg, w, g).forward(toks)
    e = w[(-1, "embed")][toks]
    want = _norm_rows(e, g[("final", -1)], cfg["eps"]) @ w[(-1, "head")].T
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)
    # the same model without the final norm gives something else
    assert np.max(np.abs(e @ w[(-1, "head")].T - want)) > 1e-2


def test_zero_queries_and_keys_average_the_values_of_the_prefix():
    # q = k = 0 makes every score 0, so query t weights keys 0..t equally:
    # attention is the running mean of the value vectors of its kv head.
    # With o the identity and down zero, one layer gives
    #   r_t = E_t + concat_h mean_{s<=t} v_{s, h // G},  v_s = norm_attn(E_s) Wv^T,
    # and the logits are norm_final(r_t) Wh^T.
    D, H, Hkv, hd = 16, 4, 2, 4
    G = H // Hkv
    cfg = _cfg(D, H, Hkv, hd, 8, 19, layers=1)
    w, g = _random_model(cfg, 12)
    w[(0, "q")] = np.zeros_like(w[(0, "q")])
    w[(0, "k")] = np.zeros_like(w[(0, "k")])
    w[(0, "o")] = np.eye(D)
    w[(0, "down")] = np.zeros_like(w[(0, "down")])
    toks = [3, 3, 18, 7, 1, 12]
    T = len(toks)
    e = w[(-1, "embed")][toks]
    hn = _norm_rows(e, g[("attn", 0)], cfg["eps"])
    vv = hn @ w[(0, "v")].T                         # [T][Hkv*hd]
    r = np.array(e, copy=True)
    for t in range(T):
        for h in range(H):
            c = h // G
            acc = np.zeros(hd)
            for s in range(t + 1):
                acc += vv[s, c * hd:(c + 1) * hd]
            r[t, h * hd:(h + 1) * hd] += acc / (t + 1)
    want = _norm_rows(r, g[("final", -1)], cfg["eps"]) @ w[(-1, "head")].T
    got = OM.DecoderFP64(cfg, w, g).forward(toks)
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-11)


def test_attention_off_leaves_the_mlp_block_on_the_residual():
    # o = 0: the attention block adds nothing, the MLP block sees
    # norm_mlp(E) (its own gain) and adds its output to E.  One hidden unit
    # written out with scalars: y = silu(h.wg) * (h.wu) * wd.
    D = 8
    cfg = _cfg(D, 2, 1, 4, 1, 13, layers=1)
    w, g = _random_model(cfg, 13)
    w[(0, "o")] = np.zeros_like(w[(0, "o")])
    toks = [2, 11, 4]
    e = w[(-1, "embed")][toks]
    hn = _norm_rows(e, g[("mlp", 0)], cfg["eps"])
    r = np.array(e, copy=True)
    wg, wu, wd = w[(0, "gate")][0], w[(0, "up")][0], w[(0, "down")][:, 0]
    for t in range(len(toks)):
        a = sum(hn[t, i] * wg[i] for i in range(D))
        b = sum(hn[t, i] * wu[i] for i in range(D))
        hid = a / (1.0 + math.exp(-a)) * b
        for j in range(D):
            r[t, j] += hid * wd[j]
    want = _norm_rows(r, g[("final", -1)], cfg["eps"]) @ w[(-1, "head")].T
    got = OM.DecoderFP64(cfg, w, g).forward(toks)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_two_wide_case_derived_by_hand():
    # d_model 2, one head of size 2, one hidden unit, eps 0, gains 1, one token:
    #   E = [1, -1]           norm(E) = [1, -1] (mean square 1)
    #   attention over the single key returns v = norm(E) Wv^T = [1, -1] (Wv = I)
    #   r = E + v Wo^T = [2, -2]                                   (Wo = I)
    #   norm(r) = [1, -1]; gate row [1, 0] -> 1, up row [0, -1] -> 1
    #   hidden = silu(1) * 1 = 1 / (1 + e^-1); down column [1, 0]
    #   r = [2 + 1/(1 + e^-1), -2]
    #   logits = norm(r) Wh^T with Wh = I, norm(r) = r / sqrt((r0^2 + r1^2) / 2)
    cfg = _cfg(2, 1, 1, 2, 1, 2, layers=1, eps=0.0)
    w = {(0, "q"): np.array([[0.3, -0.7], [1.1, 0.2]]), (0, "k"): np.array([[-0.4, 0.9], [0.5, 0.5]]),
         (0, "v"): np.eye(2), (0, "o"): np.eye(2),
         (0, "gate"): np.array([[1.0, 0.0]]), (0, "up"): np.array([[0.0, -1.0]]),
         (0, "down"): np.array([[1.0], [0.0]]),
         (-1, "embed"): np.array([[1.0, -1.0], [5.0, 5.0]]), (-1, "head"): np.eye(2)}
    got = OM.DecoderFP64(cfg, w).forward([0])
    r0, r1 = 2.0 + 1.0 / (1.0 + math.exp(-1.0)), -2.0
    s = math.sqrt((r0 * r0 + r1 * r1) / 2.0)
    np.testing.assert_allclose(got[0], [r0 / s, r1 / s], rtol=1e-15)


# ---------------------------------------------------------------- an independent incremental decoder

def _incremental_logits(cfg, w, g, toks):
    """Token-by-token decoding with a KV cache, scalar loops throughout;
    shares nothing with oracle/model.py."""
    D, H, Hkv, hd, L = (cfg[k] for k in ("d_model", "n_heads", "n_kv_heads", "head_dim", "n_layers"))
    G, half, eps, theta = H // Hkv, hd // 2, cfg["eps"], cfg["theta"]

    def norm(vec, gain):
        ms = sum(x * x for x in vec) / len(vec)
        sc = 1.0 / math.sqrt(ms + eps)
        return [vec[i] * sc * float(np.broadcast_to(gain, (len(vec),))[i]) for i in range(len(vec))]

    def matvec(W, vec):
        return [sum(W[n, k] * vec[k] for k in range(len(vec))) for n in range(W.shape[0])]

    def rotate(vec, pos):
        out = list(vec)
        for i in range(half):
            ang = pos * theta ** (-2.0 * i / hd)
            c, s = math.cos(ang), math.sin(ang)
            out[i] = vec[i] * c - vec[i + half] * s
            out[i + half] = vec[i + half] * c + vec[i] * s
        return out

    cache = [([], []) for _ in range(L)]   # per layer: keys, values (lists of per-kv-head vectors)
    logits = []
    for pos, tok in enumerate(toks):
        r = [float(x) for x in w[(-1, "embed")][tok]]
        for l in range(L):
            hn = norm(r, g[("attn", l)])
            q, k, v = matvec(w[(l, "q")], hn), matvec(w[(l, "k")], hn), matvec(w[(l, "v")], hn)
            qh = [rotate(q[h * hd:(h + 1) * hd], pos) for h in range(H)]
            kh = [rotate(k[c * hd:(c + 1) * hd], pos) for c in range(Hkv)]
            vh = [v[c * hd:(c + 1) * hd] for c in range(Hkv)]
            cache[l][0].append(kh)
            cache[l][1].append(vh)
            att = []
            for h in range(H):
                c = h // G
                sc = [sum(qh[h][i] * kk[c][i] for i in range(hd)) / math.sqrt(hd) for kk in cache[l][0]]
                m = max(sc)
                p = [math.exp(x - m) for x in sc]
                z = sum(p)
                att += [sum(p[j] * cache[l][1][j][c][i] for j in range(len(p))) / z for i in range(hd)]
            r = [a + b for a, b in zip(r, matvec(w[(l, "o")], att))]
            hn = norm(r, g[("mlp", l)])
            gt, up = matvec(w[(l, "gate")], hn), matvec(w[(l, "up")], hn)
            hid = [a / (1.0 + math.exp(-a)) * b for a, b in zip(gt, up)]
            r = [a + b for a, b in zip(r, matvec(w[(l, "down")], hid))]
        logits.append(matvec(w[(-1, "head")], norm(r, g[("final", -1)])))
    return np.array(logits)


@pytest.mark.parametrize("geom", [(16, 4, 2, 4, 2), (24, 6, 3, 4, 1), (16, 2, 2, 8, 2)])
def test_full_forward_equals_an_incremental_decoder_with_kv_cache(geom):
    D, H, Hkv, hd, layers = geom
    cfg = _cfg(D, H, Hkv, hd, 10, 17, layers, theta=500000.0 if layers == 1 else 10000.0)
    w, g = _random_model(cfg, sum(geom))
    toks = [4, 16, 4, 0, 9, 13, 2]
    got = OM.DecoderFP64(cfg, w, g).forward(toks)
    want = _incremental_logits(cfg, w, g, toks)
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-10)


def test_planted_composition_mistakes_are_visible():
    # The checks above are sensitive: each plausible slip in the composition
    # moves the logits far beyond their tolerance.  The slips are planted in a
    # copy of the decoder here, on the CPU.
    cfg = _cfg(16, 4, 2, 4, 10, 17, 2)
    w, g = _random_model(cfg, 77)
    toks = [4, 16, 4, 0, 9]
    ref = _incremental_logits(cfg, w, g, toks)

    class NoFinalNorm(OM.DecoderFP64):
        def forward(self, tokens):
            saved = OM.rmsnorm
            calls = {"n": 0}

            def counting(v, gain, eps):
                calls["n"] += 1
                if calls["n"] == 2 * self.cfg["n_layers"] + 1:   # the final norm
                    return np.asarray(v, np.float64)
                return saved(v, gain, eps)
            OM.rmsnorm = counting
            try:
                return super().forward(tokens)
            finally:
                OM.rmsnorm = saved

    swapped = dict(g)
    swapped[("attn", 0)], swapped[("mlp", 0)] = g[("mlp", 0)], g[("attn", 0)]
    for bad in (NoFinalNorm(cfg, w, g).forward(toks), OM.DecoderFP64(cfg, w, swapped).forward(toks)):
        assert np.max(np.abs(bad - ref)) > 1e-3 * np.max(np.abs(ref))

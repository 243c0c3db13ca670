"""FP64 reference decoder for the serving loop (oracle).

The paper serves Llama / Qwen decoders under vLLM (Section 5 setup) and
requires that cloaking leaves results unchanged (Section 4.1, paragraph on
virtual-physical address decoupling).  This module is the plain
definition of the decoder the serving loop runs, in FP64 on logical weights:

    r_0      = E[token]
    per layer l:
      h      = rmsnorm(r) * g_attn_l          rmsnorm(v) = v / sqrt(mean(v^2) + eps)
      q,k,v  = h Wq^T, h Wk^T, h Wv^T         GQA: H query heads, Hkv key/value heads
      q,k    = rope(q, pos), rope(k, pos)     rotate-half convention, theta
      a      = softmax(q k^T / sqrt(d) + causal mask) v   per query head, sharing
                                                          kv head  h // (H / Hkv)
      r      = r + a Wo^T
      h      = rmsnorm(r) * g_mlp_l
      r      = r + SwiGLU FFN(h)
    logits   = rmsnorm(r) * g_final  Wh^T

Readings (the paper fixes none of them; they shape cost, not the defence):
Llama-3.1-8B-like geometry, RoPE theta 500000 without scaling, eps 1e-5,
norm gains all ones unless given, greedy argmax.  Pure NumPy, no batching
tricks: each sequence is evaluated on its own, token by token positions.
"""

import numpy as np

from . import numerics as N


def rmsnorm(v, gain, eps):
    v = np.asarray(v, np.float64)
    return v / np.sqrt(np.mean(v * v, axis=-1, keepdims=True) + eps) * gain


def rope(x, pos, theta):
    """x [..., T, d] rotated by angle pos * theta^(-2i/d) on pairs (i, i + d/2)."""
    d = x.shape[-1]
    half = d // 2
    inv = theta ** (-np.arange(half, dtype=np.float64) * 2.0 / d)
    ang = np.asarray(pos, np.float64)[:, None] * inv[None, :]
    c, s = np.cos(ang), np.sin(ang)
    x1, x2 = x[..., :half], x[..., half:]
    return np.concatenate([x1 * c - x2 * s, x2 * c + x1 * s], axis=-1)


def causal_attention(q, k, v):
    """q [H, T, d], k/v [Hkv, T, d] -> [T, H*d]; query t sees keys 0..t."""
    H, T, d = q.shape
    Hkv = k.shape[0]
    group = H // Hkv
    out = np.empty((T, H * d))
    mask = np.triu(np.ones((T, T), bool), 1)
    for h in range(H):
        kh, vh = k[h // group], v[h // group]
        s = q[h] @ kh.T / np.sqrt(d)
        s[mask] = -np.inf
        s = s - s.max(axis=1, keepdims=True)
        p = np.exp(s)
        p /= p.sum(axis=1, keepdims=True)
        out[:, h * d:(h + 1) * d] = p @ vh
    return out


class DecoderFP64:
    """Logical FP64 weights of a decoder; `forward(tokens)` gives all logits."""

    def __init__(self, cfg, weights, gains=None):
        # cfg: d_model, n_heads, n_kv_heads, head_dim, d_ffn, vocab, n_layers, theta, eps
        # weights: dict (layer, kind) -> FP64 [N][K] logical array; embed/head at layer -1
        self.cfg = cfg
        self.w = weights
        L = cfg["n_layers"]
        self.g = gains if gains is not None else {
            ("attn", l): 1.0 for l in range(L)} | {("mlp", l): 1.0 for l in range(L)} | {("final", -1): 1.0}

    def forward(self, tokens):
        c = self.cfg
        T = len(tokens)
        H, Hkv, d = c["n_heads"], c["n_kv_heads"], c["head_dim"]
        pos = np.arange(T)
        r = self.w[(-1, "embed")][np.asarray(tokens)]
        for l in range(c["n_layers"]):
            h = rmsnorm(r, self.g[("attn", l)], c["eps"])
            q = N.linear(h, self.w[(l, "q")]).reshape(T, H, d).transpose(1, 0, 2)
            k = N.linear(h, self.w[(l, "k")]).reshape(T, Hkv, d).transpose(1, 0, 2)
            v = N.linear(h, self.w[(l, "v")]).reshape(T, Hkv, d).transpose(1, 0, 2)
            q, k = rope(q, pos, c["theta"]), rope(k, pos, c["theta"])
            a = causal_attention(q, k, v)
            r = r + N.linear(a, self.w[(l, "o")])
            h = rmsnorm(r, self.g[("mlp", l)], c["eps"])
            y, _ = N.swiglu_ffn(h, self.w[(l, "gate")], self.w[(l, "up")], self.w[(l, "down")])
            r = r + y
        h = rmsnorm(r, self.g[("final", -1)], c["eps"])
        return N.linear(h, self.w[(-1, "head")])

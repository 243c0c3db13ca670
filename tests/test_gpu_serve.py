"""Serving loop on the GPU: decoder step vs the FP64 oracle decoder, each
request's result alone vs in a continuous-batching mix, remap mid-run, and
admission under KV-block pressure.

Tolerance: logits per generated position, normwise max|y - y*| / max|y*|.
The decoder runs every activation in bf16 between kernels (norms, q/k/v,
attention, projections, residual stream), so against FP64 the bound is the
per-op bf16 budget summed over the ops of two layers: 3e-2.  Alone vs mix
compares two GPU runs whose only differences are kernel choices (GEMV vs
MFMA GEMM by batch size, context slicing): 1e-2.
"""

import numpy as np
import pytest

from oracle import model as OM
from oracle import numerics as ON
from paper_2606_18400_amd import synth

pytestmark = pytest.mark.gpu

TINY = dict(n_layers=2, d_model=256, n_heads=2, n_kv_heads=1, head_dim=128, d_ffn=512, vocab=1024,
            theta=500000.0, eps=1e-5)
# two kv heads, so the kv-group permutation is not trivial
GQA = dict(n_layers=2, d_model=512, n_heads=4, n_kv_heads=2, head_dim=128, d_ffn=512, vocab=1024,
           theta=500000.0, eps=1e-5)


@pytest.fixture(scope="module")
def S():
    import torch
    assert torch.cuda.is_available()
    from paper_2606_18400_amd import serve
    return serve


def tiny_weights(cfg, base_seed=1234):
    shapes = __import__("paper_2606_18400_amd.serve", fromlist=["x"]).model_shapes(cfg)
    ws = [synth.weight(t, s[2], s[3], "bf16", base_seed=base_seed)[0] for t, s in enumerate(shapes)]
    return shapes, ws


def oracle_decoder(cfg, shapes, ws):
    w = {(s[0], s[1]): ON.bf16_bits_to_f64(ws[t]) for t, s in enumerate(shapes)}
    return OM.DecoderFP64(cfg, w)


def make_engine(S, cfg, ws, **kw):
    args = dict(pool_bytes=64 << 20, page_bytes=64 << 10, seed=5, kv_blocks=256, block_size=16, max_tokens=256,
                prefill_chunk=16, max_seqs=16, split_keys=64, remap_every=0, weights=ws, record_logits=True)
    args.update(kw)
    return S.Engine(cfg, **args)


HARDENED = dict(flags=8 | 4, decoy=True, remap_every=2, remap_slices=2)   # masked map, SHA-256 draws


@pytest.mark.parametrize("cfg,head_perm,extra", [(TINY, True, {}), (TINY, False, {}), (GQA, True, {}),
                                                 (GQA, True, HARDENED)],
                         ids=["tiny-heads", "tiny-noheads", "gqa-heads", "gqa-hardened"])
def test_tiny_decoder_matches_fp64_oracle(S, cfg, head_perm, extra):
    # with head_perm the attention runs on permuted heads in stored order; the
    # hardened engine adds a masked device map re-keyed by every remap slice,
    # SHA-256 layout draws and decoy free pages
    shapes, ws = tiny_weights(cfg)
    rng = np.random.Generator(np.random.PCG64(11))
    prompt = rng.integers(0, cfg["vocab"], 40).astype(np.int32)
    forced = rng.integers(0, cfg["vocab"], 8).astype(np.int32)
    eng = make_engine(S, cfg, ws, head_perm=head_perm, **extra)
    r = S.Request(0, prompt, len(forced), forced=forced)
    eng.run([r], realtime=False)
    ref = oracle_decoder(cfg, shapes, ws).forward(np.concatenate([prompt, forced[:-1]]))
    worst = 0.0
    for i, lg in enumerate(r.logits):
        err = ON.normwise_err(lg, ref[len(prompt) - 1 + i])
        worst = max(worst, err)
        assert err <= 3e-2, (i, err)
    print(f"tiny decoder worst normwise logit error vs FP64: {worst:.3e}")
    if extra:
        assert eng.remaps >= 2
    eng.close()


def test_each_result_same_alone_and_in_the_mix(S):
    shapes, ws = tiny_weights(TINY)
    rng = np.random.Generator(np.random.PCG64(12))
    probe_prompt = rng.integers(0, TINY["vocab"], 37).astype(np.int32)
    # alone: greedy
    eng = make_engine(S, TINY, ws)
    alone = S.Request(0, probe_prompt, 12)
    eng.run([alone], realtime=False)
    eng.close()
    # in the mix: six other requests of uneven lengths arrive together; the
    # probe is teacher-forced to its own greedy tokens
    eng = make_engine(S, TINY, ws)
    others = [S.Request(1 + i, rng.integers(0, TINY["vocab"], n).astype(np.int32), m)
              for i, (n, m) in enumerate([(5, 20), (70, 6), (33, 15), (1, 9), (120, 4), (18, 30)])]
    probe = S.Request(0, probe_prompt, 12, forced=alone.out)
    eng.run(others[:3] + [probe] + others[3:], realtime=False)
    assert eng.steps > 0 and all(o.done for o in others)
    for i, (a, b) in enumerate(zip(alone.logits, probe.logits)):
        err = ON.normwise_err(b, a)
        assert err <= 1e-2, (i, err)
        # greedy tokens agree unless the alone run had a near tie
        top2 = np.sort(a)[-2:]
        if top2[1] - top2[0] > 1e-2 * np.max(np.abs(a)):
            assert int(np.argmax(b)) == alone.out[i]
    eng.close()


def test_remap_between_steps_changes_nothing(S):
    shapes, ws = tiny_weights(TINY)
    rng = np.random.Generator(np.random.PCG64(13))
    prompts = [rng.integers(0, TINY["vocab"], n).astype(np.int32) for n in (20, 45, 3)]
    outs = []
    # no remap; a whole remap after every step; remaps spread over 3 steps each
    for every, slices in ((0, 1), (1, 1), (2, 3)):
        eng = make_engine(S, TINY, ws, remap_every=every, remap_slices=slices)
        reqs = [S.Request(i, p, 10) for i, p in enumerate(prompts)]
        eng.run(reqs, realtime=False)
        if every == 1:
            assert eng.remaps == eng.steps > 0
        if slices > 1:
            assert eng.remaps >= 2
        outs.append([(r.out, [l.copy() for l in r.logits]) for r in reqs])
        eng.close()
    for other in outs[1:]:
        for (oa, la), (ob, lb) in zip(outs[0], other):
            assert oa == ob
            for x, y in zip(la, lb):
                assert np.array_equal(x, y)


def test_admission_never_overcommits_kv(S):
    shapes, ws = tiny_weights(TINY)
    rng = np.random.Generator(np.random.PCG64(14))
    eng = make_engine(S, TINY, ws, kv_blocks=12, record_logits=False)
    reqs = [S.Request(i, rng.integers(0, TINY["vocab"], n).astype(np.int32), m)
            for i, (n, m) in enumerate([(60, 30), (40, 20), (90, 5), (10, 60), (30, 30)])]
    for r in reqs:
        eng.submit(r)
    peak = 0
    while eng.waiting or eng.running:
        eng._admit(float("inf"))
        used = sum(len(r.blocks) for r in eng.running)
        assert used + len(eng.free_blocks) == 12
        peak = max(peak, used)
        eng.step()
    assert all(r.done and len(r.out) == r.max_new for r in reqs)
    assert peak <= 12
    eng.close()


# the serving geometry's attention: 32 query heads over 8 kv heads of 128
# (d_model 4096), with a small FFN and vocabulary so the FP64 reference stays
# quick; one layer, so attention's output dominates the residual stream
ATTN32 = dict(n_layers=1, d_model=4096, n_heads=32, n_kv_heads=8, head_dim=128, d_ffn=512, vocab=1024,
              theta=500000.0, eps=1e-5)


def test_attention_32_8_heads_long_context_matches_fp64_oracle(S):
    """A 4,200-token prompt prefilled in 512-token chunks (tiles of 16 new
    tokens against up to 4,200 keys, contexts cut into 512-key slices), then
    decode steps whose single query reads the whole context: the logits of the
    last prompt position and of each decoded position against the FP64
    decoder (stored-order permuted heads, 2 MiB pages)."""
    shapes, ws = tiny_weights(ATTN32)
    rng = np.random.Generator(np.random.PCG64(15))
    prompt = rng.integers(0, ATTN32["vocab"], 4200).astype(np.int32)
    forced = rng.integers(0, ATTN32["vocab"], 3).astype(np.int32)
    eng = make_engine(S, ATTN32, ws, pool_bytes=256 << 20, page_bytes=2 << 20, kv_blocks=300, max_tokens=512,
                      prefill_chunk=512, max_seqs=4, split_keys=512)
    r = S.Request(0, prompt, len(forced), forced=forced)
    eng.run([r], realtime=False)
    ref = oracle_decoder(ATTN32, shapes, ws).forward(np.concatenate([prompt, forced[:-1]]))
    assert len(r.logits) == len(forced)
    worst = 0.0
    for i, lg in enumerate(r.logits):
        err = ON.normwise_err(lg, ref[len(prompt) - 1 + i])
        worst = max(worst, err)
        assert err <= 3e-2, (i, err)
    print(f"32/8-head attention over 4200+ keys: worst normwise logit error vs FP64 {worst:.3e}")
    eng.close()


# head groups of 1, 3 and 8 query heads per kv head; group 3 has no
# single-token kernel, so every tile runs on the matrix-core path
GROUPS = {1: (2, 2), 3: (3, 1), 8: (8, 1)}


@pytest.mark.parametrize("single", ["decode", "all", "none"])
@pytest.mark.parametrize("group", [1, 3, 8])
def test_head_groups_and_attention_paths_match_fp64_oracle(S, group, single):
    """Three requests of uneven prompts decode while others prefill (mixed
    steps of single-token and 16-token tiles), contexts cut into 512-key
    slices so each wave of the single-token path walks several 16-key runs
    with ragged ends.  single='all' also sends 16-token prefill tiles down the
    single-token path, 'none' sends decode tokens down the matrix-core path:
    both must match the FP64 decoder as the default routing does."""
    n_heads, n_kv = GROUPS[group]
    cfg = dict(n_layers=1, d_model=128 * n_heads, n_heads=n_heads, n_kv_heads=n_kv, head_dim=128, d_ffn=512,
               vocab=1024, theta=500000.0, eps=1e-5)
    shapes, ws = tiny_weights(cfg)
    rng = np.random.Generator(np.random.PCG64(16 + group))
    lens, outs = [37, 301, 150], [9, 4, 6]
    reqs = [S.Request(i, rng.integers(0, cfg["vocab"], n).astype(np.int32), m,
                      forced=rng.integers(0, cfg["vocab"], m).astype(np.int32))
            for i, (n, m) in enumerate(zip(lens, outs))]
    eng = make_engine(S, cfg, ws, prefill_chunk=64, max_tokens=128, split_keys=512, single_tiles=single)
    eng.run(reqs, realtime=False)
    dec = oracle_decoder(cfg, shapes, ws)
    worst = 0.0
    for r in reqs:
        assert r.done and len(r.logits) == len(r.forced)
        ref = dec.forward(np.concatenate([r.prompt, r.forced[:-1]]))
        for i, lg in enumerate(r.logits):
            err = ON.normwise_err(lg, ref[len(r.prompt) - 1 + i])
            worst = max(worst, err)
            assert err <= 3e-2, (r.id, i, err)
    print(f"group {group}, single={single}: worst normwise logit error vs FP64 {worst:.3e}")
    eng.close()

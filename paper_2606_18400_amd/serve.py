"""Continuous-batching serving loop over cloaked weights.

The paper's serving engine (vLLM, Section 4.1) orchestrates weight loading,
KV-cache blocks and batching; CloakLM changes only where the weights live
(Section 4.2) and re-randomises their placement every so many iterations
(Section 4.2, Section 5.2, Figure 7).  This module is that engine's policy
for one GPU:

* requests arrive on a trace; a request is admitted when the free KV blocks
  cover its prompt plus its output budget (so nothing is ever preempted);
* every step runs one mixed batch: one decode token for each running
  sequence plus prefill chunks of admitted prompts up to a token budget, so
  new requests overlap with running ones on the device;
* a step is ONE native call (cloak_model_step) covering every layer; the
  host only builds the small index arrays and reads back the sampled ids;
* cloak_remap runs between steps every `remap_every` steps, or, with
  `remap_slices` > 1, one remap is spread over that many consecutive steps
  (cloak_remap_begin / cloak_remap_step), so no step pays the whole move;
* TTFT and per-token latencies are recorded for p50/p99 reporting.

PyTorch only allocates device buffers (pool, KV cache, workspace) and
provides the stream.
"""

import math
import os
import time

import numpy as np

from . import cloak as C
from . import synth

# Llama-3.1-8B-like geometry with random weights (the paper's models are not
# available here); 32 layers of the 4096/14336 layer, vocab 128256.
LLAMA8B = dict(n_layers=32, d_model=4096, n_heads=32, n_kv_heads=8, head_dim=128, d_ffn=14336, vocab=128256,
               theta=500000.0, eps=1e-5)


def model_shapes(cfg, head_perm=True):
    """Every tensor of the decoder; with head_perm the attention heads are permuted too."""
    shapes = []
    kvd = cfg["n_kv_heads"] * cfg["head_dim"]
    hd = cfg["head_dim"] if head_perm else 0
    for l in range(cfg["n_layers"]):
        shapes += synth.decoder_layer_shapes(cfg["d_model"], cfg["d_ffn"], kvd, "bf16", layer=l, head_dim=hd)
    shapes += [(-1, "embed", cfg["vocab"], cfg["d_model"], "bf16"), (-1, "head", cfg["vocab"], cfg["d_model"], "bf16")]
    return shapes


class Request:
    def __init__(self, rid, prompt, max_new, arrival=0.0, forced=None):
        self.id = rid
        self.prompt = np.asarray(prompt, np.int32)
        self.max_new = int(max_new)
        self.arrival = float(arrival)
        self.forced = None if forced is None else list(forced)
        self.blocks = []
        self.n_cached = 0          # tokens whose K/V are in the cache
        self.out = []              # generated tokens
        self.logits = []           # recorded logits per generated token (tests)
        self.t_first = None
        self.t_tokens = []
        self.done = False

    @property
    def prefilled(self):
        return self.n_cached >= len(self.prompt)


class Engine:
    """One GPU: cloaked weights, paged KV cache, continuous batching."""

    def __init__(self, cfg, pool_bytes, page_bytes=2 << 20, seed=None, flags=0, kv_blocks=4096, block_size=16,
                 max_tokens=2048, prefill_chunk=512, max_seqs=64, split_keys=512, remap_every=256,
                 weights=None, gains=None, record_logits=False, max_context=None, remap_slices=1,
                 head_perm=True, decoy=None, single_tiles="decode"):
        import torch
        self.torch = torch
        self.cfg = dict(cfg)
        self.shapes = model_shapes(cfg, head_perm)
        self.bs = block_size
        self.kv_blocks = kv_blocks
        self.max_tokens = max_tokens
        self.prefill_chunk = prefill_chunk
        self.max_seqs = max_seqs
        self.split_keys = split_keys
        # tiles declared single-token: "decode" (the leading decode tokens),
        # "all" or "none" (the last two exercise the attention paths)
        if single_tiles not in ("decode", "all", "none"):
            raise ValueError(f"single_tiles must be decode, all or none, not {single_tiles!r}")
        self.single_tiles = single_tiles
        self.remap_every = remap_every
        # a remap is spread over remap_slices consecutive steps (1 = all at once)
        self.remap_slices = max(1, int(remap_slices))
        self._remap_chunk = 0
        self.record_logits = record_logits
        self.max_context = max_context or kv_blocks * block_size
        self.cw = C.CloakedWeights(self.shapes, page_bytes, pool_bytes, seed=seed, flags=flags, decoy=decoy)
        if weights is None:
            weights = [synth.weight(t, s[2], s[3], "bf16")[0] for t, s in enumerate(self.shapes)]
        self.cw.load(weights)
        hd, nkv, L = cfg["head_dim"], cfg["n_kv_heads"], cfg["n_layers"]
        self.kv = torch.zeros(L * 2 * kv_blocks * nkv * block_size * hd, dtype=torch.bfloat16, device="cuda")
        self.gains = None
        if gains is not None:
            self.gains = torch.from_numpy(np.ascontiguousarray(gains).view(np.int16)).cuda().view(torch.bfloat16)
        mc = C.cloak_model_config(L, cfg["d_model"], cfg["n_heads"], nkv, hd, cfg["d_ffn"], cfg["vocab"], block_size,
                                  kv_blocks, cfg["theta"], cfg["eps"])
        self.model = C.cloak_model_create(self.cw.layout, self.cw.pool, mc, self.gains, self.kv)
        self.max_tiles = max_tokens // 16 + max_seqs + 1
        self.max_splits = max(1, math.ceil(self.max_context / split_keys))
        self.ws_bytes = C.cloak_model_ws_bytes(self.model, max_tokens, max_seqs, self.max_tiles, self.max_splits)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.max_blocks_per_seq = math.ceil(self.max_context / block_size)
        n_idx = 4 * max_tokens + max_seqs * self.max_blocks_per_seq + 3 * self.max_tiles + max_seqs
        self.h_idx = torch.empty(n_idx, dtype=torch.int32, pin_memory=True)
        self.d_idx = torch.empty(n_idx, dtype=torch.int32, device="cuda")
        self.d_out = torch.empty(max_seqs, dtype=torch.int32, device="cuda")
        self.h_out = torch.empty(max_seqs, dtype=torch.int32, pin_memory=True)
        self.d_logits = (torch.empty((max_seqs, cfg["vocab"]), dtype=torch.bfloat16, device="cuda")
                         if record_logits else None)
        self.free_blocks = list(range(kv_blocks))[::-1]
        self.waiting, self.running, self.finished = [], [], []
        self.steps = 0
        self.remaps = 0
        self.step_ms = []
        self.remap_events = []

    # ------------------------------------------------------------- admission
    def blocks_needed(self, r):
        return math.ceil((len(r.prompt) + r.max_new) / self.bs)

    def submit(self, r):
        if len(r.prompt) + r.max_new > self.max_context:
            raise ValueError(f"request {r.id} exceeds the context limit {self.max_context}")
        if r.max_new < 1 or len(r.prompt) < 1:
            raise ValueError(f"request {r.id} needs a prompt and at least one output token")
        self.waiting.append(r)

    def _admit(self, now):
        while self.waiting and len(self.running) < self.max_seqs and self.waiting[0].arrival <= now:
            r = self.waiting[0]
            need = self.blocks_needed(r)
            if need > len(self.free_blocks):
                break          # head-of-line waits for blocks; nothing is preempted
            self.waiting.pop(0)
            r.blocks = [self.free_blocks.pop() for _ in range(need)]
            self.running.append(r)

    # ------------------------------------------------------------- one step
    ATTN_BLOCKS = 1024    # about 4 attention blocks per compute unit
    MIN_SLICE = 128       # keys per slice at least: 2 runs of 16 keys per wave

    def key_slices(self, n_tiles, max_ctx):
        """Keys per attention slice for this step: at most split_keys, a
        multiple of 64, short enough that tiles x kv heads x slices fills the
        GPU, and no more partials than the workspace holds."""
        want = max(1, math.ceil(self.ATTN_BLOCKS / (n_tiles * self.cfg["n_kv_heads"])))
        keys = min(self.split_keys, max(self.MIN_SLICE, math.ceil(max_ctx / want / 64) * 64))
        while n_tiles * math.ceil(max_ctx / keys) > self.max_tiles * self.max_splits:
            keys += 64
        return keys, max(1, math.ceil(max_ctx / keys))

    def _plan(self):
        """Decode tokens of running sequences first, then prefill chunks."""
        batch = []    # (request, first position, n tokens, token ids)
        budget = self.max_tokens
        for r in self.running:
            if r.prefilled and budget > 0:
                tok = r.out[-1] if r.out else int(r.prompt[-1])
                batch.append((r, r.n_cached, 1, np.array([tok], np.int32)))
                budget -= 1
        for r in self.running:
            if not r.prefilled and budget > 0:
                n = min(self.prefill_chunk, len(r.prompt) - r.n_cached, budget)
                batch.append((r, r.n_cached, n, r.prompt[r.n_cached:r.n_cached + n]))
                budget -= n
        return batch

    def step(self):
        batch = self._plan()
        if not batch:
            return 0
        torch = self.torch
        T = sum(b[2] for b in batch)
        S = len(batch)
        maxb = max(len(b[0].blocks) for b in batch)
        tokens = np.concatenate([b[3] for b in batch]).astype(np.int32)
        positions = np.concatenate([np.arange(b[1], b[1] + b[2], dtype=np.int32) for b in batch])
        tok_seq = np.concatenate([np.full(b[2], i, np.int32) for i, b in enumerate(batch)])
        table = np.zeros((S, maxb), np.int32)
        for i, b in enumerate(batch):
            table[i, :len(b[0].blocks)] = b[0].blocks
        tile_seq, tile_tok0, tile_ntok = [], [], []
        row = 0
        logit_rows, logit_reqs = [], []
        max_ctx = 0
        for i, (r, p0, n, _) in enumerate(batch):
            for j in range(0, n, 16):
                tile_seq.append(i)
                tile_tok0.append(row + j)
                tile_ntok.append(min(16, n - j))
            if p0 + n >= len(r.prompt):         # this step produces the next token
                logit_rows.append(row + n - 1)
                logit_reqs.append(r)
            max_ctx = max(max_ctx, p0 + n)
            row += n
        split_keys, n_splits = self.key_slices(len(tile_seq), max_ctx)
        # decode tokens come first, one tile each: the single-token attention path
        n_single = next((k for k, n in enumerate(tile_ntok) if n != 1), len(tile_ntok))
        n_single = {"decode": n_single, "all": len(tile_ntok), "none": 0}[self.single_tiles]
        parts = [tokens, positions, tok_seq, table.reshape(-1), np.array(tile_seq, np.int32),
                 np.array(tile_tok0, np.int32), np.array(tile_ntok, np.int32), np.array(logit_rows, np.int32)]
        offs, cur = [], 0
        for p in parts:
            offs.append(cur)
            cur += len(p)
        flat = np.concatenate(parts)
        self.h_idx[:cur].copy_(torch.from_numpy(flat))
        self.d_idx[:cur].copy_(self.h_idx[:cur], non_blocking=True)
        base = self.d_idx.data_ptr()
        ptr = [base + 4 * o for o in offs]
        st = C.cloak_step(T, S, maxb, len(logit_rows), len(tile_seq), n_splits, split_keys, n_single,
                          ptr[0], ptr[1], ptr[2], ptr[3], ptr[4], ptr[5], ptr[6], ptr[7] if logit_rows else None,
                          self.d_out.data_ptr() if logit_rows else None,
                          self.d_logits.data_ptr() if (self.record_logits and logit_rows) else None)
        t0 = time.perf_counter()
        C.cloak_model_step(self.model, st, self.ws, self.ws_bytes)
        R = len(logit_rows)
        if R:
            self.h_out[:R].copy_(self.d_out[:R], non_blocking=True)
        logits = self.d_logits[:R].float().cpu().numpy() if (self.record_logits and R) else None
        torch.cuda.current_stream().synchronize()
        now = time.perf_counter()
        self.step_ms.append((now - t0) * 1e3)
        out = self.h_out[:R].numpy().copy() if R else []
        for (r, p0, n, _) in batch:
            r.n_cached = p0 + n
        for k, r in enumerate(logit_reqs):
            tok = int(out[k])
            if r.forced is not None and len(r.out) < len(r.forced):
                tok = r.forced[len(r.out)]
            r.out.append(tok)
            if logits is not None:
                r.logits.append(logits[k])
            if r.t_first is None:
                r.t_first = now
            r.t_tokens.append(now)
            if len(r.out) >= r.max_new:
                r.done = True
        for r in [r for r in self.running if r.done]:
            self.running.remove(r)
            self.free_blocks.extend(r.blocks[::-1])
            r.blocks = []
            self.finished.append(r)
        self.steps += 1
        pending = C.cloak_query(self.cw.layout, "REMAP_PENDING") if self.remap_slices > 1 else 0
        due = not pending and self.remap_every and self.steps % self.remap_every == 0
        if pending or due:
            # the move is timed on the stream (events), not on the host
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            if pending:
                self.cw.remap_step(self._remap_chunk)
            else:
                seed = int.from_bytes(os.urandom(8), "little")
                if self.remap_slices == 1:
                    self.cw.remap(seed)
                else:
                    self.cw.remap_begin(seed)
                    total = C.cloak_query(self.cw.layout, "REMAP_PENDING")
                    self._remap_chunk = max(1, math.ceil(total / self.remap_slices))
                    self.cw.remap_step(self._remap_chunk)
                self.remaps += 1
            ev1.record()
            self.remap_events.append((ev0, ev1))
        return T

    def remap_ms(self, since=0):
        """Device time of each remap (slice) enqueued since event index `since`."""
        self.torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in self.remap_events[since:]]

    # ------------------------------------------------------------- driver
    def run(self, requests, realtime=True, time_limit=None, progress=None, progress_every=30.0):
        """Serve a trace; arrival times are seconds from the start.  progress,
        if given, is called as progress(finished, total, seconds) at most every
        progress_every seconds."""
        for r in sorted(requests, key=lambda r: r.arrival):
            self.submit(r)
        t_start = time.perf_counter()
        t_told = t_start
        n0 = len(self.finished)
        for r in requests:
            r.arrival_wall = t_start + r.arrival if realtime else t_start
        while self.waiting or self.running:
            now = time.perf_counter() - t_start
            if not realtime:
                now = float("inf")
            self._admit(now)
            if not self.running:
                nxt = self.waiting[0].arrival
                time.sleep(max(0.0, min(nxt - (time.perf_counter() - t_start), 0.05)))
                continue
            self.step()
            t_now = time.perf_counter()
            if progress and t_now - t_told >= progress_every:
                progress(len(self.finished) - n0, len(requests), t_now - t_start)
                t_told = t_now
            if time_limit and t_now - t_start > time_limit:
                break
        return self.report(requests, time.perf_counter() - t_start)

    @staticmethod
    def report(requests, wall):
        done = [r for r in requests if r.done and r.t_first is not None]
        ttft = np.array([(r.t_first - r.arrival_wall) * 1e3 for r in done]) if done else np.zeros(0)
        gaps = np.concatenate([np.diff(r.t_tokens) * 1e3 for r in done if len(r.t_tokens) > 1]) \
            if any(len(r.t_tokens) > 1 for r in done) else np.zeros(0)
        tpot = np.array([(r.t_tokens[-1] - r.t_first) * 1e3 / (len(r.t_tokens) - 1)
                         for r in done if len(r.t_tokens) > 1])
        pct = lambda a, q: float(np.percentile(a, q)) if len(a) else None
        toks = sum(len(r.out) for r in done)
        return dict(requests=len(requests), completed=len(done), wall_s=wall, output_tokens=toks,
                    output_tok_per_s=toks / wall if wall > 0 else None,
                    ttft_ms_p50=pct(ttft, 50), ttft_ms_p99=pct(ttft, 99),
                    tpot_ms_p50=pct(tpot, 50), tpot_ms_p99=pct(tpot, 99),
                    itl_ms_p50=pct(gaps, 50), itl_ms_p99=pct(gaps, 99), itl_ms_p999=pct(gaps, 99.9))

    def close(self):
        self.torch.cuda.synchronize()
        if self.model:
            C.cloak_model_free(self.model)
            self.model = None
        self.cw.close()

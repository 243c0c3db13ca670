"""Benchmark of the cloaked linear layer on one MI355X.

Workload (one step): a decode pass through every linear layer of one
Llama-3.1-8B-class decoder layer in BF16 (d_model 4096, d_ffn 14336, 8 KV
heads of 128: q/o 4096x4096, k/v 1024x4096, gate/up 14336x4096, down
4096x14336) at batch M=1, with the weights cut into 2 MiB pages scattered
over an 8 GiB pool.  Sixteen independent copies of the layer live in the
pool and are cycled, so the 6.5 GiB working set is far larger than the
256 MB Infinity Cache.  One step = cloak_linear_fused(q,k,v) + cloak_linear(o)
+ cloak_swiglu(gate,up) + cloak_down.

Reported: algorithmic GB/s of the cloaked step (weights + activations read,
results written, each counted once); the same for the untranslated twin on
the contiguous identity layout (native) and their ratio; the same at M in
{8, 32, 64}; the dominant kernel (the gate/up SwiGLU GEMV) against the
8 TB/s HBM peak, timed with HIP events on the launch stream; the in-place
remap of all 4096 pages against a device-to-device copy of the same bytes;
and the CPU oracle timed on a bounded sample of the same step.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cloaked/native ratio of decode GB/s and prefill TFLOP/s; p50/p99 token latency"
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0
COPIES = 16
TENSORS_PER_LAYER = 7   # q k v o gate up down
HERE = ROOT
# HBM bytes of one gate/up SwiGLU GEMV launch at M=1 from hardware counters
# (FETCH_SIZE and WRITE_SIZE, one rocprofv3 --pmc pass each, scaled by what the
# same counters read for an elementwise copy of known size), valid for the
# kernel sources with this digest; None until counters are taken.
SWIGLU_COUNTERS = dict(sources="3c8ea2d9cfb16c14", fetch_bytes=235092549, write_bytes=114745)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def layer_bytes(cfg, M):
    """Algorithmic bytes of one step, per call: (qkv, o, swiglu, down)."""
    d, f, kv = cfg["d_model"], cfg["d_ffn"], cfg["d_kv"]
    e = 2
    qkv = (d * d + 2 * kv * d) * e + M * d * e + M * (d + 2 * kv) * e
    o = d * d * e + M * d * e + M * d * e
    swiglu = 2 * f * d * e + M * d * e + M * f * e
    down = d * f * e + M * f * e + M * d * e
    return qkv, o, swiglu, down


class Variant:
    """A pool holding COPIES layer copies, plus activation buffers."""

    def __init__(self, C, shapes, weights, cfg, flags, seed, vmm=False, decoy=None, stored=False):
        # stored: q/k/v and o in stored order (cloak_linear_stored), as the
        # decoder step runs them around attention
        self.stored = stored
        self.cw = C.CloakedWeights(shapes, cfg["page_bytes"], cfg["pool_bytes"], seed=seed, flags=flags, vmm=vmm,
                                   decoy=decoy)
        self.cw.load(weights)
        self.C = C
        self.cfg = cfg

    def buffers(self, M):
        import torch
        from paper_2606_18400_amd import synth
        d, f, kv = self.cfg["d_model"], self.cfg["d_ffn"], self.cfg["d_kv"]
        x = torch.from_numpy(synth.activations(M, d, "bf16").view(np.int16)).cuda().view(torch.bfloat16)
        C, L = self.C, self.cw.layout
        # one workspace large enough for every call of the step (split-K partial sums)
        need = max(C.cloak_linear_fused_ws_bytes(L, [0, 1, 2], M), C.cloak_ws_bytes(L, C.CLOAK_OP_LINEAR, 3, M),
                   C.cloak_ws_bytes(L, C.CLOAK_OP_SWIGLU, 0, M), C.cloak_ws_bytes(L, C.CLOAK_OP_DOWN, 0, M))
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        return dict(x=x, ws=ws,
                    qkv=torch.empty((M, d + 2 * kv), dtype=torch.bfloat16, device="cuda"),
                    o=torch.empty((M, d), dtype=torch.bfloat16, device="cuda"),
                    h=torch.empty((M, f), dtype=torch.bfloat16, device="cuda"),
                    y=torch.empty((M, d), dtype=torch.bfloat16, device="cuda"))

    def step(self, i, M, b, ev=None):
        C, cw = self.C, self.cw
        L, pool = cw.layout, cw.pool
        l = i % COPIES
        t0 = TENSORS_PER_LAYER * l
        ws, wsb = b["ws"], b["ws"].numel()
        if self.stored:
            C.cloak_linear_stored(L, pool, [t0, t0 + 1, t0 + 2], b["x"], M, b["qkv"], ws, wsb)
            C.cloak_linear_stored(L, pool, [t0 + 3], b["x"], M, b["o"], ws, wsb)
        else:
            C.cloak_linear_fused(L, pool, [t0, t0 + 1, t0 + 2], b["x"], M, b["qkv"], ws, wsb)
            C.cloak_linear(L, pool, t0 + 3, b["x"], M, b["o"], ws, wsb)
        if ev is not None:
            ev[0].record()
        C.cloak_swiglu(L, pool, l, b["x"], M, b["h"], ws, wsb)
        if ev is not None:
            ev[1].record()
        C.cloak_down(L, pool, l, b["h"], M, b["y"], ws, wsb)


def time_steps(var, M, steps, warmup, kernel_events=False, spread=None):
    """Mean ms per step over `steps` back-to-back steps (events around the whole
    loop).  With `spread` (a dict), also events between consecutive steps on
    the launch stream, whose p10/p50/p90 are stored into it."""
    import torch
    b = var.buffers(M)
    for i in range(warmup):
        var.step(i, M, b)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)] if kernel_events else None
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)] if spread is not None else None
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for i in range(steps):
        if marks:
            marks[i].record()
        var.step(i, M, b, evs[i] if evs else None)
    if marks:
        marks[steps].record()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    kms = None
    if evs:
        kms = float(np.mean([a.elapsed_time(z) for a, z in evs]))
    if marks:
        per = np.array([marks[i].elapsed_time(marks[i + 1]) for i in range(steps)])
        spread.update({f"ms_p{q}": float(np.percentile(per, q)) for q in (10, 50, 90)})
    return ms, kms


def time_swiglu_loop(var, M, reps, warmup=8):
    """Average duration of the dominant kernel: `reps` back-to-back cloak_swiglu
    launches cycling over the layer copies (so no launch finds its weights in
    the 256 MB last-level cache), bracketed by events on the launch stream."""
    import torch
    b = var.buffers(M)
    C, cw = var.C, var.cw
    ws, wsb = b["ws"], b["ws"].numel()
    for i in range(warmup):
        C.cloak_swiglu(cw.layout, cw.pool, i % COPIES, b["x"], M, b["h"], ws, wsb)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for i in range(reps):
        C.cloak_swiglu(cw.layout, cw.pool, i % COPIES, b["x"], M, b["h"], ws, wsb)
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / reps


def kernel_sources_digest():
    """Digest of the sources the decode GEMV is built from; hardware byte
    counters recorded for one build are reported only while it matches."""
    import hashlib
    h = hashlib.sha256()
    for f in ("gemv.hip", "kernels.hpp"):
        with open(os.path.join(HERE, "paper_2606_18400_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def layer_flops(cfg, M):
    d, f, kv = cfg["d_model"], cfg["d_ffn"], cfg["d_kv"]
    return 2 * M * (d * d + 2 * kv * d + d * d + 3 * f * d)


def time_prefill(var, M, reps, warmup):
    """One prefill step (q,k,v fused, o, SwiGLU gate/up, down) at M tokens."""
    import torch
    b = var.buffers(M)
    for i in range(warmup):
        var.step(i, M, b)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for i in range(reps):
        var.step(i, M, b, evs[i])
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    k_ms = float(np.mean([a.elapsed_time(z) for a, z in evs]))
    del b
    return ms, k_ms


def time_remap(var, reps, with_copy=True):
    import torch
    pool_bytes = var.cfg["pool_bytes"]
    var.cw.remap(1000)   # warm
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for r in range(reps):
        var.cw.remap(1001 + r)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    wall_ms = (time.perf_counter() - t0) * 1e3 / reps
    if not with_copy:
        return dict(pool_bytes=pool_bytes, ms=ms, wall_ms=wall_ms, gbs=2 * pool_bytes / ms / 1e6)
    # device-to-device copy of the same number of bytes (read once, written once)
    half = pool_bytes // 2
    src = var.cw.pool[:half]
    dst = torch.empty(half, dtype=torch.uint8, device="cuda")
    dst.copy_(src)
    torch.cuda.synchronize()
    start.record()
    for _ in range(reps):
        dst.copy_(src)
        src.copy_(dst)
    stop.record()
    torch.cuda.synchronize()
    copy_ms = start.elapsed_time(stop) / reps
    del dst
    traffic = 2 * pool_bytes
    return dict(pool_bytes=pool_bytes, ms=ms, gbs=traffic / ms / 1e6, memcpy_ms=copy_ms,
                memcpy_gbs=traffic / copy_ms / 1e6, ratio=(traffic / ms) / (traffic / copy_ms),
                frac_of_peak=traffic / ms / 1e6 / HBM_PEAK_GBS)


def vendor_gemm(M, shapes_nk, reps=10):
    """The library GEMM (torch.nn.functional.linear on a contiguous nn.Linear
    [N][K] BF16 weight, untranslated) at the prefill shapes for comparison:
    TFLOP/s per (N, K)."""
    import torch
    import torch.nn.functional as F
    out = {}
    x = {}
    for (n, k) in shapes_nk:
        if k not in x:
            x[k] = torch.empty((M, k), dtype=torch.bfloat16, device="cuda").normal_()
        w = torch.empty((n, k), dtype=torch.bfloat16, device="cuda").normal_()
        y = F.linear(x[k], w)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            y = F.linear(x[k], w)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        out[f"{n}x{k}"] = dict(ms=ms, tflops=2 * M * n * k / ms / 1e9)
        del w, y
    del x
    torch.cuda.empty_cache()
    return out


def bench_prefill(args):
    """The BF16 prefill GEMM alone: the gate/up SwiGLU launch of the 4096/14336
    layer at 8192 tokens (cloaked and native), back to back over 16 layer
    copies, and the library GEMM at the same shapes.  A short run for
    hardware-counter passes of the prefill kernel."""
    import torch
    from paper_2606_18400_amd import cloak as C
    from paper_2606_18400_amd import synth
    cfg = synth.LAYER4096
    d, f, kv = cfg["d_model"], cfg["d_ffn"], cfg["d_kv"]
    one = synth.decoder_layer_shapes(d, f, kv, "bf16", layer=0)
    shapes = [(l, k, n, kk, dt) for l in range(COPIES) for (_, k, n, kk, dt) in one]
    w1 = [synth.weight(t, s[2], s[3], "bf16")[0] for t, s in enumerate(one)]
    weights = [w1[t % TENSORS_PER_LAYER] for t in range(len(shapes))]
    M = args.prefill_tokens
    res = {}
    for name, flags in (("cloaked", 0), ("native", C.CLOAK_IDENTITY | C.CLOAK_NATIVE)):
        var = Variant(C, shapes, weights, cfg, flags, seed=1)
        b = var.buffers(M)
        cw = var.cw
        ws, wsb = b["ws"], b["ws"].numel()
        reps = max(args.steps // 20, 5)
        for i in range(2):
            C.cloak_swiglu(cw.layout, cw.pool, i, b["x"], M, b["h"], ws, wsb)
        torch.cuda.synchronize()
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for i in range(reps):
            C.cloak_swiglu(cw.layout, cw.pool, i % COPIES, b["x"], M, b["h"], ws, wsb)
        z.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(z) / reps
        fl = 2 * M * 2 * f * d
        res[name] = dict(ms=ms, tflops=fl / ms / 1e9, frac=fl / ms / 1e9 / MFMA_BF16_PEAK_TFLOPS)
        log(f"{name} SwiGLU GEMM {M} tokens: {ms:.3f} ms, {fl / ms / 1e9:.0f} TFLOP/s")
        del b
        cw.close()
        torch.cuda.empty_cache()
    res["library_gemm"] = vendor_gemm(M, [(2 * f, d)])
    out = {"metric": "prefill SwiGLU GEMM TFLOP/s", "value": res["cloaked"]["tflops"], "unit": "TFLOP/s",
           "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": f"gate/up SwiGLU GEMM of the 4096/14336 BF16 layer at {M} tokens, 2 MiB pages "
                                  f"over an 8 GiB pool, 16 layer copies cycled"},
           "prefill": res}
    print(json.dumps(out), flush=True)


def time_uniform_remap(C, shapes, cfg, reps):
    """The uniform remap (CLOAK_REMAP_UNIFORM: a fresh rho over all pages, two
    passes of page-pair swaps) on a layout of the same shapes and pool.  Bytes
    moved: each swapped pair reads and writes two pages."""
    import torch
    cw = C.CloakedWeights(shapes, cfg["page_bytes"], cfg["pool_bytes"], seed=1, flags=C.CLOAK_REMAP_UNIFORM)
    cw.remap(2000)
    torch.cuda.synchronize()
    pairs = []
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    total = 0.0
    for r in range(reps):
        C.cloak_remap_begin(cw.layout, 2001 + r)
        pairs.append(C.cloak_query(cw.layout, "REMAP_PENDING"))
        start.record()
        C.cloak_remap_step(cw.layout, cw.pool, 0)
        stop.record()
        torch.cuda.synchronize()
        total += start.elapsed_time(stop)
    ms = total / reps
    moved = 4 * cfg["page_bytes"] * float(np.mean(pairs))
    cw.close()
    return dict(ms=ms, pairs_mean=float(np.mean(pairs)), bytes_moved=moved, gbs=moved / ms / 1e6,
                frac_of_peak=moved / ms / 1e6 / HBM_PEAK_GBS, pool_remaps_per_s=1e3 / ms)


def copy_calibration(nbytes=1 << 30):
    """A plain elementwise copy of known size (reads and writes nbytes once);
    hardware byte counters of the decode kernels are scaled by what they read
    for this kernel."""
    import torch
    src = torch.ones(nbytes // 2, dtype=torch.bfloat16, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1, out=dst)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    torch.mul(src, 1, out=dst)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    del src, dst
    return dict(bytes_read=nbytes, bytes_written=nbytes, ms=ms, gbs=2 * nbytes / ms / 1e6)


def read_ceiling(nbytes, copies=16, reps=64):
    """Plain streaming-read rate (cloak_stream_read) over `copies` distinct
    regions of nbytes, cycled so that no launch finds its bytes in the
    last-level cache: the practical ceiling of a kernel that reads nbytes."""
    import torch
    from paper_2606_18400_amd import cloak as C
    nbytes = nbytes // 256 * 256
    buf = torch.ones(copies * nbytes, dtype=torch.uint8, device="cuda")
    out = torch.zeros(1, dtype=torch.int32, device="cuda")
    for i in range(copies):
        C.cloak_stream_read(buf[i * nbytes:], nbytes, out)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for i in range(reps):
        C.cloak_stream_read(buf[(i % copies) * nbytes:], nbytes, out)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    del buf
    torch.cuda.empty_cache()
    return dict(bytes=nbytes, ms=ms, gbs=nbytes / ms / 1e6)


def vendor_gemv(rows, cols, copies=16, reps=64):
    """The library GEMV (torch.mv on contiguous BF16 matrices of the SwiGLU
    kernel's shape) for comparison: `copies` distinct matrices cycled so that no
    call finds its matrix in the last-level cache; events on the stream."""
    import torch
    w = torch.empty((copies, rows, cols), dtype=torch.bfloat16, device="cuda").normal_()
    x = torch.empty(cols, dtype=torch.bfloat16, device="cuda").normal_()
    for i in range(copies):
        torch.mv(w[i], x)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for i in range(reps):
        torch.mv(w[i % copies], x)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    del w
    torch.cuda.empty_cache()
    return dict(rows=rows, cols=cols, ms=ms, gbs=(rows * cols + cols + rows) * 2 / ms / 1e6)


def cpu_model_name():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_oracle_baseline(cfg, weights, runs=3, budget_s=4.0):
    """The oracle's FP64 decode step (decode stored weights, then the products),
    timed around the compute only: `runs` runs of about budget_s each with the
    BLAS pool at its default size (median reported), then one run on 1 thread."""
    from oracle import numerics as ON
    from paper_2606_18400_amd import synth
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count()
    d = cfg["d_model"]
    x = ON.bf16_bits_to_f64(synth.activations(1, d, "bf16"))
    step_bytes = sum(layer_bytes(cfg, 1))

    def one_run(budget):
        steps, el = 0, 0.0
        while el < budget and steps < 20:
            t0 = time.perf_counter()
            w = [ON.weights_f64(weights[t], "bf16") for t in range(TENSORS_PER_LAYER)]
            for t in range(4):
                ON.linear(x, w[t])
            ON.swiglu_ffn(x, w[4], w[5], w[6])
            el += time.perf_counter() - t0
            del w
            steps += 1
        return step_bytes * steps / el / 1e9, steps, el

    res = [one_run(budget_s) for _ in range(runs)]
    vals = sorted(r[0] for r in res)
    one_thread = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            one_thread = one_run(budget_s)[0]
    steps, el = sum(r[1] for r in res), sum(r[2] for r in res)
    return dict(value=float(np.median(vals)), unit="GB/s", cores=int(threads), kind="oracle",
                runs=[float(v) for v in vals], one_thread_value=one_thread, cpu=cpu_model_name(),
                sample=f"{runs} runs, {steps} decode steps (M=1) in all, of one 4096/14336 BF16 layer: bf16->FP64 "
                       f"weight decode plus FP64 products, {el:.1f} s of compute; median of the runs")


def gpu_clocks():
    """Clocks and power of the GPU now (rocm-smi in a child process), or None."""
    import shutil
    import subprocess
    exe = shutil.which("rocm-smi") or "/opt/rocm/bin/rocm-smi"
    try:
        r = subprocess.run([exe, "--showclocks", "--showpower", "--json"], capture_output=True, text=True,
                           timeout=30)
        data = json.loads(r.stdout)
    except Exception:
        return None
    card = data.get("card0") or next(iter(data.values()), {})
    keep = {}
    for k, v in card.items():
        kl = k.lower()
        if "sclk" in kl or "mclk" in kl or "fclk" in kl or "power" in kl:
            keep[k] = v
    return keep or None


def serve_weights():
    """Weights of the 32-layer serving stack: one decoder layer's random weights
    in every layer (each layer still has its own placement), embed and head."""
    from paper_2606_18400_amd import serve, synth
    cfg = serve.LLAMA8B
    shapes = serve.model_shapes(cfg)
    layer_w = [synth.weight(t, s[2], s[3], "bf16")[0] for t, s in enumerate(shapes[:TENSORS_PER_LAYER])]
    emb = synth.weight(len(shapes) - 2, cfg["vocab"], cfg["d_model"], "bf16")[0]
    head = synth.weight(len(shapes) - 1, cfg["vocab"], cfg["d_model"], "bf16")[0]
    return [layer_w[t % TENSORS_PER_LAYER] for t in range(len(shapes) - 2)] + [emb, head]


def serve_variants(weights, rates, requests, hardened=False, remap_sweep="", cadence_rates=None, only=None):
    """Serving trace on the 32-layer 4096/14336 BF16 stack (vocab 128256):
    Poisson arrivals, prompts U[128,4096], outputs U[64,1024], continuous
    batching with paged KV, remap every 256 steps (cloaked) vs the identity
    layout with untranslated kernels and no remap (native)."""
    import torch
    from paper_2606_18400_amd import cloak as C
    from paper_2606_18400_amd import serve, synth
    cfg = serve.LLAMA8B
    results = {}
    every_default = 256
    variants = [("cloaked", 0, every_default, None), ("native", C.CLOAK_IDENTITY | C.CLOAK_NATIVE, 0, None)]
    if hardened:
        # permuted heads (default), SHA-256 draws, masked device map re-keyed by every remap, decoy free pages
        variants.append(("hardened", C.CLOAK_CSPRNG | C.CLOAK_MASKED_MAP, every_default, True))
    if only:
        variants = [v for v in variants if v[0] in only]
    for name, flags, every, decoy in variants:
        log(f"{name}: loading 32 layers into a 16 GiB pool")
        eng = serve.Engine(cfg, pool_bytes=16 << 30, page_bytes=2 << 20, seed=1, flags=flags, kv_blocks=24576,
                           max_tokens=2048, prefill_chunk=512, max_seqs=64, split_keys=512, remap_every=every,
                           weights=weights, max_context=8192, decoy=decoy)
        results[name] = {}

        def one_run(rate):
            trace = synth.poisson_trace(requests, rate, 128, 4096, 64, 1024, cfg["vocab"], seed=7)
            reqs = [serve.Request(t["id"], t["prompt"], t["max_new"], t["arrival"]) for t in trace]
            steps0, remaps0, ms0, ev0 = eng.steps, eng.remaps, len(eng.step_ms), len(eng.remap_events)
            rep = eng.run(reqs, progress=lambda done, n, t: log(f"  rate {rate}/s: {done}/{n} requests done, {t:.0f} s"))
            rep["steps"] = eng.steps - steps0
            rep["remaps"] = eng.remaps - remaps0
            sm = np.array(eng.step_ms[ms0:])
            rep.update({f"step_ms_p{q}": float(np.percentile(sm, q)) for q in (50, 99, 99.9)})
            rep["step_ms_max"] = float(sm.max())
            rm = eng.remap_ms(ev0)
            rep["remap_slices_run"] = len(rm)
            rep["remap_slice_ms_max"] = max(rm) if rm else 0.0
            rep["remap_ms_total"] = float(sum(rm))
            rep["remap_share_of_step_time"] = float(sum(rm)) / float(sm.sum()) if sm.size else 0.0
            return rep

        for rate in rates:
            rep = one_run(rate)
            results[name][str(rate)] = rep
            log(f"{name} rate {rate}/s: ttft p50 {rep['ttft_ms_p50']:.0f} p99 {rep['ttft_ms_p99']:.0f} ms, "
                f"tpot p50 {rep['tpot_ms_p50']:.1f} p99 {rep['tpot_ms_p99']:.1f} ms, "
                f"{rep['output_tok_per_s']:.0f} tok/s, {rep['steps']} steps, {rep['remaps']} remaps")
        if name == "cloaked" and remap_sweep:
            # cadence sweep: remap every N steps, spread over S steps (N=0: never), at each cadence rate
            results["cadence"] = {}
            for crate in (cadence_rates or rates[:1]):
                results["cadence"][str(crate)] = {}
                for item in remap_sweep.split(","):
                    every, slices = (int(v) for v in item.split(":"))
                    eng.remap_every, eng.remap_slices = every, slices
                    rep = one_run(crate)
                    results["cadence"][str(crate)][item] = rep
                    log(f"cadence at {crate}/s every {every} over {slices} steps: itl p50 {rep['itl_ms_p50']:.1f} "
                        f"p99 {rep['itl_ms_p99']:.1f} p99.9 {rep['itl_ms_p999']:.1f} ms, {rep['remaps']} remaps, "
                        f"largest remap stall {rep['remap_slice_ms_max']:.2f} ms, remap share of step time "
                        f"{100 * rep['remap_share_of_step_time']:.2f}%")
            eng.remap_every, eng.remap_slices = every_default, 1
        eng.close()
        del eng
        torch.cuda.empty_cache()
    return results


def bench_serve(args):
    from paper_2606_18400_amd import serve
    log("generating weights (one decoder layer's random weights in every layer, distinct placement)")
    weights = serve_weights()
    rates = [float(r) for r in args.rates.split(",")]
    crates = [float(r) for r in args.cadence_rates.split(",")] if args.cadence_rates else None
    only = args.serve_variants.split(",") if args.serve_variants else None
    results = serve_variants(weights, rates, args.requests, args.hardened, args.remap_sweep, crates, only)
    first = str(rates[0])
    lead = "cloaked" if "cloaked" in results else next(iter(results))
    out = {"metric": METRIC, "value": results[lead][first]["output_tok_per_s"] if first in results[lead] else None,
           "unit": "tokens/s",
           "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": f"serving trace on a 32-layer 4096/14336/1024 BF16 stack, vocab 128256, "
                                  f"{args.requests} requests per rate, Poisson rates {rates} req/s, prompts "
                                  f"U[128,4096], outputs U[64,1024], remap every 256 steps"},
           "serving": results}
    print(json.dumps(out), flush=True)


def stack_shapes(cfg):
    shapes = []
    for l in range(cfg["n_layers"]):
        shapes += synth_decoder(cfg, l)
    shapes.append((-1, "head", cfg["vocab"], cfg["d_model"], "bf16"))
    return shapes


def synth_decoder(cfg, l):
    from paper_2606_18400_amd import synth
    return synth.decoder_layer_shapes(cfg["d_model"], cfg["d_ffn"], cfg["d_kv"], "fp8", layer=l)


def bench_stack(args):
    """Decode step through a 64-layer FP8 E4M3 stack (5120/27648/1024, per-row
    FP32 scales) and its BF16 head (152064 x 5120), 2 MiB pages over 34 GiB."""
    import torch
    from paper_2606_18400_amd import cloak as C
    from paper_2606_18400_amd import synth
    cfg = synth.STACK5120
    shapes = stack_shapes(cfg)
    log("generating and quantising one FP8 layer (reused by all 64 layers, distinct placement) and the head")
    lw = [synth.weight(t, s[2], s[3], "fp8") for t, s in enumerate(shapes[:TENSORS_PER_LAYER])]
    head = synth.weight(len(shapes) - 1, cfg["vocab"], cfg["d_model"], "bf16")[0]
    weights = [lw[t % TENSORS_PER_LAYER][0] for t in range(len(shapes) - 1)] + [head]
    scales = [lw[t % TENSORS_PER_LAYER][1] for t in range(len(shapes) - 1)] + [None]
    L = cfg["n_layers"]
    d, f, kv, V = cfg["d_model"], cfg["d_ffn"], cfg["d_kv"], cfg["vocab"]
    layer_bytes_fp8 = (d * d * 2 + 2 * kv * d + 3 * f * d) + (d + 2 * kv + d + 3 * f) * 4

    def step_bytes(M):
        acts = L * 2 * M * (d + (d + 2 * kv) + d + d + d + f + f + d) + 2 * M * (d + V)
        return L * layer_bytes_fp8 + V * d * 2 + acts

    res = {}
    for name, flags in [("cloaked", 0), ("native", C.CLOAK_IDENTITY | C.CLOAK_NATIVE)]:
        log(f"{name}: loading 64 FP8 layers + head into a 34 GiB pool")
        cw = C.CloakedWeights(shapes, cfg["page_bytes"], cfg["pool_bytes"], seed=1, flags=flags)
        cw.load(weights, scales)
        res[name] = {}
        for M in [int(m) for m in args.stack_batches.split(",")]:
            x = torch.from_numpy(synth.activations(M, d, "bf16").view(np.int16)).cuda().view(torch.bfloat16)
            qkv = torch.empty((M, d + 2 * kv), dtype=torch.bfloat16, device="cuda")
            o = torch.empty((M, d), dtype=torch.bfloat16, device="cuda")
            h = torch.empty((M, f), dtype=torch.bfloat16, device="cuda")
            y = torch.empty((M, d), dtype=torch.bfloat16, device="cuda")
            logits = torch.empty((M, V), dtype=torch.bfloat16, device="cuda")
            need = max(C.cloak_linear_fused_ws_bytes(cw.layout, [0, 1, 2], M),
                       C.cloak_ws_bytes(cw.layout, C.CLOAK_OP_SWIGLU, 0, M),
                       C.cloak_ws_bytes(cw.layout, C.CLOAK_OP_DOWN, 0, M),
                       C.cloak_ws_bytes(cw.layout, C.CLOAK_OP_LINEAR, len(shapes) - 1, M))
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")

            def one_step():
                for l in range(L):
                    t0 = TENSORS_PER_LAYER * l
                    C.cloak_linear_fused(cw.layout, cw.pool, [t0, t0 + 1, t0 + 2], x, M, qkv, ws, ws.numel())
                    C.cloak_linear(cw.layout, cw.pool, t0 + 3, x, M, o, ws, ws.numel())
                    C.cloak_swiglu(cw.layout, cw.pool, l, x, M, h, ws, ws.numel())
                    C.cloak_down(cw.layout, cw.pool, l, h, M, y, ws, ws.numel())
                C.cloak_linear(cw.layout, cw.pool, len(shapes) - 1, x, M, logits, ws, ws.numel())

            one_step()
            torch.cuda.synchronize()
            reps = max(args.steps // 40, 3)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                one_step()
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            res[name][str(M)] = dict(ms=ms, gbs=step_bytes(M) / ms / 1e6)
            log(f"{name} M={M}: {ms:.2f} ms/step, {step_bytes(M) / ms / 1e6:.0f} GB/s")
        pm = args.prefill_tokens
        if pm > 0:
            # prefill of one FP8 layer (FP8 x FP8 MFMA on per-token E4M3 activations), cycling layers
            x = torch.from_numpy(synth.activations(pm, d, "bf16").view(np.int16)).cuda().view(torch.bfloat16)
            qkv = torch.empty((pm, d + 2 * kv), dtype=torch.bfloat16, device="cuda")
            o = torch.empty((pm, d), dtype=torch.bfloat16, device="cuda")
            h = torch.empty((pm, f), dtype=torch.bfloat16, device="cuda")
            y = torch.empty((pm, d), dtype=torch.bfloat16, device="cuda")
            need = max(C.cloak_linear_fused_ws_bytes(cw.layout, [0, 1, 2], pm),
                       C.cloak_ws_bytes(cw.layout, C.CLOAK_OP_LINEAR, 3, pm),
                       C.cloak_ws_bytes(cw.layout, C.CLOAK_OP_SWIGLU, 0, pm),
                       C.cloak_ws_bytes(cw.layout, C.CLOAK_OP_DOWN, 0, pm))
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")

            def prefill_layer(l):
                t0 = TENSORS_PER_LAYER * l
                C.cloak_linear_fused(cw.layout, cw.pool, [t0, t0 + 1, t0 + 2], x, pm, qkv, ws, ws.numel())
                C.cloak_linear(cw.layout, cw.pool, t0 + 3, x, pm, o, ws, ws.numel())
                C.cloak_swiglu(cw.layout, cw.pool, l, x, pm, h, ws, ws.numel())
                C.cloak_down(cw.layout, cw.pool, l, h, pm, y, ws, ws.numel())

            prefill_layer(0)
            torch.cuda.synchronize()
            reps = 8
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for i in range(reps):
                prefill_layer(1 + i)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            fl = 2 * pm * (d * d * 2 + 2 * kv * d + 3 * f * d)
            res[name]["prefill"] = dict(tokens=pm, ms=ms, tflops=fl / ms / 1e9, peak_fp8_tflops=5000.0,
                                        frac=fl / ms / 1e9 / 5000.0)
            log(f"{name} FP8 prefill {pm} tokens: {ms:.2f} ms per layer, {fl / ms / 1e9:.0f} TFLOP/s")
            del x, qkv, o, h, y, ws
        cw.close()
        torch.cuda.empty_cache()
    for M in res["cloaked"]:
        res["cloaked"][M]["ratio"] = res["native"][M]["ms"] / res["cloaked"][M]["ms"]
    m0 = args.stack_batches.split(",")[0]
    out = {"metric": METRIC, "value": res["cloaked"][m0]["gbs"], "unit": "GB/s", "n_gpus": 1,
           "ms_per_step": res["cloaked"][m0]["ms"], "higher_is_better": True, "vs_baseline": None, "dtype": "fp8",
           "data": "synthetic",
           "config": {"workload": "decode step through a 64-layer FP8 E4M3 5120/27648/1024 stack with per-row FP32 "
                                  "scales and a BF16 152064x5120 head, 2 MiB pages over a 34 GiB pool",
                      "step_bytes_M1": step_bytes(1)},
           "stack": res}
    print(json.dumps(out), flush=True)


def bench_oracle(args):
    """The CPU oracle timed on the host at every workload it can finish: the
    decode step of the 4096/14336 layer, its 8192-token prefill (full FP64
    products per tensor), the 64-layer FP8 5120/27648 stack (one layer and
    the head timed, extrapolated to 64 layers), and the page remap of an 8 GiB
    pool in NumPy.  Compute only, inputs made beforehand; median of `runs` runs
    with the BLAS pool at its default size, and one run on one thread (for the
    prefill on 512 of the 8192 tokens, scaled)."""
    from oracle import numerics as ON
    from oracle import remap as OR
    from paper_2606_18400_amd import synth
    from threadpoolctl import threadpool_info, threadpool_limits
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    runs = 3

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    def med_and_one(fn, one=None, scale=1.0):
        ts = sorted(timed(fn) for _ in range(runs))
        with threadpool_limits(limits=1):
            t1 = timed(one or fn) * scale
        return dict(s_median=ts[len(ts) // 2], s_runs=ts, s_one_thread=t1)

    out = {"threads": int(threads), "cpu": cpu_model_name(), "runs": runs}
    cfg = synth.LAYER4096
    d, f, kv = cfg["d_model"], cfg["d_ffn"], cfg["d_kv"]
    shapes = synth.decoder_layer_shapes(d, f, kv, "bf16", layer=0)
    log("oracle: 4096/14336 layer weights")
    stored = [synth.weight(t, s[2], s[3], "bf16")[0] for t, s in enumerate(shapes)]
    x1 = ON.bf16_bits_to_f64(synth.activations(1, d, "bf16"))

    def decode(x):
        # the oracle's step: exact FP64 values of the stored weights, then the products
        w64 = [ON.weights_f64(w, "bf16") for w in stored]
        for t in range(4):
            ON.linear(x, w64[t])
        ON.swiglu_ffn(x, w64[4], w64[5], w64[6])

    r = med_and_one(lambda: decode(x1))
    r["gbs_median"] = sum(layer_bytes(cfg, 1)) / r["s_median"] / 1e9
    out["decode_layer4096_M1"] = r
    log(f"oracle decode M=1: {r['s_median'] * 1e3:.0f} ms")
    M = 8192
    xp = ON.bf16_bits_to_f64(synth.activations(M, d, "bf16"))
    r = med_and_one(lambda: decode(xp), lambda: decode(xp[:512]), M / 512)
    r["tflops_median"] = layer_flops(cfg, M) / r["s_median"] / 1e12
    r["note"] = "one-thread figure: 512 of the 8192 tokens, scaled by 16"
    out["prefill_layer4096_M8192"] = r
    log(f"oracle prefill 8192 tokens: {r['s_median']:.1f} s ({r['tflops_median'] * 1e3:.0f} GFLOP/s)")
    del stored, xp
    sc = synth.STACK5120
    d, f, kv, V = sc["d_model"], sc["d_ffn"], sc["d_kv"], sc["vocab"]
    fshapes = synth.decoder_layer_shapes(d, f, kv, "fp8", layer=0)
    log("oracle: 5120/27648 FP8 layer and the 152064 x 5120 head")
    fw = [synth.weight(t, s[2], s[3], "fp8") for t, s in enumerate(fshapes)]
    head = synth.weight(7, V, d, "bf16")[0]
    xs = ON.bf16_bits_to_f64(synth.activations(1, d, "bf16"))

    def one_layer():
        # the layer decoded from its stored E4M3 bytes and row scales, then the products
        w = [ON.weights_f64(q, "fp8", s) for q, s in fw]
        for t in range(4):
            ON.linear(xs, w[t])
        ON.swiglu_ffn(xs, w[4], w[5], w[6])

    def head_step():
        ON.linear(xs, ON.weights_f64(head, "bf16"))

    r = med_and_one(one_layer)
    rh = med_and_one(head_step)
    r["head"] = rh
    r["note"] = "one layer timed (s_median), the head separately; s_extrapolated = 64 layers + the head"
    r["s_extrapolated_64_layers"] = r["s_median"] * 64 + rh["s_median"]
    r["s_extrapolated_one_thread"] = r["s_one_thread"] * 64 + rh["s_one_thread"]
    out["stack5120_fp8_M1"] = r
    log(f"oracle stack: {r['s_median']:.1f} s per layer, head {rh['s_median']:.1f} s, "
        f"64 layers ~{r['s_extrapolated_64_layers']:.0f} s")
    del fw, head
    B, P = 2 << 20, 4096
    log("oracle: remap of an 8 GiB pool")
    pool = np.zeros(B * P, np.uint8)
    phi = list(range(P))
    ts = []
    for rsd in range(runs):
        t0 = time.perf_counter()
        OR.remap(pool, phi, 1 + rsd, B)
        ts.append(time.perf_counter() - t0)
    ts.sort()
    out["remap_pool8GiB"] = dict(s_median=ts[len(ts) // 2], s_runs=ts, gbs_median=2 * B * P / ts[len(ts) // 2] / 1e9,
                                 note="NumPy page copies into a second pool image (the oracle's definition)")
    log(f"oracle remap of 8 GiB: {ts[len(ts) // 2]:.1f} s")
    print(json.dumps({"metric": "CPU oracle host timings", "oracle": out}), flush=True)


MOE = dict(slots=8, experts=128, top_k=8, d_model=2048, d_ffn=768, page_bytes=2 << 20, pool_bytes=12 << 30)


def bench_moe(args):
    """Decode through MoE layers of 128 cloaked BF16 experts (2048 -> 768 -> 2048,
    a Qwen-3-30B-A3B-like expert shape), top-8 routing, 8 layer slots cycled."""
    import torch
    from paper_2606_18400_amd import cloak as C
    from paper_2606_18400_amd import synth
    cfg = MOE
    E, k, d, F = cfg["experts"], cfg["top_k"], cfg["d_model"], cfg["d_ffn"]
    shapes = []
    for l in range(cfg["slots"]):
        for e in range(E):
            shapes += synth.ffn_block_shapes(d, F, "bf16", layer=l * E + e)
    log("generating 8 distinct experts (reused by every expert slot, distinct placement)")
    base = [synth.weight(t, s[2], s[3], "bf16")[0] for t, s in enumerate(shapes[:24])]
    weights = [base[t % 24] for t in range(len(shapes))]
    expert_bytes = 3 * d * F * 2
    res = {}
    batches = [int(m) for m in args.moe_batches.split(",") if m]
    for name, flags in [("cloaked", 0), ("native", C.CLOAK_IDENTITY | C.CLOAK_NATIVE)]:
        log(f"{name}: loading {cfg['slots']} x {E} experts into a {cfg['pool_bytes'] >> 30} GiB pool")
        cw = C.CloakedWeights(shapes, cfg["page_bytes"], cfg["pool_bytes"], seed=1, flags=flags)
        cw.load(weights)
        res[name] = {}
        for M in batches:
            rng = np.random.Generator(np.random.PCG64(17 + M))   # the same routing for both layouts
            ids = np.stack([rng.choice(E, k, replace=False) for _ in range(M)]).astype(np.int32)
            w = rng.random((M, k)).astype(np.float32)
            w /= w.sum(axis=1, keepdims=True)
            active = len(set(ids.ravel().tolist()))
            nbytes = active * expert_bytes + 2 * M * d * 2 + M * k * 8
            x = torch.from_numpy(synth.activations(M, d, "bf16").view(np.int16)).cuda().view(torch.bfloat16)
            y = torch.empty((M, d), dtype=torch.bfloat16, device="cuda")
            d_ids, d_w = torch.from_numpy(ids).cuda(), torch.from_numpy(w).cuda()
            need = C.cloak_moe_ws_bytes(cw.layout, 0, E, k, M)
            ws = torch.empty(need, dtype=torch.uint8, device="cuda")

            def call(i):
                C.cloak_moe(cw.layout, cw.pool, (i % cfg["slots"]) * E, E, k, x, M, d_ids, d_w, y, ws, need)

            for i in range(args.warmup):
                call(i)
            torch.cuda.synchronize()
            reps = max(args.steps, 16)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for i in range(reps):
                call(i)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / reps
            res[name][str(M)] = dict(ms=ms, gbs=nbytes / ms / 1e6, active_experts=active, bytes=nbytes)
            log(f"{name} M={M}: {ms * 1e3:.1f} us per MoE layer, {active} experts, {nbytes / ms / 1e6:.0f} GB/s")
        cw.close()
        torch.cuda.empty_cache()
    for M in res["cloaked"]:
        res["cloaked"][M]["ratio"] = res["native"][M]["ms"] / res["cloaked"][M]["ms"]
    m0 = str(batches[0])
    out = {"metric": METRIC, "value": res["cloaked"][m0]["gbs"], "unit": "GB/s", "n_gpus": 1,
           "ms_per_step": res["cloaked"][m0]["ms"], "higher_is_better": True, "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic",
           "config": {"workload": f"decode through one MoE layer of {E} BF16 experts {d}/{F}, top-{k} routing, "
                                  f"{cfg['slots']} layer slots cycled, 2 MiB pages over a 12 GiB pool",
                      "expert_bytes": expert_bytes},
           "moe": res}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--batches", default="8,32,64", help="extra decode batch sizes reported beside M=1")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--vmm", action="store_true",
                    help="also time the hardware-translated (VMM-mapped) twin of the cloaked layout")
    ap.add_argument("--hardened", action="store_true",
                    help="also time the hardened layout (permuted attention heads run in stored order, SHA-256 "
                         "draws, masked device page map, decoy free pages)")
    ap.add_argument("--remap-reps", type=int, default=5)
    ap.add_argument("--prefill-tokens", type=int, default=8192, help="prefill batch (0 skips the prefill pass)")
    ap.add_argument("--moe-batches", default="1,8,32,64,256", help="moe: decode batch sizes")
    ap.add_argument("--workload", default="layer", choices=["layer", "serve", "stack", "moe", "oracle", "prefill"],
                    help="layer: the headline decode layer (default); serve: serving trace; stack: 64-layer FP8")
    ap.add_argument("--rates", default="2,8", help="serve: Poisson arrival rates (req/s)")
    ap.add_argument("--requests", type=int, default=32, help="serve: requests per rate")
    ap.add_argument("--cadence-rates", default="", help="serve: rates of the cadence sweep (default: the first rate)")
    ap.add_argument("--serve-variants", default="", help="serve: comma list of cloaked,native,hardened (default all)")
    ap.add_argument("--remap-sweep", default="",
                    help="serve: cadence sweep 'every:slices,...' (e.g. 64:1,256:1,256:32,0:1) at the first rate")
    ap.add_argument("--stack-batches", default="1,8,32,64,256", help="stack: decode batch sizes")
    ap.add_argument("--serve-requests", type=int, default=24,
                    help="layer: requests of the short serving pass (0 skips it)")
    ap.add_argument("--serve-rate", type=float, default=2.0, help="layer: arrival rate of the short serving pass")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the multi-GPU (tensor-parallel) "
              "path is not built; each GPU would hold its own cloaked shard with its own seed", file=sys.stderr)
        sys.exit(2)

    if args.workload == "oracle":
        return bench_oracle(args)
    import torch
    from paper_2606_18400_amd import cloak as C
    from paper_2606_18400_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "stack":
        return bench_stack(args)
    if args.workload == "moe":
        return bench_moe(args)
    if args.workload == "prefill":
        return bench_prefill(args)
    cfg = synth.LAYER4096
    d, f, kv = cfg["d_model"], cfg["d_ffn"], cfg["d_kv"]
    one = synth.decoder_layer_shapes(d, f, kv, "bf16", layer=0)
    shapes = []
    for l in range(COPIES):
        shapes += [(l, k, n, kk, dt) for (_, k, n, kk, dt) in one]
    log("generating one BF16 layer of weights")
    w1 = [synth.weight(t, s[2], s[3], "bf16")[0] for t, s in enumerate(one)]
    weights = [w1[t % TENSORS_PER_LAYER] for t in range(len(shapes))]
    log("uploading 16 cloaked copies")
    cl = Variant(C, shapes, weights, cfg, 0, seed=1)
    log("uploading 16 native copies")
    nat = Variant(C, shapes, weights, cfg, C.CLOAK_IDENTITY | C.CLOAK_NATIVE, seed=1)
    # the translating kernels on the contiguous identity layout: separates the
    # cost of in-kernel translation from the effect of scattered placement
    log("uploading 16 identity-layout copies for the translating kernels")
    ident = Variant(C, shapes, weights, cfg, C.CLOAK_IDENTITY, seed=1)
    clocks_before = gpu_clocks()

    step_bytes = sum(layer_bytes(cfg, 1))
    swiglu_bytes = layer_bytes(cfg, 1)[2]
    log(f"timing M=1: {args.warmup} warmup + {args.steps} steps")
    spread, spread_nat, spread_id = {}, {}, {}
    ms, _ = time_steps(cl, 1, args.steps, args.warmup, spread=spread)
    ms_nat, _ = time_steps(nat, 1, args.steps, args.warmup, spread=spread_nat)
    ms_id, _ = time_steps(ident, 1, args.steps, args.warmup, spread=spread_id)
    # the dominant kernel alone, back to back, events around the whole loop
    k_ms = time_swiglu_loop(cl, 1, max(args.steps, 64))
    k_ms_nat = time_swiglu_loop(nat, 1, max(args.steps, 64))
    value = step_bytes / ms / 1e6
    native = step_bytes / ms_nat / 1e6
    log(f"M=1 cloaked {value:.0f} GB/s native {native:.0f} GB/s")
    decode = {"1": dict(cloaked_gbs=value, native_gbs=native, ratio=value / native, ms=ms, native_ms=ms_nat,
                        identity_translated_gbs=step_bytes / ms_id / 1e6, identity_translated_ms=ms_id,
                        cloaked_step_ms=spread, native_step_ms=spread_nat, identity_translated_step_ms=spread_id)}
    for M in [int(m) for m in args.batches.split(",") if m]:
        b = sum(layer_bytes(cfg, M))
        n_steps = max(args.steps // 4, 10)
        sp, sp_nat = {}, {}
        m_cl, _ = time_steps(cl, M, n_steps, args.warmup, spread=sp)
        m_nat, _ = time_steps(nat, M, n_steps, args.warmup, spread=sp_nat)
        m_id, _ = time_steps(ident, M, n_steps, args.warmup)
        decode[str(M)] = dict(cloaked_gbs=b / m_cl / 1e6, native_gbs=b / m_nat / 1e6, ratio=m_nat / m_cl,
                              ms=m_cl, native_ms=m_nat, identity_translated_gbs=b / m_id / 1e6,
                              identity_translated_ms=m_id, cloaked_step_ms=sp, native_step_ms=sp_nat)
        log(f"M={M} cloaked {b / m_cl / 1e6:.0f} GB/s native {b / m_nat / 1e6:.0f} GB/s "
            f"identity-translated {b / m_id / 1e6:.0f} GB/s")

    pm = args.prefill_tokens
    prefill = None
    if pm > 0:
        log(f"timing prefill M={pm}")
        p_ms, p_kms = time_prefill(cl, pm, max(args.steps // 20, 5), 2)
        n_ms, n_kms = time_prefill(nat, pm, max(args.steps // 20, 5), 2)
        i_ms, _ = time_prefill(ident, pm, max(args.steps // 20, 5), 2)
        fl = layer_flops(cfg, pm)
        sw_fl = 2 * pm * 2 * f * d
        prefill = dict(tokens=pm, cloaked_tflops=fl / p_ms / 1e9, native_tflops=fl / n_ms / 1e9,
                       ratio=n_ms / p_ms, ms=p_ms, native_ms=n_ms, identity_translated_tflops=fl / i_ms / 1e9,
                       identity_translated_ms=i_ms,
                       roofline=dict(kernel="gemm_kernel SwiGLU (gate+up, bf16 MFMA)", bound="mfma",
                                     achieved=sw_fl / p_kms / 1e9, peak=MFMA_BF16_PEAK_TFLOPS, unit="TFLOP/s",
                                     frac=sw_fl / p_kms / 1e9 / MFMA_BF16_PEAK_TFLOPS, flops_per_launch=sw_fl,
                                     avg_launch_ms=p_kms, native_avg_launch_ms=n_kms))
        log(f"prefill cloaked {fl / p_ms / 1e9:.0f} TFLOP/s native {fl / n_ms / 1e9:.0f} TFLOP/s")
        prefill["library_gemm"] = vendor_gemm(pm, [(d + 2 * kv, d), (d, d), (2 * f, d), (d, f)])
        log("library GEMM (torch linear) at the prefill shapes: " +
            ", ".join(f"{k} {v['tflops']:.0f}" for k, v in prefill["library_gemm"].items()) + " TFLOP/s")
    calib = copy_calibration()
    vendor = vendor_gemv(2 * f, d)
    log(f"library GEMV (torch.mv, {2 * f}x{d} bf16): {vendor['gbs']:.0f} GB/s")
    ceiling = read_ceiling(swiglu_bytes)
    log(f"streaming read of {swiglu_bytes} B regions: {ceiling['gbs']:.0f} GB/s")
    log("timing remap of the whole pool")
    remap = time_remap(cl, args.remap_reps)
    log(f"remap {remap['gbs']:.0f} GB/s vs device copy {remap['memcpy_gbs']:.0f} GB/s")
    remap["uniform"] = time_uniform_remap(C, shapes, cfg, args.remap_reps)
    log(f"uniform remap {remap['uniform']['ms']:.2f} ms, {remap['uniform']['gbs']:.0f} GB/s over "
        f"{remap['uniform']['pairs_mean']:.0f} pairs")
    vmm = None
    if args.vmm:
        # the paper's own arrangement: the same cloaked layout with its pages
        # mapped into a virtual range by the MMU, kernels untranslated
        try:
            log("uploading 16 copies into the hardware-translated (VMM) twin")
            hw = Variant(C, shapes, weights, cfg, 0, seed=1, vmm=True)
        except C.CloakError as e:
            log(f"no VMM twin: {e}")
            hw = None
        if hw is not None:
            v_ms, _ = time_steps(hw, 1, args.steps, args.warmup)
            vmm = {"decode": {"1": dict(gbs=step_bytes / v_ms / 1e6, ms=v_ms, ratio_to_native=ms_nat / v_ms,
                                        ratio_to_software=ms / v_ms)}}
            for M in [int(m) for m in args.batches.split(",") if m]:
                b = sum(layer_bytes(cfg, M))
                m_hw, _ = time_steps(hw, M, max(args.steps // 4, 10), args.warmup)
                vmm["decode"][str(M)] = dict(gbs=b / m_hw / 1e6, ms=m_hw)
            if pm > 0:
                h_ms, _ = time_prefill(hw, pm, max(args.steps // 20, 5), 2)
                vmm["prefill"] = dict(tflops=layer_flops(cfg, pm) / h_ms / 1e9, ms=h_ms)
            vmm["remap"] = time_remap(hw, max(1, args.remap_reps // 2), with_copy=False)
            vmm["swiglu_kernel_ms"] = time_swiglu_loop(hw, 1, max(args.steps, 64))
            log(f"VMM twin: M=1 {vmm['decode']['1']['gbs']:.0f} GB/s, remap {vmm['remap']['ms']:.1f} ms on the "
                f"stream / {vmm['remap']['wall_ms']:.1f} ms wall")
            hw.cw.close()

    hard = None
    if args.hardened:
        one_h = synth.decoder_layer_shapes(d, f, kv, "bf16", layer=0, head_dim=128)
        hshapes = [(l,) + tuple(s[1:]) for l in range(COPIES) for s in one_h]
        log("uploading 16 hardened copies")
        hv = Variant(C, hshapes, weights, cfg, C.CLOAK_CSPRNG | C.CLOAK_MASKED_MAP, seed=1, decoy=True, stored=True)
        h_ms, _ = time_steps(hv, 1, args.steps, args.warmup)
        hard = {"decode": {"1": dict(gbs=step_bytes / h_ms / 1e6, ms=h_ms, ratio_to_cloaked=ms / h_ms)}}
        for M in [int(m) for m in args.batches.split(",") if m]:
            b = sum(layer_bytes(cfg, M))
            m_h, _ = time_steps(hv, M, max(args.steps // 4, 10), args.warmup)
            hard["decode"][str(M)] = dict(gbs=b / m_h / 1e6, ms=m_h, ratio_to_cloaked=decode[str(M)]["ms"] / m_h)
        if pm > 0:
            h_pms, _ = time_prefill(hv, pm, max(args.steps // 20, 5), 2)
            hard["prefill"] = dict(tflops=layer_flops(cfg, pm) / h_pms / 1e9, ms=h_pms,
                                   ratio_to_cloaked=prefill["ms"] / h_pms)
        hard["swiglu_kernel_ms"] = time_swiglu_loop(hv, 1, max(args.steps, 64))
        log(f"hardened: M=1 {hard['decode']['1']['gbs']:.0f} GB/s")
        hv.cw.close()

    achieved = swiglu_bytes / k_ms / 1e6
    digest = kernel_sources_digest()
    traffic = None
    if SWIGLU_COUNTERS["sources"] == digest:
        traffic = SWIGLU_COUNTERS["fetch_bytes"] + SWIGLU_COUNTERS["write_bytes"]
    roofline = dict(kernel="gemv_kernel SwiGLU (gate+up, bf16, M=1)", bound="hbm", achieved=achieved,
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                    bytes_per_launch=swiglu_bytes, avg_launch_ms=k_ms, native_avg_launch_ms=k_ms_nat,
                    kernel_sources=digest, read_ceiling_gbs=ceiling["gbs"],
                    frac_of_read_ceiling=achieved / ceiling["gbs"])

    clocks_after = gpu_clocks()
    contiguity = C.cloak_query(cl.cw.layout, "CONTIGUITY")
    for v in (cl, nat, ident):
        v.cw.close()
    del cl, nat, ident
    torch.cuda.empty_cache()

    serving = None
    if args.serve_requests > 0:
        from paper_2606_18400_amd import serve
        log(f"short serving pass: {args.serve_requests} requests at {args.serve_rate} req/s, cloaked and native")
        sres = serve_variants(serve_weights(), [args.serve_rate], args.serve_requests)
        key = str(float(args.serve_rate))
        keys = ("ttft_ms_p50", "ttft_ms_p99", "tpot_ms_p50", "tpot_ms_p99", "itl_ms_p50", "itl_ms_p99",
                "output_tok_per_s", "steps", "remaps", "completed")
        serving = {"rate_req_s": args.serve_rate, "requests": args.serve_requests,
                   "workload": "32-layer 4096/14336/1024 BF16 stack, vocab 128256, Poisson arrivals, prompts "
                               "U[128,4096], outputs U[64,1024], remap every 256 steps (cloaked)"}
        for name in ("cloaked", "native"):
            serving[name] = {k: sres[name][key][k] for k in keys}
        serving["tpot_p50_ratio"] = serving["native"]["tpot_ms_p50"] / serving["cloaked"]["tpot_ms_p50"]

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_oracle_baseline(cfg, w1)

    out = {
        "metric": METRIC, "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "decode M=1 through one 4096/14336/1024 BF16 decoder layer (q,k,v,o,gate,up,"
                               "down), 2 MiB pages scattered over an 8 GiB pool, 16 layer copies cycled",
                   "layout_seed": 1, "pages": 4096, "used_pages": 16 * 208},
        "cloaked_native_ratio": value / native,
        "decode": decode,
        "prefill": prefill,
        "remap": remap,
        "vmm_twin": vmm,
        "hardened": hard,
        "copy_calibration": calib,
        "vendor_gemv": vendor,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "contiguity": contiguity,
        "serving": serving,
        "gpu_clocks": {"before": clocks_before, "after": clocks_after},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

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

    def __init__(self, C, shapes, weights, cfg, flags, seed):
        self.cw = C.CloakedWeights(shapes, cfg["page_bytes"], cfg["pool_bytes"], seed=seed, flags=flags)
        self.cw.load(weights)
        self.C = C
        self.cfg = cfg

    def buffers(self, M):
        import torch
        from paper_2606_18400_amd import synth
        d, f, kv = self.cfg["d_model"], self.cfg["d_ffn"], self.cfg["d_kv"]
        x = torch.from_numpy(synth.activations(M, d, "bf16").view(np.int16)).cuda().view(torch.bfloat16)
        return dict(x=x,
                    qkv=torch.empty((M, d + 2 * kv), dtype=torch.bfloat16, device="cuda"),
                    o=torch.empty((M, d), dtype=torch.bfloat16, device="cuda"),
                    h=torch.empty((M, f), dtype=torch.bfloat16, device="cuda"),
                    y=torch.empty((M, d), dtype=torch.bfloat16, device="cuda"))

    def step(self, i, M, b, ev=None):
        C, cw = self.C, self.cw
        L, pool = cw.layout, cw.pool
        l = i % COPIES
        t0 = TENSORS_PER_LAYER * l
        C.cloak_linear_fused(L, pool, [t0, t0 + 1, t0 + 2], b["x"], M, b["qkv"])
        C.cloak_linear(L, pool, t0 + 3, b["x"], M, b["o"])
        if ev is not None:
            ev[0].record()
        C.cloak_swiglu(L, pool, l, b["x"], M, b["h"])
        if ev is not None:
            ev[1].record()
        C.cloak_down(L, pool, l, b["h"], M, b["y"])


def time_steps(var, M, steps, warmup, kernel_events=False):
    import torch
    b = var.buffers(M)
    for i in range(warmup):
        var.step(i, M, b)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)] if kernel_events else None
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for i in range(steps):
        var.step(i, M, b, evs[i] if evs else None)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    kms = None
    if evs:
        kms = float(np.mean([a.elapsed_time(z) for a, z in evs]))
    return ms, kms


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


def time_remap(var, reps):
    import torch
    pool_bytes = var.cfg["pool_bytes"]
    var.cw.remap(1000)   # warm
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for r in range(reps):
        var.cw.remap(1001 + r)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
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


def cpu_oracle_baseline(cfg, weights, budget_s=12.0):
    """The oracle's FP64 decode step (decode stored weights, then the products)."""
    from oracle import numerics as ON
    from paper_2606_18400_amd import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    d = cfg["d_model"]
    x = ON.bf16_bits_to_f64(synth.activations(1, d, "bf16"))
    step_bytes = sum(layer_bytes(cfg, 1))
    steps, t0 = 0, time.perf_counter()
    while True:
        w = [ON.weights_f64(weights[t], "bf16") for t in range(TENSORS_PER_LAYER)]
        for t in range(4):
            ON.linear(x, w[t])
        ON.swiglu_ffn(x, w[4], w[5], w[6])
        del w
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 20:
            break
    return dict(value=step_bytes * steps / el / 1e9, unit="GB/s", cores=int(threads), kind="oracle",
                sample=f"{steps} decode steps (M=1) of one 4096/14336 BF16 layer: bf16->FP64 weight decode "
                       f"plus FP64 products, {el:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--batches", default="8,32,64", help="extra decode batch sizes reported beside M=1")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--remap-reps", type=int, default=5)
    ap.add_argument("--prefill-tokens", type=int, default=8192, help="prefill batch (0 skips the prefill pass)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the cloaked layer needs no "
              "cross-GPU exchange, see the sharding notes in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2606_18400_amd import cloak as C
    from paper_2606_18400_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
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

    step_bytes = sum(layer_bytes(cfg, 1))
    swiglu_bytes = layer_bytes(cfg, 1)[2]
    log(f"timing M=1: {args.warmup} warmup + {args.steps} steps")
    ms, k_ms = time_steps(cl, 1, args.steps, args.warmup, kernel_events=True)
    ms_nat, k_ms_nat = time_steps(nat, 1, args.steps, args.warmup, kernel_events=True)
    value = step_bytes / ms / 1e6
    native = step_bytes / ms_nat / 1e6
    log(f"M=1 cloaked {value:.0f} GB/s native {native:.0f} GB/s")
    decode = {"1": dict(cloaked_gbs=value, native_gbs=native, ratio=value / native, ms=ms, native_ms=ms_nat)}
    for M in [int(m) for m in args.batches.split(",") if m]:
        b = sum(layer_bytes(cfg, M))
        m_cl, _ = time_steps(cl, M, max(args.steps // 4, 10), args.warmup)
        m_nat, _ = time_steps(nat, M, max(args.steps // 4, 10), args.warmup)
        decode[str(M)] = dict(cloaked_gbs=b / m_cl / 1e6, native_gbs=b / m_nat / 1e6, ratio=m_nat / m_cl,
                              ms=m_cl, native_ms=m_nat)
        log(f"M={M} cloaked {b / m_cl / 1e6:.0f} GB/s native {b / m_nat / 1e6:.0f} GB/s")

    pm = args.prefill_tokens
    prefill = None
    if pm > 0:
        log(f"timing prefill M={pm}")
        p_ms, p_kms = time_prefill(cl, pm, max(args.steps // 20, 5), 2)
        n_ms, n_kms = time_prefill(nat, pm, max(args.steps // 20, 5), 2)
        fl = layer_flops(cfg, pm)
        sw_fl = 2 * pm * 2 * f * d
        prefill = dict(tokens=pm, cloaked_tflops=fl / p_ms / 1e9, native_tflops=fl / n_ms / 1e9,
                       ratio=n_ms / p_ms, ms=p_ms, native_ms=n_ms,
                       roofline=dict(kernel="gemm_kernel SwiGLU (gate+up, bf16 MFMA)", bound="mfma",
                                     achieved=sw_fl / p_kms / 1e9, peak=MFMA_BF16_PEAK_TFLOPS, unit="TFLOP/s",
                                     frac=sw_fl / p_kms / 1e9 / MFMA_BF16_PEAK_TFLOPS, flops_per_launch=sw_fl,
                                     avg_launch_ms=p_kms, native_avg_launch_ms=n_kms))
        log(f"prefill cloaked {fl / p_ms / 1e9:.0f} TFLOP/s native {fl / n_ms / 1e9:.0f} TFLOP/s")
    calib = copy_calibration()
    log("timing remap of the whole pool")
    remap = time_remap(cl, args.remap_reps)
    log(f"remap {remap['gbs']:.0f} GB/s vs device copy {remap['memcpy_gbs']:.0f} GB/s")

    achieved = swiglu_bytes / k_ms / 1e6
    roofline = dict(kernel="gemv_kernel SwiGLU (gate+up, bf16, M=1)", bound="hbm", achieved=achieved,
                    peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS, traffic=None,
                    bytes_per_launch=swiglu_bytes, avg_launch_ms=k_ms, native_avg_launch_ms=k_ms_nat)

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
        "copy_calibration": calib,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "contiguity": C.cloak_query(cl.cw.layout, "CONTIGUITY"),
    }
    print(json.dumps(out), flush=True)
    cl.cw.close()
    nat.cw.close()


if __name__ == "__main__":
    main()

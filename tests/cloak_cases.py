"""Shared builders for the GPU parity tests (inputs only; no method arithmetic).

Everything device-side goes through the C-ABI binding; the expected values
come from ``oracle/`` on the same seeded inputs.
"""

import numpy as np

from oracle import layout as OL
from oracle import numerics as ON
from paper_2606_18400_amd import synth

TOL = {"f32": 1e-5, "bf16": 1e-2, "fp8": 5e-2}


def make_weights(shapes, base_seed=1234):
    ws, scs = [], []
    for t, s in enumerate(shapes):
        w, sc = synth.weight(t, s[2], s[3], s[4], base_seed=base_seed)
        ws.append(w)
        scs.append(sc)
    return ws, scs


def oracle_layout(seed, shapes, page_bytes, pool_bytes, identity=False):
    return OL.build_layout(seed, [OL.Shape(*s) for s in shapes], page_bytes, pool_bytes, identity=identity)


def w64(shapes, ws, scs, t):
    return ON.weights_f64(ws[t], shapes[t][4], scs[t])


def to_device_x(x_np):
    import torch
    if x_np.dtype == np.float32:
        return torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    return torch.from_numpy(np.ascontiguousarray(x_np).view(np.int16)).cuda().view(torch.bfloat16)


def from_device(y):
    import torch
    if y.dtype == torch.float32:
        return y.cpu().numpy()
    return y.view(torch.int16).cpu().numpy().view(np.uint16)


def values_f64(arr):
    if arr.dtype == np.float32:
        return arr.astype(np.float64)
    return ON.bf16_bits_to_f64(arr)


def act_dtype(wdtype):
    return "f32" if wdtype == "f32" else "bf16"


def decoder_shapes(d, ffn, dkv, dtype, layers=1, extra=(), head_dim=0):
    shapes = []
    for l in range(layers):
        shapes += synth.decoder_layer_shapes(d, ffn, dkv, dtype, layer=l, head_dim=head_dim)
    return shapes + list(extra)

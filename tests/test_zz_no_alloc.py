"""cloak_mlp_noalloc (the FFN for callers that cannot allocate) against cloak_mlp.

Both run the same kernels, so the results must be bit-identical; the FP64
oracle checks the values too.  Each case makes two calls in a row on the one
static workspace, the second with fewer tokens, so stale bytes of the first
call are still in the array when the second runs.
"""

import numpy as np
import pytest

from cloak_cases import TOL, decoder_shapes, from_device, make_weights, to_device_x, values_f64, w64
from oracle import numerics as ON
from paper_2606_18400_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    import torch
    assert torch.cuda.is_available()
    from paper_2606_18400_amd import cloak
    return cloak


def oracle_mlp(shapes, ws, scs, layer, x_np):
    ig = next(t for t, s in enumerate(shapes) if s[0] == layer and s[1] == "gate")
    iu = next(t for t, s in enumerate(shapes) if s[0] == layer and s[1] == "up")
    idn = next(t for t, s in enumerate(shapes) if s[0] == layer and s[1] == "down")
    y, _ = ON.swiglu_ffn(values_f64(x_np), w64(shapes, ws, scs, ig), w64(shapes, ws, scs, iu),
                         w64(shapes, ws, scs, idn))
    return y


@pytest.mark.parametrize("dtype,d,ffn,calls", [
    ("bf16", 1024, 2816, (200, 5)),      # LDS-ring skinny tiles, then the split-K 16-token tile
    ("bf16", 1024, 2816, (64, 1)),       # split-K partials, then the GEMV (no partials)
    ("fp8", 1024, 2816, (128, 3)),
    ("bf16", 4096, 14336, (256, 8)),     # the full-size layer near the top of the range
])
def test_noalloc_matches_cloak_mlp(C, dtype, d, ffn, calls):
    import torch
    shapes = decoder_shapes(d, ffn, d // 4, dtype, layers=2)
    B = 2 << 20
    ws, scs = make_weights(shapes)
    need = sum(-(-s[2] * s[3] * (1 if dtype == "fp8" else 2) // B) for s in shapes)
    cw = C.CloakedWeights(shapes, B, B * (need + 16), seed=21)
    cw.load(ws, scs)
    for k, M in enumerate(calls):
        layer = k % 2
        print(f"noalloc case dtype={dtype} d={d} ffn={ffn} M={M} layer={layer}", flush=True)
        x_np = synth.activations(M, d, "bf16", seed=900 + k)
        x = to_device_x(x_np)
        y_ref = cw.mlp(layer, x)
        y = torch.empty_like(x)
        C.cloak_mlp_noalloc(cw.layout, cw.pool, layer, x, M, y)
        torch.cuda.synchronize()
        assert torch.equal(y.view(torch.int16), y_ref.view(torch.int16)), (dtype, M)
        err = ON.normwise_err(values_f64(from_device(y)), oracle_mlp(shapes, ws, scs, layer, x_np))
        assert err <= TOL[dtype], (dtype, M, err)
    cw.close()


def test_noalloc_refuses_calls_beyond_its_array(C):
    import torch
    shapes = decoder_shapes(1024, 2816, 256, "bf16")
    B = 2 << 20
    ws, scs = make_weights(shapes)
    cw = C.CloakedWeights(shapes, B, B * 32, seed=5)
    cw.load(ws, scs)
    M = 16384   # h alone is 92 MB, above the 64 MiB array
    assert C.cloak_mlp_ws_bytes(cw.layout, 0, M) > 64 << 20
    x = torch.zeros((M, 1024), dtype=torch.bfloat16, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(C.CloakError) as e:
        C.cloak_mlp_noalloc(cw.layout, cw.pool, 0, x, M, y)
    assert e.value.code == C.CLOAK_EINVAL and "static" in C.cloak_last_error()
    torch.cuda.synchronize()
    assert not y.any().item()
    # M = 0 is a no-op, as for cloak_mlp
    C.cloak_mlp_noalloc(cw.layout, cw.pool, 0, x, 0, y)
    cw.close()

"""Mixture-of-experts FFN on cloaked expert tensors (oracle).

The paper serves a Qwen 3 MoE model (Section 5 setup) but describes the
defence per tensor; nothing in it is specific to experts.  Reading: every
expert is its own SwiGLU FFN -- gate, up and down tensors with their own
hidden-neuron permutation, placed like any other tensor by the tensor-order
shuffle -- and a MoE layer's output for token m is the router-weighted sum of
its chosen experts' outputs,

    y[m] = sum_j  w[m][j] * FFN_{e[m][j]}(x[m])      over the top-k slots j,

with FFN_e(x) = down_e(silu(gate_e x) * (up_e x)) on logical weights.  Slots
whose expert id lies outside [0, E) contribute nothing.  Routing itself (the
router projection and the top-k choice) is an ordinary dense step outside
the cloaked path; ids and weights are inputs here.
"""

import numpy as np

from . import numerics as N


def moe_ffn(x64, ids, wts, experts):
    """x64 [M][d] FP64; ids [M][k] int; wts [M][k]; experts: list of
    (gate [F][d], up [F][d], down [d][F]) logical FP64 arrays.  Returns y [M][d]."""
    x64 = np.asarray(x64, np.float64)
    ids = np.asarray(ids)
    wts = np.asarray(wts, np.float64)
    M, d = x64.shape
    y = np.zeros((M, d))
    for m in range(M):
        for j in range(ids.shape[1]):
            e = int(ids[m, j])
            if not 0 <= e < len(experts):
                continue
            g, u, dn = experts[e]
            out, _ = N.swiglu_ffn(x64[m:m + 1], g, u, dn)
            y[m] += wts[m, j] * out[0]
    return y

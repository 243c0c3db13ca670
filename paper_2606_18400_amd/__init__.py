"""CloakLM's cloaked linear layer, native to AMD MI355X (gfx950).

Weights are hidden-neuron shuffled (intra-layer), tensor-order shuffled
(inter-layer) and cut into pages scattered over a device pool through a
seeded page map; hand-written HIP kernels translate virtual tiles to physical
pages while they stream the weights, and a remap kernel re-randomises the
placement in place (CloakLM, arXiv 2606.18400, Section 4.2).

``paper_2606_18400_amd.cloak`` is the thin ctypes binding of the C-ABI
library ``libcloak.so`` (declared in ``include/cloak.h``); importing it fails
loudly when the library has not been built.  ``synth`` holds the seeded input
generators, ``serve`` the continuous-batching serving loop.
"""

import importlib

__all__ = ["cloak", "synth", "serve", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)

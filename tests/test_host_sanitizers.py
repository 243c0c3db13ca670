"""The library's host C++ (layout, queries, host images, remaps, SHA-256) under
AddressSanitizer and UndefinedBehaviorSanitizer.

host_sanitize_driver.c calls every host-only entry point, including error
paths, against layout.cpp and sha256.cpp built with -fsanitize=address,undefined
(g++, no HIP code involved).  The run must report no sanitizer finding, and its
page-map and pool-image digests must equal those of the normal library on the
same inputs (replayed here through the ctypes binding).
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2606_18400_amd import cloak as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_18400_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def fnv(data):
    """FNV-1a over little-endian 64-bit words, as the driver computes it."""
    h = 1469598103934665603
    data = data + bytes(-len(data) % 8)      # a short last word is zero padded
    for w in np.frombuffer(data, dtype="<u8").tolist():
        h = ((h ^ w) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def model_shapes(dtype, head_dim):
    nk = [(256, 256), (64, 256), (64, 256), (256, 256), (384, 256), (384, 256), (256, 384)]
    kinds = ["q", "k", "v", "o", "gate", "up", "down"]
    s = []
    for l in range(2):
        for k, (n, kk) in zip(kinds, nk):
            s.append((l, k, n, kk, dtype, head_dim if k in ("q", "k", "v", "o") else 0))
    return s + [(-1, "embed", 100, 256, dtype, 0), (-1, "head", 100, 256, dtype, 0)]


def replay(flags, dtype, head_dim, page_bytes, P, slice_pairs):
    shapes = model_shapes(dtype, head_dim)
    L = C.cloak_layout_build(0xC10A4, shapes, page_bytes, page_bytes * P, flags)
    pool = np.zeros(page_bytes * P, np.uint8)
    elt = {"f32": 4, "bf16": 2, "fp8": 1}[dtype]
    npdt = {"f32": np.uint32, "bf16": np.uint16, "fp8": np.uint8}[dtype]
    for t, s in enumerate(shapes):
        nbytes = s[2] * s[3] * elt
        w = ((np.arange(nbytes, dtype=np.uint64) * 131 + t * 7 + 1) & 255).astype(np.uint8)
        C.cloak_pack_host(L, t, w.view(npdt).reshape(s[2], s[3]), pool)
    if not flags & C.CLOAK_IDENTITY:
        C.cloak_pool_decoy_host(L, pool, 77)
        C.cloak_remap_host(L, pool, 5)
        C.cloak_remap_begin(L, 6)
        while C.cloak_remap_step_host(L, pool, slice_pairs) > 0:
            pass
    phi = np.asarray(C.cloak_query(L, "PHI"), np.int32)
    v = C.cloak_query(L, "V")
    C.cloak_layout_free(L)
    return v, fnv(phi.tobytes()), fnv(pool.tobytes())


@pytest.mark.slow
def test_host_code_under_asan_and_ubsan(tmp_path):
    gxx, gcc = shutil.which("g++"), shutil.which("gcc")
    if not gxx or not gcc:
        pytest.skip("no host compiler")
    inc = ["-I", os.path.join(ROOT, "include")]
    objs = []
    for src in ("layout.cpp", "sha256.cpp"):
        obj = str(tmp_path / (src + ".o"))
        subprocess.run([gxx, "-std=c++17", *SAN, *inc, "-c", os.path.join(CSRC, src), "-o", obj], check=True)
        objs.append(obj)
    drv = str(tmp_path / "driver.o")
    subprocess.run([gcc, "-std=c99", *SAN, *inc, "-c", os.path.join(ROOT, "tests", "host_sanitize_driver.c"), "-o",
                    drv], check=True)
    exe = str(tmp_path / "driver")
    subprocess.run([gxx, *SAN, drv, *objs, "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    env.pop("LD_PRELOAD", None) if "libasan" in env.get("LD_PRELOAD", "") else None
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.returncode, r.stderr[-4000:])
    lines = [l for l in r.stdout.splitlines() if l.startswith("case")]
    assert len(lines) == 5 and "errors ok=1" in r.stdout
    dt = {0: "f32", 1: "bf16", 2: "fp8"}
    for line in lines:
        f = dict(kv.split("=") for kv in line.split()[1:])
        v, hphi, hpool = replay(int(f["flags"]), dt[int(f["dtype"])], int(f["head_dim"]), int(f["page"]),
                                int(f["P"]), int(f["slice"]))
        assert int(f["V"]) == v, line
        assert int(f["phi"], 16) == hphi, line
        assert int(f["pool"], 16) == hpool, line

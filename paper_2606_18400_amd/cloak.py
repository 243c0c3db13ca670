"""ctypes binding of libcloak (include/cloak.h): argument marshalling only.

Every function here has the name and meaning of the C entry point it wraps;
all of the work happens in the library (host layout code and HIP kernels).
Device buffers may be passed as torch tensors (their ``data_ptr()`` is used)
or as raw integer addresses; host buffers are NumPy arrays.  ``stream=None``
means torch's current stream on the current device.

Importing this module fails loudly when ``libcloak.so`` has not been built;
there is no fallback of any kind.
"""

import ctypes
import os

import numpy as np

# PyTorch ships its own HIP runtime (same SONAME as /opt/rocm's).  It must be
# loaded before libcloak so that the library binds to that one runtime:
# device pointers and streams handed over from torch are only valid there.
import torch  # noqa: F401,E402

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcloak.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2606_18400_amd.build` "
        "(or __graft_entry__.build()); the cloaked path has no fallback")
_lib = ctypes.CDLL(LIB_PATH)

# ---------------------------------------------------------------- constants
CLOAK_OK, CLOAK_EINVAL, CLOAK_ENOMEM, CLOAK_EHIP, CLOAK_ESHAPE, CLOAK_EDTYPE, CLOAK_ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESHAPE", -5: "EDTYPE", -6: "ESTATE"}
DTYPES = {"f32": 0, "bf16": 1, "fp8": 2}
KINDS = {"q": 0, "k": 1, "v": 2, "o": 3, "gate": 4, "up": 5, "down": 6, "embed": 7, "head": 8}
CLOAK_IDENTITY = 1
CLOAK_NATIVE = 2
CLOAK_CSPRNG = 4
CLOAK_MASKED_MAP = 8
CLOAK_REMAP_UNIFORM = 16
QUERY = dict(P=1, V=2, T=3, PAGE_BYTES=4, PHI=5, SIGMA=6, PI=7, VBASE=8, NPAGES=9, CONTIGUITY=10,
             UPLOAD_ORDER=11, REMAPS=12, TENSOR=13, DFFN=14, REMAP_PENDING=15, ROW_PERM=16, COL_PERM=17,
             SHAPE=18, MAP_KEY=19)
CLOAK_OP_LINEAR, CLOAK_OP_MLP, CLOAK_OP_SWIGLU, CLOAK_OP_DOWN = 1, 2, 3, 4
STORAGE = {"f32": np.float32, "bf16": np.uint16, "fp8": np.uint8}


class cloak_shape(ctypes.Structure):
    _fields_ = [("layer", ctypes.c_int32), ("kind", ctypes.c_int32), ("n_out", ctypes.c_int64),
                ("k_in", ctypes.c_int64), ("dtype", ctypes.c_int32), ("head_dim", ctypes.c_int32)]


class CloakError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__(f"{fn} failed with {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class cloak_model_config(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("d_model", ctypes.c_int32), ("n_heads", ctypes.c_int32),
                ("n_kv_heads", ctypes.c_int32), ("head_dim", ctypes.c_int32), ("d_ffn", ctypes.c_int32),
                ("vocab", ctypes.c_int32), ("block_size", ctypes.c_int32), ("num_blocks", ctypes.c_int64),
                ("rope_theta", ctypes.c_float), ("norm_eps", ctypes.c_float)]


class cloak_step(ctypes.Structure):
    _fields_ = [("n_tokens", ctypes.c_int32), ("n_seqs", ctypes.c_int32), ("max_blocks", ctypes.c_int32),
                ("n_logits", ctypes.c_int32), ("n_tiles", ctypes.c_int32), ("n_splits", ctypes.c_int32),
                ("split_keys", ctypes.c_int32), ("n_single", ctypes.c_int32),
                ("d_tokens", ctypes.c_void_p), ("d_positions", ctypes.c_void_p), ("d_tok_seq", ctypes.c_void_p),
                ("d_block_table", ctypes.c_void_p), ("d_tile_seq", ctypes.c_void_p),
                ("d_tile_tok0", ctypes.c_void_p), ("d_tile_ntok", ctypes.c_void_p),
                ("d_logit_rows", ctypes.c_void_p), ("d_out_tokens", ctypes.c_void_p),
                ("d_out_logits", ctypes.c_void_p)]


_vp, _i32, _i64, _u64, _u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
_SIGS = {
    "cloak_layout_build": ([_u64, ctypes.POINTER(cloak_shape), _i32, _u64, _u64, _u32, ctypes.POINTER(_vp)], _i32),
    "cloak_layout_free": ([_vp], _i32),
    "cloak_layout_to_device": ([_vp, _vp], _i32),
    "cloak_query": ([_vp, _i32, _i64, _vp, _u64], _i32),
    "cloak_pool_init": ([_vp, _vp, _vp], _i32),
    "cloak_pool_decoy": ([_vp, _vp, _u64, _vp], _i32),
    "cloak_device_map_read": ([_vp, _vp, _vp], _i32),
    "cloak_pool_decoy_host": ([_vp, _vp, _u64, _u64], _i32),
    "cloak_load": ([_vp, _vp, _i32, _vp, _vp, _vp], _i32),
    "cloak_load_all": ([_vp, _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp], _i32),
    "cloak_unload": ([_vp, _vp, _i32, _vp, _vp], _i32),
    "cloak_pack_host": ([_vp, _i32, _vp, _vp, _u64], _i32),
    "cloak_ws_bytes": ([_vp, _i32, _i32, _i64], _u64),
    "cloak_linear_fused_ws_bytes": ([_vp, ctypes.POINTER(_i32), _i32, _i64], _u64),
    "cloak_linear": ([_vp, _vp, _i32, _vp, _i64, _vp, _vp, _u64, _vp], _i32),
    "cloak_linear_fused": ([_vp, _vp, ctypes.POINTER(_i32), _i32, _vp, _i64, _vp, _vp, _u64, _vp], _i32),
    "cloak_linear_stored": ([_vp, _vp, ctypes.POINTER(_i32), _i32, _vp, _i64, _vp, _vp, _u64, _vp], _i32),
    "cloak_mlp": ([_vp, _vp, _i32, _vp, _i64, _vp, _vp, _u64, _vp], _i32),
    "cloak_mlp_ws_bytes": ([_vp, _i32, _i64], _u64),
    "cloak_mlp_noalloc": ([_vp, _vp, _i32, _vp, _i64, _vp, _vp], _i32),
    "cloak_swiglu": ([_vp, _vp, _i32, _vp, _i64, _vp, _vp, _u64, _vp], _i32),
    "cloak_down": ([_vp, _vp, _i32, _vp, _i64, _vp, _vp, _u64, _vp], _i32),
    "cloak_quantize_fp8": ([_vp, _i64, _i64, _i64, _vp, _vp, _vp], _i32),
    "cloak_moe_ws_bytes": ([_vp, _i32, _i32, _i32, _i64], _u64),
    "cloak_stream_read": ([_vp, _u64, _vp, _vp], _i32),
    "cloak_moe": ([_vp, _vp, _i32, _i32, _i32, _vp, _i64, _vp, _vp, _vp, _vp, _u64, _vp], _i32),
    "cloak_remap": ([_vp, _vp, _u64, _vp], _i32),
    "cloak_remap_host": ([_vp, _vp, _u64, _u64], _i32),
    "cloak_remap_begin": ([_vp, _u64], _i32),
    "cloak_vmm_pool_create": ([_vp, ctypes.POINTER(_vp)], _i32),
    "cloak_vmm_pool_free": ([_vp], _i32),
    "cloak_remap_step": ([_vp, _vp, _i64, ctypes.POINTER(_i64), _vp], _i32),
    "cloak_remap_step_host": ([_vp, _vp, _u64, _i64, ctypes.POINTER(_i64)], _i32),
    "cloak_model_create": ([_vp, _vp, ctypes.POINTER(cloak_model_config), _vp, _vp, ctypes.POINTER(_vp)], _i32),
    "cloak_model_free": ([_vp], _i32),
    "cloak_model_ws_bytes": ([_vp, _i64, _i64, _i64, _i64], _u64),
    "cloak_model_step": ([_vp, ctypes.POINTER(cloak_step), _vp, _u64, _vp], _i32),
    "cloak_last_error": ([], ctypes.c_char_p),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes, _f.restype = _args, _res

EXPORTED = tuple(_SIGS)


def cloak_last_error():
    return _lib.cloak_last_error().decode()


def _check(rc, fn):
    if rc != CLOAK_OK:
        raise CloakError(rc, fn, cloak_last_error())


def _ptr(obj):
    if obj is None:
        return None
    if isinstance(obj, int):
        return obj
    if hasattr(obj, "data_ptr"):
        return obj.data_ptr()
    if isinstance(obj, np.ndarray):
        if not obj.flags["C_CONTIGUOUS"]:
            raise ValueError("host arrays must be C-contiguous")
        return obj.ctypes.data
    raise TypeError(f"cannot take the address of {type(obj)}")


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if hasattr(stream, "cuda_stream"):
        return stream.cuda_stream
    return stream


def _shape(s):
    """(layer, kind, n_out, k_in, dtype[, head_dim]) -> cloak_shape."""
    layer, kind, n, k, dtype = s[:5]
    head_dim = int(s[5]) if len(s) > 5 else 0
    return cloak_shape(int(layer), KINDS[kind] if isinstance(kind, str) else int(kind), int(n), int(k),
                       DTYPES[dtype] if isinstance(dtype, str) else int(dtype), head_dim)


# ---------------------------------------------------------------- entry points
def cloak_layout_build(seed, shapes, page_bytes, pool_bytes, flags=0):
    arr = (cloak_shape * len(shapes))(*[_shape(s) for s in shapes])
    out = _vp()
    _check(_lib.cloak_layout_build(seed & ((1 << 64) - 1), arr, len(shapes), page_bytes, pool_bytes, flags,
                                   ctypes.byref(out)), "cloak_layout_build")
    return out.value


def cloak_layout_free(layout):
    _check(_lib.cloak_layout_free(layout), "cloak_layout_free")


def cloak_layout_to_device(layout, stream=None):
    _check(_lib.cloak_layout_to_device(layout, _stream(stream)), "cloak_layout_to_device")


def cloak_query(layout, what, index=0):
    """Returns an int / float, or a NumPy array for the table selectors."""
    q = QUERY[what] if isinstance(what, str) else what
    if q in (QUERY["P"], QUERY["V"], QUERY["T"], QUERY["PAGE_BYTES"], QUERY["REMAPS"], QUERY["TENSOR"],
             QUERY["DFFN"], QUERY["REMAP_PENDING"]):
        v = _i64()
        _check(_lib.cloak_query(layout, q, index, ctypes.byref(v), 8), "cloak_query")
        return v.value
    if q == QUERY["MAP_KEY"]:
        v = ctypes.c_uint64()
        _check(_lib.cloak_query(layout, q, index, ctypes.byref(v), 8), "cloak_query")
        return v.value
    if q == QUERY["CONTIGUITY"]:
        v = ctypes.c_double()
        _check(_lib.cloak_query(layout, q, index, ctypes.byref(v), 8), "cloak_query")
        return v.value
    sizes = {QUERY["PHI"]: lambda: cloak_query(layout, "P"),
         QUERY["SIGMA"]: lambda: cloak_query(layout, "T"),
         QUERY["VBASE"]: lambda: cloak_query(layout, "T"),
         QUERY["NPAGES"]: lambda: cloak_query(layout, "T"),
         QUERY["UPLOAD_ORDER"]: lambda: int(cloak_query(layout, "NPAGES")[index]),
         QUERY["PI"]: lambda: cloak_query(layout, "DFFN", index),
         QUERY["ROW_PERM"]: lambda: int(cloak_query(layout, "SHAPE", index)[0]),
         QUERY["COL_PERM"]: lambda: int(cloak_query(layout, "SHAPE", index)[1]),
         QUERY["SHAPE"]: lambda: 4}
    if q not in sizes:
        v = _i64()   # unknown selector: let the library report it
        _check(_lib.cloak_query(layout, q, index, ctypes.byref(v), 8), "cloak_query")
        return v.value
    n = sizes[q]()
    dtype = np.int64 if q in (QUERY["VBASE"], QUERY["NPAGES"], QUERY["SHAPE"]) else np.int32
    out = np.zeros(n, dtype=dtype)
    _check(_lib.cloak_query(layout, q, index, out.ctypes.data, out.nbytes), "cloak_query")
    return out


def cloak_pool_init(layout, pool, stream=None):
    _check(_lib.cloak_pool_init(layout, _ptr(pool), _stream(stream)), "cloak_pool_init")


def cloak_device_map_read(layout, stream=None):
    """The device page-map table as stored (uint32 entries)."""
    out = np.zeros(cloak_query(layout, "P"), dtype=np.int32)
    _check(_lib.cloak_device_map_read(layout, out.ctypes.data, _stream(stream)), "cloak_device_map_read")
    return out.view(np.uint32)


def cloak_pool_decoy(layout, pool, decoy_seed, stream=None):
    _check(_lib.cloak_pool_decoy(layout, _ptr(pool), decoy_seed & ((1 << 64) - 1), _stream(stream)),
           "cloak_pool_decoy")


def cloak_pool_decoy_host(layout, pool_image, decoy_seed):
    _check(_lib.cloak_pool_decoy_host(layout, pool_image.ctypes.data, pool_image.nbytes,
                                      decoy_seed & ((1 << 64) - 1)), "cloak_pool_decoy_host")


def cloak_load(layout, pool, tensor, src, scales=None, stream=None):
    src = np.ascontiguousarray(src)
    sc = None if scales is None else np.ascontiguousarray(scales, dtype=np.float32)
    _check(_lib.cloak_load(layout, _ptr(pool), tensor, src.ctypes.data, None if sc is None else sc.ctypes.data,
                           _stream(stream)), "cloak_load")


def cloak_load_all(layout, pool, weights, scales=None, stream=None):
    """Every tensor; the library sends them in the layout's tensor order."""
    srcs = [np.ascontiguousarray(w) for w in weights]
    scs = None if scales is None else [None if s is None else np.ascontiguousarray(s, dtype=np.float32)
                                       for s in scales]
    src_tab = (_vp * len(srcs))(*[a.ctypes.data for a in srcs])
    sc_tab = None if scs is None else (_vp * len(scs))(*[None if a is None else a.ctypes.data for a in scs])
    _check(_lib.cloak_load_all(layout, _ptr(pool), src_tab, sc_tab, _stream(stream)), "cloak_load_all")


def cloak_unload(layout, pool, tensor, dst, stream=None):
    _check(_lib.cloak_unload(layout, _ptr(pool), tensor, _ptr(dst), _stream(stream)), "cloak_unload")


def cloak_pack_host(layout, tensor, src, pool_image):
    src = np.ascontiguousarray(src)
    _check(_lib.cloak_pack_host(layout, tensor, src.ctypes.data, _ptr(pool_image), pool_image.nbytes),
           "cloak_pack_host")


def cloak_mlp_ws_bytes(layout, layer, M):
    v = _lib.cloak_mlp_ws_bytes(layout, layer, M)
    if v == (1 << 64) - 1:
        raise CloakError(CLOAK_EINVAL, "cloak_mlp_ws_bytes", "bad arguments")
    return v


def cloak_ws_bytes(layout, op, index, M):
    v = _lib.cloak_ws_bytes(layout, op, index, M)
    if v == (1 << 64) - 1:
        raise CloakError(CLOAK_EINVAL, "cloak_ws_bytes", "bad arguments")
    return v


def cloak_linear_fused_ws_bytes(layout, tensors, M):
    arr = (_i32 * len(tensors))(*tensors)
    v = _lib.cloak_linear_fused_ws_bytes(layout, arr, len(tensors), M)
    if v == (1 << 64) - 1:
        raise CloakError(CLOAK_EINVAL, "cloak_linear_fused_ws_bytes", cloak_last_error() or "bad arguments")
    return v


def cloak_linear(layout, pool, tensor, x, M, y, ws=None, ws_bytes=0, stream=None):
    _check(_lib.cloak_linear(layout, _ptr(pool), tensor, _ptr(x), M, _ptr(y), _ptr(ws), ws_bytes,
                             _stream(stream)), "cloak_linear")


def cloak_linear_fused(layout, pool, tensors, x, M, y, ws=None, ws_bytes=0, stream=None):
    arr = (_i32 * len(tensors))(*tensors)
    _check(_lib.cloak_linear_fused(layout, _ptr(pool), arr, len(tensors), _ptr(x), M, _ptr(y), _ptr(ws),
                                   ws_bytes, _stream(stream)), "cloak_linear_fused")


def cloak_linear_stored(layout, pool, tensors, x, M, y, ws=None, ws_bytes=0, stream=None):
    arr = (_i32 * len(tensors))(*tensors)
    _check(_lib.cloak_linear_stored(layout, _ptr(pool), arr, len(tensors), _ptr(x), M, _ptr(y), _ptr(ws),
                                    ws_bytes, _stream(stream)), "cloak_linear_stored")


def cloak_mlp(layout, pool, layer, x, M, y, ws, ws_bytes, stream=None):
    _check(_lib.cloak_mlp(layout, _ptr(pool), layer, _ptr(x), M, _ptr(y), _ptr(ws), ws_bytes, _stream(stream)),
           "cloak_mlp")


def cloak_mlp_noalloc(layout, pool, layer, x, M, y, stream=None):
    _check(_lib.cloak_mlp_noalloc(layout, _ptr(pool), layer, _ptr(x), M, _ptr(y), _stream(stream)),
           "cloak_mlp_noalloc")


def cloak_swiglu(layout, pool, layer, x, M, h, ws=None, ws_bytes=0, stream=None):
    _check(_lib.cloak_swiglu(layout, _ptr(pool), layer, _ptr(x), M, _ptr(h), _ptr(ws), ws_bytes, _stream(stream)),
           "cloak_swiglu")


def cloak_down(layout, pool, layer, h, M, y, ws=None, ws_bytes=0, stream=None):
    _check(_lib.cloak_down(layout, _ptr(pool), layer, _ptr(h), M, _ptr(y), _ptr(ws), ws_bytes, _stream(stream)),
           "cloak_down")


def cloak_remap(layout, pool, remap_seed, stream=None):
    _check(_lib.cloak_remap(layout, _ptr(pool), remap_seed & ((1 << 64) - 1), _stream(stream)), "cloak_remap")


def cloak_stream_read(src, nbytes, out, stream=None):
    _check(_lib.cloak_stream_read(_ptr(src), nbytes, _ptr(out), _stream(stream)), "cloak_stream_read")


def cloak_moe_ws_bytes(layout, first_layer, n_experts, top_k, M):
    v = _lib.cloak_moe_ws_bytes(layout, first_layer, n_experts, top_k, M)
    if v == (1 << 64) - 1:
        raise CloakError(CLOAK_EINVAL, "cloak_moe_ws_bytes", cloak_last_error() or "bad arguments")
    return v


def cloak_moe(layout, pool, first_layer, n_experts, top_k, x, M, ids, weights, y, ws, ws_bytes, stream=None):
    _check(_lib.cloak_moe(layout, _ptr(pool), first_layer, n_experts, top_k, _ptr(x), M, _ptr(ids), _ptr(weights),
                          _ptr(y), _ptr(ws), ws_bytes, _stream(stream)), "cloak_moe")


def cloak_quantize_fp8(x, M, q, s, stream=None):
    """Per-token E4M3 quantisation of bf16 rows x[M][K] into q [M][K] uint8 and s [M] f32."""
    K = x.shape[-1]
    ldx = x.stride(0) if x.dim() > 1 else K
    _check(_lib.cloak_quantize_fp8(_ptr(x), M, K, ldx, _ptr(q), _ptr(s), _stream(stream)), "cloak_quantize_fp8")


def cloak_vmm_pool_create(layout):
    """Pool view (int device address) of the hardware-translated twin."""
    out = _vp()
    _check(_lib.cloak_vmm_pool_create(layout, ctypes.byref(out)), "cloak_vmm_pool_create")
    return out.value


def cloak_vmm_pool_free(layout):
    _check(_lib.cloak_vmm_pool_free(layout), "cloak_vmm_pool_free")


def cloak_remap_begin(layout, remap_seed):
    _check(_lib.cloak_remap_begin(layout, remap_seed & ((1 << 64) - 1)), "cloak_remap_begin")


def cloak_remap_step(layout, pool, max_pairs=0, stream=None):
    """Swap the next max_pairs pairs of the remap in progress; returns pairs left."""
    left = _i64(0)
    _check(_lib.cloak_remap_step(layout, _ptr(pool), max_pairs, ctypes.byref(left), _stream(stream)),
           "cloak_remap_step")
    return left.value


def cloak_remap_step_host(layout, pool_image, max_pairs=0):
    left = _i64(0)
    _check(_lib.cloak_remap_step_host(layout, _ptr(pool_image), pool_image.nbytes, max_pairs, ctypes.byref(left)),
           "cloak_remap_step_host")
    return left.value


def cloak_remap_host(layout, pool_image, remap_seed):
    _check(_lib.cloak_remap_host(layout, _ptr(pool_image), pool_image.nbytes, remap_seed & ((1 << 64) - 1)),
           "cloak_remap_host")


def cloak_model_create(layout, pool, cfg, gains, kv):
    out = _vp()
    _check(_lib.cloak_model_create(layout, _ptr(pool), ctypes.byref(cfg), _ptr(gains), _ptr(kv), ctypes.byref(out)),
           "cloak_model_create")
    return out.value


def cloak_model_free(model):
    _check(_lib.cloak_model_free(model), "cloak_model_free")


def cloak_model_ws_bytes(model, max_tokens, max_logits, max_tiles, max_splits):
    v = _lib.cloak_model_ws_bytes(model, max_tokens, max_logits, max_tiles, max_splits)
    if v == (1 << 64) - 1:
        raise CloakError(CLOAK_EINVAL, "cloak_model_ws_bytes", "bad arguments")
    return v


def cloak_model_step(model, step, ws, ws_bytes, stream=None):
    _check(_lib.cloak_model_step(model, ctypes.byref(step), _ptr(ws), ws_bytes, _stream(stream)),
           "cloak_model_step")


# ---------------------------------------------------------------- convenience
class CloakedWeights:
    """A layout, its device pool and the tensors loaded into it.

    ``seed=None`` draws the layout seed from the operating system's entropy
    source, as the paper does before deployment; tests pass fixed seeds.
    PyTorch only allocates the pool and workspaces and supplies the stream.
    """

    def __init__(self, shapes, page_bytes, pool_bytes, seed=None, flags=0, vmm=False, decoy=None):
        import torch
        self.shapes = [tuple(s) for s in shapes]
        self.seed = int.from_bytes(os.urandom(8), "little") if seed is None else int(seed)
        self.flags = flags
        self.layout = cloak_layout_build(self.seed, self.shapes, page_bytes, pool_bytes, flags)
        cloak_layout_to_device(self.layout)
        # vmm=True: the library's hardware-translated twin (the pool is an int
        # device address of its pool view); otherwise a caller-owned tensor
        self.vmm = bool(vmm)
        if self.vmm:
            self.pool = cloak_vmm_pool_create(self.layout)
        else:
            self.pool = torch.empty(pool_bytes, dtype=torch.uint8, device="cuda")
        cloak_pool_init(self.layout, self.pool)
        # decoy: None / False leaves free pages zero; True fills them from a
        # fresh os.urandom decoy seed, an int from that seed (never the layout's)
        if decoy is not None and decoy is not False:
            ds = int.from_bytes(os.urandom(8), "little") if decoy is True else int(decoy)
            cloak_pool_decoy(self.layout, self.pool, ds)
        self.page_bytes, self.pool_bytes = page_bytes, pool_bytes
        self._ws = {}

    def index(self, layer, kind):
        return cloak_query(self.layout, "TENSOR", (int(layer) << 8) | KINDS[kind])

    def load(self, weights, scales=None):
        """Upload every tensor; the library keeps the shuffled tensor order (sigma)."""
        cloak_load_all(self.layout, self.pool, weights, scales)

    def workspace(self, nbytes):
        import torch
        nbytes = max(int(nbytes), 256)
        ws = self._ws.get("mlp")
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            self._ws["mlp"] = ws
        return ws

    def linear(self, t, x, out=None):
        import torch
        n = self.shapes[t][2]
        M = x.shape[0]
        if out is None:
            out = torch.empty((M, n), dtype=x.dtype, device=x.device)
        need = cloak_ws_bytes(self.layout, CLOAK_OP_LINEAR, t, M)
        ws = self.workspace(need) if need else None
        cloak_linear(self.layout, self.pool, t, x, M, out, ws, 0 if ws is None else ws.numel())
        return out

    def linear_fused(self, ts, x, out=None):
        import torch
        n = sum(self.shapes[t][2] for t in ts)
        M = x.shape[0]
        if out is None:
            out = torch.empty((M, n), dtype=x.dtype, device=x.device)
        need = cloak_linear_fused_ws_bytes(self.layout, list(ts), M)
        ws = self.workspace(need) if need else None
        cloak_linear_fused(self.layout, self.pool, list(ts), x, M, out, ws, 0 if ws is None else ws.numel())
        return out

    def mlp(self, layer, x, out=None):
        import torch
        M = x.shape[0]
        need = cloak_mlp_ws_bytes(self.layout, layer, M)
        ws = self.workspace(need)
        if out is None:
            out = torch.empty_like(x)
        cloak_mlp(self.layout, self.pool, layer, x, M, out, ws, ws.numel())
        return out

    def remap(self, remap_seed=None):
        s = int.from_bytes(os.urandom(8), "little") if remap_seed is None else int(remap_seed)
        cloak_remap(self.layout, self.pool, s)

    def remap_begin(self, remap_seed=None):
        s = int.from_bytes(os.urandom(8), "little") if remap_seed is None else int(remap_seed)
        cloak_remap_begin(self.layout, s)

    def remap_step(self, max_pairs=0):
        """Swap the next max_pairs page pairs of the remap in progress; returns pairs left."""
        return cloak_remap_step(self.layout, self.pool, max_pairs)

    def close(self):
        if self.layout:
            import torch
            torch.cuda.synchronize()
            cloak_layout_free(self.layout)
            self.layout = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

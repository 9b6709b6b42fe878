"""paper_1610_03525_amd -- Python binding of libptg (polynomial gradient-noise fBm on MI355X).

Argument marshalling only: tensors become device pointers, the current torch stream
becomes the hipStream_t, and every step of the computation runs in the HIP kernels of
``libptg.so`` (C ABI in ``include/ptg.h``).  There is no CPU fallback: if the library
is not built, every call raises ``RuntimeError``.

Method: Thorimbert & Chopard, "Polynomial methods for fast Procedural Terrain Generation"
(arXiv:1610.03525) -- boundary-constrained cell polynomials (Sec. 2, Sec. 3.4) summed over
fBm octaves (Sec. 4).
"""
import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptg.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ptg.h")

PTG_OK = 0
PTG_EINVAL = -1
PTG_ENOMEM = -2
PTG_E2BIG = -3
PTG_EAGAIN = -4
PTG_ETIMEDOUT = -5
PTG_ESHUTDOWN = -6
PTG_EHIP = -7
PTG_ENOENT = -8

PTG_F32 = 0
PTG_F16 = 1
FORMS = {"plain": 0, "mfma_f16": 1, "mfma_bf16": 2}
BASES = {"monomial": 0, "centred": 1, "hermite": 2}
PATHS = {"auto": 0, "general": 1, "dyadic": 2}
MODELS = {"gradient": 0, "zero_gradient": 1, "height_gradient": 2, "perlin": 3, "simplex": 4}
PTG_MODEL_GRADIENT = 0
PTG_MODEL_ZERO_GRADIENT = 1
PTG_MODEL_HEIGHT_GRADIENT = 2
PTG_MODEL_PERLIN = 3
PTG_MODEL_SIMPLEX = 4


class PtgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ptg error {code}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("smoothness", ctypes.c_int32),
        ("octaves", ctypes.c_int32),
        ("out_dtype", ctypes.c_int32),
        ("persistence", ctypes.c_double),
        ("lacunarity", ctypes.c_double),
        ("base_freq", ctypes.c_double),
        ("seed", ctypes.c_uint32),
        ("form", ctypes.c_int32),
        ("basis", ctypes.c_int32),
        ("path", ctypes.c_int32),
        ("model", ctypes.c_int32),
        ("gradient_weight", ctypes.c_double),
    ]


class ServerCfg(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_int64),
        ("max_items", ctypes.c_int32),
        ("workgroups", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("executor", ctypes.c_int32),
        ("fake_tile_ns", ctypes.c_int64),
        ("tiles_per_item", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("tile_h", ctypes.c_int32),
        ("lattice_cache", ctypes.c_int32),
    ]


class TileReq(ctypes.Structure):
    _fields_ = [
        ("params", Params),
        ("origin", ctypes.c_int64 * 3),
        ("extent", ctypes.c_int64 * 3),
        ("user_tag", ctypes.c_uint64),
    ]


class TileResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("kernel", ctypes.c_int32),
        ("out_dev", ctypes.c_void_p),
        ("bytes", ctypes.c_int64),
        ("user_tag", ctypes.c_uint64),
        ("t_submit_ns", ctypes.c_int64),
        ("t_admit_ns", ctypes.c_int64),
        ("t_done_ns", ctypes.c_int64),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "submitted", "admitted", "completed", "released", "tiles_done", "pending", "in_flight",
        "bytes_in_use", "bytes_peak", "budget", "kernel_launches")] + [("tile_h", ctypes.c_int32 * 2)] + [
        (n, ctypes.c_int64) for n in ("lat_blocks", "lat_bytes", "lat_hits", "lat_misses", "lat_evictions")]


PTG_TUNE_GENERAL_2D, PTG_TUNE_STRIP_2D, PTG_TUNE_GENERAL_3D, PTG_TUNE_STRIP_3D, PTG_TUNE_DYADIC_2D = 1, 2, 3, 4, 5
TUNE_NAMES = {1: "general_2d", 2: "strip_2d", 3: "general_3d", 4: "strip_3d", 5: "dyadic_2d"}


class TuneResult(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_int32),
        ("value", ctypes.c_int32),
        ("n", ctypes.c_int32),
        ("default_value", ctypes.c_int32),
        ("candidates", ctypes.c_int32 * 4),
        ("us", ctypes.c_double * 4),
    ]


PTG_EXEC_GPU = 0
PTG_EXEC_HOST = 1


class BatchStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("launches", "nodes", "instantiations", "updates", "instances",
                                              "pending")]

_LIB = None
_i32, _u32, _i64, _f32, _f64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
_vp = ctypes.c_void_p
_PP = ctypes.POINTER(Params)


def lib():
    """The loaded libptg.so; raises RuntimeError when it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    L.ptg_version.restype = ctypes.c_char_p
    L.ptg_last_error.restype = ctypes.c_char_p
    L.ptg_params_default.argtypes = [_PP]
    L.ptg_fbm_2d.argtypes = [_PP, _i64, _i64, _i64, _i64, _vp, _i64, _vp]
    L.ptg_fbm_3d.argtypes = [_PP, _i64, _i64, _i64, _i64, _i64, _i64, _vp, _vp]
    L.ptg_fbm_2d_grad.argtypes = [_PP, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _i64, _vp]
    L.ptg_coords.argtypes = [_f64, _f64, _i32, _i64, _i64, _vp, _vp, _vp]
    L.ptg_lattice_2d.argtypes = [_u32, _i32, _i64, _i64, _i64, _i64, _vp, _vp, _vp]
    L.ptg_lattice_3d.argtypes = [_u32, _i32, _i64, _i64, _i64, _i64, _i64, _i64, _vp, _vp, _vp, _vp]
    L.ptg_heights_2d.argtypes = [_u32, _i32, _i64, _i64, _i64, _i64, _vp, _vp]
    L.ptg_cells_2d.argtypes = [_i32, _vp, _i64, _i64, _f32, _vp, _vp]
    L.ptg_cells_3d.argtypes = [_i32, _vp, _i64, _i64, _i64, _f32, _vp, _vp]
    L.ptg_server_create.argtypes = [ctypes.POINTER(ServerCfg), ctypes.POINTER(ctypes.c_void_p)]
    L.ptg_tiles_submit.argtypes = [_vp, ctypes.POINTER(TileReq), _i32, ctypes.POINTER(ctypes.c_uint64)]
    L.ptg_tiles_wait.argtypes = [_vp, ctypes.c_uint64, _i64, ctypes.POINTER(TileResult)]
    L.ptg_tiles_wait_any.argtypes = [_vp, _i64, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(TileResult)]
    L.ptg_tile_release.argtypes = [_vp, ctypes.c_uint64]
    L.ptg_server_stats_get.argtypes = [_vp, ctypes.POINTER(ServerStats)]
    L.ptg_server_destroy.argtypes = [_vp]
    _TR = ctypes.POINTER(TuneResult)
    _IP = ctypes.POINTER(_i32)
    L.ptg_tune_2d.argtypes = [_PP, _i64, _i64, _i64, _i64, _vp, _i64, _vp, _i32, _TR]
    L.ptg_tune_3d.argtypes = [_PP, _i64, _i64, _i64, _i64, _i64, _i64, _vp, _vp, _i32, _TR]
    L.ptg_tune_query_2d.argtypes = [_PP, _i64, _i64, _IP, _IP]
    L.ptg_tune_query_3d.argtypes = [_PP, _i64, _i64, _i64, _IP, _IP]
    L.ptg_tune_set_2d.argtypes = [_PP, _i64, _i64, _i32]
    L.ptg_tune_set_3d.argtypes = [_PP, _i64, _i64, _i64, _i32]
    L.ptg_tune_reset.argtypes = []
    L.ptg_tune_reset.restype = None
    L.ptg_tune_save.argtypes = [ctypes.c_char_p]
    L.ptg_tune_load.argtypes = [ctypes.c_char_p, _IP]
    L.ptg_batch_create.argtypes = [_i32, ctypes.POINTER(ctypes.c_void_p)]
    L.ptg_batch_add_2d.argtypes = [_vp, _PP, _i64, _i64, _i64, _i64, _vp, _i64]
    L.ptg_batch_add_3d.argtypes = [_vp, _PP, _i64, _i64, _i64, _i64, _i64, _i64, _vp]
    L.ptg_batch_launch.argtypes = [_vp, _vp]
    L.ptg_batch_clear.argtypes = [_vp]
    L.ptg_batch_stats_get.argtypes = [_vp, ctypes.POINTER(BatchStats)]
    L.ptg_batch_destroy.argtypes = [_vp]
    for name in ("ptg_fbm_2d", "ptg_fbm_2d_grad", "ptg_fbm_3d", "ptg_coords", "ptg_lattice_2d", "ptg_lattice_3d", "ptg_heights_2d",
                 "ptg_cells_2d", "ptg_cells_3d", "ptg_server_create", "ptg_tiles_submit", "ptg_tiles_wait",
                 "ptg_tile_release", "ptg_server_stats_get", "ptg_server_destroy", "ptg_tune_2d", "ptg_tune_3d",
                 "ptg_tune_query_2d", "ptg_tune_query_3d", "ptg_tune_set_2d", "ptg_tune_set_3d",
                 "ptg_batch_create", "ptg_batch_add_2d", "ptg_batch_add_3d", "ptg_batch_launch", "ptg_batch_clear",
                 "ptg_batch_stats_get", "ptg_batch_destroy"):
        getattr(L, name).restype = _i32
    _LIB = L
    return L


def declared_symbols():
    """Names of the functions include/ptg.h declares (PTG_API prototypes)."""
    with open(HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"PTG_API\s+[\w\s\*]*?\b(ptg_\w+)\s*\(", text)))


def last_error() -> str:
    return lib().ptg_last_error().decode()


def _check(rc):
    if rc != PTG_OK:
        raise PtgError(rc, last_error())


def params(dim=2, smoothness=1, octaves=8, persistence=0.5, lacunarity=2.0, base_freq=1.0 / 512, seed=1,
           out_dtype=PTG_F32, form="plain", basis="monomial", path="auto", model="gradient",
           gradient_weight=0.01) -> Params:
    p = Params()
    p.dim = dim
    p.smoothness = smoothness
    p.octaves = octaves
    p.out_dtype = out_dtype
    p.persistence = persistence
    p.lacunarity = lacunarity
    p.base_freq = base_freq
    p.seed = seed & 0xFFFFFFFF
    p.form = FORMS[form] if isinstance(form, str) else int(form)
    p.basis = BASES[basis] if isinstance(basis, str) else int(basis)
    p.path = PATHS[path] if isinstance(path, str) else int(path)
    p.model = MODELS[model] if isinstance(model, str) else int(model)
    p.gradient_weight = gradient_weight
    return p


def _stream(stream):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _dev_ptr(t, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device (cuda) torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    return t.data_ptr()


def _out_dtype(t):
    import torch
    if t.dtype == torch.float32:
        return PTG_F32
    if t.dtype == torch.float16:
        return PTG_F16
    raise TypeError("output must be float32 or float16")


# ---- dense fields -------------------------------------------------------------------

def fbm_2d_raw(p: Params, x0, y0, nx, ny, out_ptr, pitch, stream_handle):
    _check(lib().ptg_fbm_2d(ctypes.byref(p), x0, y0, nx, ny, out_ptr, pitch, stream_handle))


def fbm_3d_raw(p: Params, x0, y0, z0, nx, ny, nz, out_ptr, stream_handle):
    _check(lib().ptg_fbm_3d(ctypes.byref(p), x0, y0, z0, nx, ny, nz, out_ptr, stream_handle))


def fbm_2d(out, *, x0=0, y0=0, stream=None, **kw):
    """Fill a 2D (ny, nx) float32/float16 device tensor (row stride >= nx) with the fBm field
    whose element (j, i) is world sample (x0 + i, y0 + j)."""
    if out.dim() != 2 or out.stride(1) != 1:
        raise ValueError("out must be 2D with unit column stride")
    p = params(dim=2, out_dtype=_out_dtype(out), **kw)
    ny, nx = out.shape
    fbm_2d_raw(p, x0, y0, nx, ny, _dev_ptr(out) if out.numel() else None, out.stride(0), _stream(stream))
    return out


def fbm_2d_grad(out, out_dx, out_dy, *, x0=0, y0=0, stream=None, **kw):
    """The 2D field into out and its world-space gradient dH/dX, dH/dY into out_dx, out_dy
    (three (ny, nx) tensors of one dtype and row stride)."""
    for t in (out, out_dx, out_dy):
        if t.dim() != 2 or t.stride(1) != 1 or t.shape != out.shape or t.stride(0) != out.stride(0) \
                or t.dtype != out.dtype:
            raise ValueError("outputs must be 2D tensors of one shape, dtype and row stride")
    p = params(dim=2, out_dtype=_out_dtype(out), **kw)
    ny, nx = out.shape
    ptrs = [_dev_ptr(t) if t.numel() else None for t in (out, out_dx, out_dy)]
    _check(lib().ptg_fbm_2d_grad(ctypes.byref(p), x0, y0, nx, ny, *ptrs, out.stride(0), _stream(stream)))
    return out, out_dx, out_dy


def fbm_3d(out, *, x0=0, y0=0, z0=0, stream=None, **kw):
    """Fill a contiguous (nz, ny, nx) device tensor with the 3D fBm volume."""
    if out.dim() != 3 or not out.is_contiguous():
        raise ValueError("out must be a contiguous 3D tensor")
    p = params(dim=3, out_dtype=_out_dtype(out), **kw)
    nz, ny, nx = out.shape
    fbm_3d_raw(p, x0, y0, z0, nx, ny, nz, _dev_ptr(out) if out.numel() else None, _stream(stream))
    return out


# ---- stages -------------------------------------------------------------------------
# The stage entry points take no buffer sizes, so every wrapper checks each tensor's dtype,
# exact shape and contiguity against the sizes it passes before anything is launched.

def _need(t, name, shape, dtype):
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name}: expected dtype {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(int(v) for v in shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    return t


def _ptrs(*ts):
    """Device pointers of already checked tensors (None stays None)."""
    return [None if t is None else _dev_ptr(t) for t in ts]


def coords(base_freq, lacunarity, octaves, x0, cells_out, frac_out, stream=None):
    """a1: cells_out (octaves, n) int64 and frac_out (octaves, n) float32 device tensors."""
    import torch
    if cells_out.dim() != 2:
        raise ValueError("cells_out must be (octaves, n)")
    n = cells_out.shape[1]
    cp, fp = _ptrs(_need(cells_out, "cells_out", (octaves, n), torch.int64),
                   _need(frac_out, "frac_out", (octaves, n), torch.float32))
    _check(lib().ptg_coords(base_freq, lacunarity, octaves, x0, n, cp, fp, _stream(stream)))


def lattice_2d(seed, octave, ix0, iy0, keys_out=None, grad_out=None, stream=None):
    """K1: keys_out (ny, nx) int32 tensor (uint32 bits) and/or grad_out (2, ny, nx) float32."""
    import torch
    if keys_out is None and grad_out is None:
        raise ValueError("lattice_2d needs keys_out or grad_out")
    ref = keys_out if keys_out is not None else grad_out
    if ref.dim() < 2:
        raise ValueError("keys_out must be (ny, nx) and grad_out (2, ny, nx)")
    ny, nx = ref.shape[-2:]
    kp, gp = _ptrs(_need(keys_out, "keys_out", (ny, nx), torch.int32) if keys_out is not None else None,
                   _need(grad_out, "grad_out", (2, ny, nx), torch.float32) if grad_out is not None else None)
    _check(lib().ptg_lattice_2d(seed & 0xFFFFFFFF, octave, ix0, iy0, nx, ny, kp, gp, _stream(stream)))


def heights_2d(seed, octave, ix0, iy0, out, stream=None):
    """K1 of the zero-gradient model: node heights into out (ny, nx) float32."""
    import torch
    if out.dim() != 2:
        raise ValueError("out must be (ny, nx)")
    ny, nx = out.shape
    hp, = _ptrs(_need(out, "out", (ny, nx), torch.float32))
    _check(lib().ptg_heights_2d(seed & 0xFFFFFFFF, octave, ix0, iy0, nx, ny, hp, _stream(stream)))


def lattice_3d(seed, octave, ix0, iy0, iz0, keys_out=None, second_out=None, grad_out=None, stream=None):
    """K1, 3D: keys_out / second_out (nz, ny, nx) int32 and/or grad_out (3, nz, ny, nx) float32."""
    import torch
    if keys_out is None and second_out is None and grad_out is None:
        raise ValueError("lattice_3d needs at least one output")
    ref = keys_out if keys_out is not None else (second_out if second_out is not None else grad_out)
    if ref.dim() < 3:
        raise ValueError("keys_out / second_out must be (nz, ny, nx) and grad_out (3, nz, ny, nx)")
    nz, ny, nx = ref.shape[-3:]
    kp, sp, gp = _ptrs(
        _need(keys_out, "keys_out", (nz, ny, nx), torch.int32) if keys_out is not None else None,
        _need(second_out, "second_out", (nz, ny, nx), torch.int32) if second_out is not None else None,
        _need(grad_out, "grad_out", (3, nz, ny, nx), torch.float32) if grad_out is not None else None)
    _check(lib().ptg_lattice_3d(seed & 0xFFFFFFFF, octave, ix0, iy0, iz0, nx, ny, nz, kp, sp, gp, _stream(stream)))


def cells_2d(smoothness, grad, amplitude, coeff_out, stream=None):
    """K2: grad (2, nny, nnx) float32 -> coeff_out (nny-1, nnx-1, n+1, n+1) float32."""
    import torch
    if grad.dim() != 3 or grad.shape[1] < 2 or grad.shape[2] < 2:
        raise ValueError("grad must be (2, nny, nnx) with nny, nnx >= 2")
    _, nny, nnx = grad.shape
    n1 = 2 * int(smoothness) + 2
    gp, cp = _ptrs(_need(grad, "grad", (2, nny, nnx), torch.float32),
                   _need(coeff_out, "coeff_out", (nny - 1, nnx - 1, n1, n1), torch.float32))
    _check(lib().ptg_cells_2d(smoothness, gp, nnx, nny, amplitude, cp, _stream(stream)))


def cells_3d(smoothness, grad, amplitude, coeff_out, stream=None):
    """K2, 3D: grad (3, nnz, nny, nnx) -> coeff_out (nnz-1, nny-1, nnx-1, n+1, n+1, n+1)."""
    import torch
    if grad.dim() != 4 or min(grad.shape[1:]) < 2:
        raise ValueError("grad must be (3, nnz, nny, nnx) with every node count >= 2")
    _, nnz, nny, nnx = grad.shape
    n1 = 2 * int(smoothness) + 2
    gp, cp = _ptrs(_need(grad, "grad", (3, nnz, nny, nnx), torch.float32),
                   _need(coeff_out, "coeff_out", (nnz - 1, nny - 1, nnx - 1, n1, n1, n1), torch.float32))
    _check(lib().ptg_cells_3d(smoothness, gp, nnx, nny, nnz, amplitude, cp, _stream(stream)))


def version() -> str:
    return lib().ptg_version().decode()


# ---- serving ------------------------------------------------------------------------

# ---- a6: tile-shape autotuner -----------------------------------------------------

def _tune_dict(r: TuneResult) -> dict:
    return {"kernel": TUNE_NAMES.get(r.kernel, r.kernel), "value": r.value, "default": r.default_value,
            "candidates": {int(r.candidates[i]): float(r.us[i]) for i in range(r.n)}}


def tune_2d(out, *, x0=0, y0=0, stream=None, reps=5, **kw) -> dict:
    """Time every candidate shape of the kernel class that fbm_2d(out, ...) runs, record the
    fastest (used by later calls of that class) and return the timings (us per launch).
    out receives the field."""
    if out.dim() != 2 or out.stride(1) != 1:
        raise ValueError("out must be a 2D tensor with unit column stride")
    p = params(dim=2, out_dtype=_out_dtype(out), **kw)
    ny, nx = out.shape
    r = TuneResult()
    _check(lib().ptg_tune_2d(p, x0, y0, nx, ny, _dev_ptr(out), out.stride(0), _stream(stream), reps,
                             ctypes.byref(r)))
    return _tune_dict(r)


def tune_3d(out, *, x0=0, y0=0, z0=0, stream=None, reps=5, **kw) -> dict:
    if out.dim() != 3 or not out.is_contiguous():
        raise ValueError("out must be a contiguous 3D tensor")
    p = params(dim=3, out_dtype=_out_dtype(out), **kw)
    nz, ny, nx = out.shape
    r = TuneResult()
    _check(lib().ptg_tune_3d(p, x0, y0, z0, nx, ny, nz, _dev_ptr(out), _stream(stream), reps, ctypes.byref(r)))
    return _tune_dict(r)


def tune_query(shape, out_dtype=PTG_F32, **kw):
    """(kernel class name, shape) a call over `shape` ((ny, nx) or (nz, ny, nx)) would use
    now; host only."""
    k, v = _i32(), _i32()
    if len(shape) == 2:
        p = params(dim=2, out_dtype=out_dtype, **kw)
        _check(lib().ptg_tune_query_2d(p, shape[1], shape[0], ctypes.byref(k), ctypes.byref(v)))
    else:
        p = params(dim=3, out_dtype=out_dtype, **kw)
        _check(lib().ptg_tune_query_3d(p, shape[2], shape[1], shape[0], ctypes.byref(k), ctypes.byref(v)))
    return TUNE_NAMES.get(k.value, k.value), v.value


def tune_set(shape, value, out_dtype=PTG_F32, **kw):
    """Record a shape for the kernel class of a call over `shape`."""
    if len(shape) == 2:
        _check(lib().ptg_tune_set_2d(params(dim=2, out_dtype=out_dtype, **kw), shape[1], shape[0], value))
    else:
        _check(lib().ptg_tune_set_3d(params(dim=3, out_dtype=out_dtype, **kw), shape[2], shape[1], shape[0], value))


def tune_reset():
    lib().ptg_tune_reset()


def tune_save(path):
    """Write the recorded shapes to `path`, keyed by the current device."""
    _check(lib().ptg_tune_save(os.fsencode(path)))


def tune_load(path) -> int:
    """Add the shapes of a file written for this device; returns how many were taken (0 for
    a table of another device)."""
    n = ctypes.c_int32()
    _check(lib().ptg_tune_load(os.fsencode(path), ctypes.byref(n)))
    return n.value


class Batch:
    """Dense-field calls launched together as one HIP graph (ptg_batch in the C ABI): the
    graph of a batch shape is instantiated once, later batches of that shape update its
    arguments.  The calls of one batch may run concurrently (outputs must not overlap)."""

    def __init__(self, max_calls=256):
        h = ctypes.c_void_p()
        _check(lib().ptg_batch_create(max_calls, ctypes.byref(h)))
        self.h = h

    def add_2d(self, out, *, x0=0, y0=0, **kw):
        if out.dim() != 2 or out.stride(1) != 1:
            raise ValueError("out must be 2D with unit column stride")
        p = params(dim=2, out_dtype=_out_dtype(out), **kw)
        ny, nx = out.shape
        _check(lib().ptg_batch_add_2d(self.h, ctypes.byref(p), x0, y0, nx, ny, _dev_ptr(out) if out.numel() else None,
                                      out.stride(0)))

    def add_3d(self, out, *, x0=0, y0=0, z0=0, **kw):
        if out.dim() != 3 or not out.is_contiguous():
            raise ValueError("out must be a contiguous 3D tensor")
        p = params(dim=3, out_dtype=_out_dtype(out), **kw)
        nz, ny, nx = out.shape
        _check(lib().ptg_batch_add_3d(self.h, ctypes.byref(p), x0, y0, z0, nx, ny, nz,
                                      _dev_ptr(out) if out.numel() else None))

    def launch(self, stream=None):
        _check(lib().ptg_batch_launch(self.h, _stream(stream)))

    def clear(self):
        _check(lib().ptg_batch_clear(self.h))

    def stats(self) -> dict:
        st = BatchStats()
        _check(lib().ptg_batch_stats_get(self.h, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in BatchStats._fields_}

    def close(self):
        if self.h:
            rc = lib().ptg_batch_destroy(self.h)
            self.h = None
            _check(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def tile_req(dim=2, origin=(0, 0, 0), extent=(64, 64, 1), user_tag=0, **kw) -> TileReq:
    r = TileReq()
    r.params = params(dim=dim, **kw)
    for i in range(3):
        r.origin[i] = origin[i] if i < len(origin) else 0
        r.extent[i] = extent[i] if i < len(extent) else 1
    r.user_tag = user_tag
    return r


class Server:
    """Continuous-batching tile server (a persistent kernel + host scheduler in libptg)."""

    def __init__(self, budget_bytes, max_items=1 << 16, workgroups=0, device=0, executor=PTG_EXEC_GPU,
                 fake_tile_ns=0, tiles_per_item=0, autotune=0, tile_h=0, lattice_cache=0):
        cfg = ServerCfg(budget_bytes, max_items, workgroups, device, executor, fake_tile_ns, tiles_per_item,
                        autotune, tile_h, lattice_cache)
        h = ctypes.c_void_p()
        _check(lib().ptg_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h

    def submit(self, reqs):
        n = len(reqs)
        arr = (TileReq * n)(*reqs)
        tickets = (ctypes.c_uint64 * n)()
        _check(lib().ptg_tiles_submit(self.h, arr, n, tickets))
        return list(tickets)

    def wait(self, ticket, timeout_ns=-1):
        """TileResult of a ticket; raises PtgError(PTG_ETIMEDOUT) when still pending."""
        res = TileResult()
        _check(lib().ptg_tiles_wait(self.h, ticket, timeout_ns, ctypes.byref(res)))
        return res

    def wait_any(self, timeout_ns=-1):
        """(ticket, TileResult) of the next request to complete, in completion order; raises
        PtgError(PTG_ETIMEDOUT) when none completes in time, PTG_ENOENT when none can."""
        res = TileResult()
        t = ctypes.c_uint64()
        _check(lib().ptg_tiles_wait_any(self.h, timeout_ns, ctypes.byref(t), ctypes.byref(res)))
        return t.value, res

    def release(self, ticket):
        _check(lib().ptg_tile_release(self.h, ticket))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().ptg_server_stats_get(self.h, ctypes.byref(st)))
        d = {n: getattr(st, n) for n, _ in ServerStats._fields_}
        d["tile_h"] = list(st.tile_h)
        return d

    def close(self):
        if self.h:
            rc = lib().ptg_server_destroy(self.h)
            self.h = None
            _check(rc)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


_HIP = None


def device_copy(dst_ptr, src_ptr, nbytes):
    """Device-to-device copy between raw device pointers (e.g. a served tile into a torch
    tensor), complete when this returns.  A device-to-device hipMemcpy may return before the
    copy has run, so the null stream it is queued on is synchronised as well (only that
    stream: the server's own stream is non-blocking and never waited for)."""
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.argtypes = [_vp, _vp, ctypes.c_size_t, ctypes.c_int]
        _HIP.hipMemcpy.restype = ctypes.c_int
        _HIP.hipStreamSynchronize.argtypes = [_vp]
        _HIP.hipStreamSynchronize.restype = ctypes.c_int
    rc = _HIP.hipMemcpy(dst_ptr, src_ptr, nbytes, 3)  # hipMemcpyDeviceToDevice
    if rc == 0:
        rc = _HIP.hipStreamSynchronize(None)
    if rc != 0:
        raise PtgError(PTG_EHIP, f"hipMemcpy failed ({rc})")

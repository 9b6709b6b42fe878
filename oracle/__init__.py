"""FP64 CPU oracle for polynomial gradient-noise fBm -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and its
binding) never imports it; the two share no code.

Everything here is a thin ctypes view of ``ptg_oracle.c``; see that file for the
definitions and the paper passages they follow (Sec. 2 model, Sec. 3 special cases,
Sec. 4 fBm octave sum).  If the shared library is missing it is compiled on first
use with ``gcc`` (host only, no GPU involved).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None

_i32 = ctypes.c_int32
_u32 = ctypes.c_uint32
_i64 = ctypes.c_int64
_f64 = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)
_pi64 = ctypes.POINTER(ctypes.c_int64)


def lib():
    """Load (building if needed) the oracle shared library."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC):
        _build.build()
    L = ctypes.CDLL(_build.LIB)
    L.orc_fmix32.argtypes = [_u32]
    L.orc_fmix32.restype = _u32
    L.orc_prefix.argtypes = [_u32, _i32]
    L.orc_prefix.restype = _u32
    L.orc_key2.argtypes = [_i64, _i64, _i32, _u32]
    L.orc_key2.restype = _u32
    L.orc_key3.argtypes = [_i64, _i64, _i64, _i32, _u32]
    L.orc_key3.restype = _u32
    L.orc_key3_second.argtypes = [_u32]
    L.orc_key3_second.restype = _u32
    L.orc_grad2.argtypes = [_u32, _pd]
    L.orc_grad3.argtypes = [_u32, _pd]
    L.orc_octave_params.argtypes = [_f64, _f64, _f64, _i32, _pd, _pd]
    L.orc_coord.argtypes = [_i64, _f64, _pi64, _pd]
    L.orc_basis.argtypes = [_i32, _f64, _pd, _pd]
    L.orc_hermite_closed.argtypes = [_i32, _f64, _pd, _pd]
    L.orc_cell_2d.argtypes = [_i32, _pd, _f64, _f64]
    L.orc_cell_2d.restype = _f64
    L.orc_cell_3d.argtypes = [_i32, _pd, _f64, _f64, _f64]
    L.orc_cell_3d.restype = _f64
    L.orc_coeffs_2d.argtypes = [_i32, _pd, _pd]
    L.orc_coeffs_3d.argtypes = [_i32, _pd, _pd]
    L.orc_perlin_cell.argtypes = [_i32, _pd, _f64, _f64]
    L.orc_perlin_cell.restype = _f64
    L.orc_fbm_2d.argtypes = [_i32, _i32, _f64, _f64, _f64, _u32, _i64, _i64, _i64, _i64, _pd, _i32]
    L.orc_fbm_2d.restype = _i32
    L.orc_fbm_3d.argtypes = [_i32, _i32, _f64, _f64, _f64, _u32, _i64, _i64, _i64, _i64, _i64, _i64,
                             _pd, _i32]
    L.orc_fbm_3d.restype = _i32
    L.orc_fbm_points_2d.argtypes = [_i32, _i32, _f64, _f64, _f64, _u32, _pi64, _pi64, _i64, _pd, _i32]
    L.orc_fbm_points_2d.restype = _i32
    L.orc_fbm_points_3d.argtypes = [_i32, _i32, _f64, _f64, _f64, _u32, _pi64, _pi64, _pi64, _i64,
                                    _pd, _i32]
    L.orc_fbm_points_3d.restype = _i32
    L.orc_perlin_2d.argtypes = [_i32, _i32, _f64, _f64, _f64, _u32, _i64, _i64, _i64, _i64, _pd, _i32]
    L.orc_perlin_2d.restype = _i32
    L.orc_height2.argtypes = [_u32]
    L.orc_height2.restype = _f64
    L.orc_zg_cell.argtypes = [_pd, _f64, _f64]
    L.orc_zg_cell.restype = _f64
    L.orc_zg_fbm_2d.argtypes = [_i32, _f64, _f64, _f64, _u32, _i64, _i64, _i64, _i64, _pd, _i32]
    L.orc_zg_fbm_2d.restype = _i32
    L.orc_zg_fbm_points_2d.argtypes = [_i32, _f64, _f64, _f64, _u32, _pi64, _pi64, _i64, _pd, _i32]
    L.orc_zg_fbm_points_2d.restype = _i32
    L.orc_height2_second.argtypes = [_u32]
    L.orc_height2_second.restype = _f64
    L.orc_hg_cell.argtypes = [_i32, _pd, _pd, _f64, _f64, _f64]
    L.orc_hg_cell.restype = _f64
    L.orc_hg_fbm_2d.argtypes = [_i32, _i32, _f64, _f64, _f64, _f64, _u32, _i64, _i64, _i64, _i64, _pd, _i32]
    L.orc_simplex_at.argtypes = [_f64, _f64, _i32, _u32]
    L.orc_simplex_at.restype = _f64
    L.orc_simplex_2d.argtypes = [_i32, _f64, _f64, _f64, _u32, _i64, _i64, _i64, _i64, _pd, _i32]
    L.orc_height3.argtypes = [_u32]
    L.orc_height3.restype = _f64
    L.orc_hg_cell_3d.argtypes = [_i32, _pd, _pd, _f64, _f64, _f64, _f64]
    L.orc_hg_cell_3d.restype = _f64
    L.orc_hg_fbm_3d.argtypes = [_i32, _i32, _f64, _f64, _f64, _f64, _u32, _i64, _i64, _i64, _i64, _i64, _i64, _pd,
                                _i32]
    L.orc_hg_fbm_points_3d.argtypes = [_i32, _i32, _f64, _f64, _f64, _f64, _u32, _pi64, _pi64, _pi64, _i64, _pd,
                                       _i32]
    L.orc_hg_fbm_2d.restype = _i32
    L.orc_hg_fbm_points_2d.argtypes = [_i32, _i32, _f64, _f64, _f64, _f64, _u32, _pi64, _pi64, _i64, _pd, _i32]
    L.orc_hg_fbm_points_2d.restype = _i32
    L.orc_basis_deriv.argtypes = [_i32, _f64, _pd, _pd]
    L.orc_cell_2d_grad.argtypes = [_i32, _i32, _pd, _pd, _f64, _f64, _f64, _pd]
    L.orc_fbm_2d_grad.argtypes = [_i32, _i32, _i32, _f64, _f64, _f64, _f64, _u32, _i64, _i64, _i64, _i64, _pd, _pd,
                                  _pd, _i32]
    L.orc_fbm_2d_grad.restype = _i32
    L.orc_max_threads.argtypes = []
    L.orc_max_threads.restype = _i32
    _LIB = L
    return L


def _dp(a):
    return a.ctypes.data_as(_pd)


def _ip(a):
    return a.ctypes.data_as(_pi64)


# --- lattice ---------------------------------------------------------------

def fmix32(h: int) -> int:
    return int(lib().orc_fmix32(h & 0xFFFFFFFF))


def key2(ix: int, iy: int, octave: int, seed: int) -> int:
    return int(lib().orc_key2(ix, iy, octave, seed & 0xFFFFFFFF))


def key3(ix: int, iy: int, iz: int, octave: int, seed: int) -> int:
    return int(lib().orc_key3(ix, iy, iz, octave, seed & 0xFFFFFFFF))


def key3_second(key: int) -> int:
    return int(lib().orc_key3_second(key & 0xFFFFFFFF))


def grad2(key: int) -> np.ndarray:
    g = np.zeros(2)
    lib().orc_grad2(key & 0xFFFFFFFF, _dp(g))
    return g


def grad3(key: int) -> np.ndarray:
    g = np.zeros(3)
    lib().orc_grad3(key & 0xFFFFFFFF, _dp(g))
    return g


def keys2_box(ix0, iy0, nx, ny, octave, seed) -> np.ndarray:
    """uint32 keys of the node box [ix0, ix0+nx) x [iy0, iy0+ny), shape (ny, nx)."""
    L = lib()
    out = np.empty((ny, nx), dtype=np.uint32)
    for j in range(ny):
        for i in range(nx):
            out[j, i] = L.orc_key2(ix0 + i, iy0 + j, octave, seed & 0xFFFFFFFF)
    return out


def keys3_box(ix0, iy0, iz0, nx, ny, nz, octave, seed) -> np.ndarray:
    L = lib()
    out = np.empty((nz, ny, nx), dtype=np.uint32)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                out[k, j, i] = L.orc_key3(ix0 + i, iy0 + j, iz0 + k, octave, seed & 0xFFFFFFFF)
    return out


# --- coordinates / octaves -------------------------------------------------

def octave_params(f0: float, lac: float, pers: float, n: int):
    f = np.zeros(n)
    a = np.zeros(n)
    lib().orc_octave_params(f0, lac, pers, n, _dp(f), _dp(a))
    return f, a


def coord(X: int, f: float):
    c = np.zeros(1, dtype=np.int64)
    t = np.zeros(1)
    lib().orc_coord(X, f, _ip(c), _dp(t))
    return int(c[0]), float(t[0])


def basis(smooth: int, t: float):
    b0 = np.zeros(2)
    b1 = np.zeros(2)
    lib().orc_basis(smooth, t, _dp(b0), _dp(b1))
    return b0, b1


def hermite_closed(M: int, t: float):
    """The four 1D bases of order M from their closed forms (any M <= 6)."""
    b0 = np.zeros(2)
    b1 = np.zeros(2)
    lib().orc_hermite_closed(M, t, _dp(b0), _dp(b1))
    return b0, b1


# --- one cell --------------------------------------------------------------

def cell_2d(smooth: int, grad: np.ndarray, tx: float, ty: float) -> float:
    g = np.ascontiguousarray(grad, dtype=np.float64).reshape(8)
    return float(lib().orc_cell_2d(smooth, _dp(g), tx, ty))


def cell_3d(smooth: int, grad: np.ndarray, tx: float, ty: float, tz: float) -> float:
    g = np.ascontiguousarray(grad, dtype=np.float64).reshape(24)
    return float(lib().orc_cell_3d(smooth, _dp(g), tx, ty, tz))


def coeffs_2d(smooth: int, grad: np.ndarray) -> np.ndarray:
    n1 = 2 * smooth + 2
    g = np.ascontiguousarray(grad, dtype=np.float64).reshape(8)
    c = np.zeros(n1 * n1)
    lib().orc_coeffs_2d(smooth, _dp(g), _dp(c))
    return c.reshape(n1, n1)


def coeffs_3d(smooth: int, grad: np.ndarray) -> np.ndarray:
    n1 = 2 * smooth + 2
    g = np.ascontiguousarray(grad, dtype=np.float64).reshape(24)
    c = np.zeros(n1 ** 3)
    lib().orc_coeffs_3d(smooth, _dp(g), _dp(c))
    return c.reshape(n1, n1, n1)


def perlin_cell(fade_order: int, grad: np.ndarray, x: float, y: float) -> float:
    g = np.ascontiguousarray(grad, dtype=np.float64).reshape(8)
    return float(lib().orc_perlin_cell(fade_order, _dp(g), x, y))


# --- fields ----------------------------------------------------------------

def _chk(rc):
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (rc={rc})")


def fbm_2d(smooth, octaves, pers, lac, f0, seed, x0, y0, nx, ny, nthreads=0) -> np.ndarray:
    out = np.empty((ny, nx), dtype=np.float64)
    _chk(lib().orc_fbm_2d(smooth, octaves, pers, lac, f0, seed & 0xFFFFFFFF, x0, y0, nx, ny,
                          _dp(out), nthreads))
    return out


def fbm_3d(smooth, octaves, pers, lac, f0, seed, x0, y0, z0, nx, ny, nz, nthreads=0) -> np.ndarray:
    out = np.empty((nz, ny, nx), dtype=np.float64)
    _chk(lib().orc_fbm_3d(smooth, octaves, pers, lac, f0, seed & 0xFFFFFFFF, x0, y0, z0, nx, ny, nz,
                          _dp(out), nthreads))
    return out


def fbm_points_2d(smooth, octaves, pers, lac, f0, seed, X, Y, nthreads=0) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.int64)
    Y = np.ascontiguousarray(Y, dtype=np.int64)
    out = np.empty(X.shape[0], dtype=np.float64)
    _chk(lib().orc_fbm_points_2d(smooth, octaves, pers, lac, f0, seed & 0xFFFFFFFF, _ip(X), _ip(Y),
                                 X.shape[0], _dp(out), nthreads))
    return out


def fbm_points_3d(smooth, octaves, pers, lac, f0, seed, X, Y, Z, nthreads=0) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.int64)
    Y = np.ascontiguousarray(Y, dtype=np.int64)
    Z = np.ascontiguousarray(Z, dtype=np.int64)
    out = np.empty(X.shape[0], dtype=np.float64)
    _chk(lib().orc_fbm_points_3d(smooth, octaves, pers, lac, f0, seed & 0xFFFFFFFF, _ip(X), _ip(Y),
                                 _ip(Z), X.shape[0], _dp(out), nthreads))
    return out


def perlin_2d(fade_order, octaves, pers, lac, f0, seed, x0, y0, nx, ny, nthreads=0) -> np.ndarray:
    out = np.empty((ny, nx), dtype=np.float64)
    _chk(lib().orc_perlin_2d(fade_order, octaves, pers, lac, f0, seed & 0xFFFFFFFF, x0, y0, nx, ny,
                             _dp(out), nthreads))
    return out


# --- zero-gradient D2M1N3 (Sec. 3.3) ------------------------------------------

def height2(key: int) -> float:
    """Node height of the zero-gradient model, uniform on [-1, 1)."""
    return float(lib().orc_height2(key & 0xFFFFFFFF))


def zg_cell(h, x: float, y: float) -> float:
    """Zero-gradient D2M1N3 cell at local (x, y); h = (h00, h10, h01, h11)."""
    hh = np.ascontiguousarray(h, dtype=np.float64).reshape(4)
    return float(lib().orc_zg_cell(_dp(hh), x, y))


def zg_fbm_2d(octaves, pers, lac, f0, seed, x0, y0, nx, ny, nthreads=0) -> np.ndarray:
    out = np.empty((ny, nx), dtype=np.float64)
    _chk(lib().orc_zg_fbm_2d(octaves, pers, lac, f0, seed & 0xFFFFFFFF, x0, y0, nx, ny, _dp(out), nthreads))
    return out


def zg_fbm_points_2d(octaves, pers, lac, f0, seed, X, Y, nthreads=0) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.int64)
    Y = np.ascontiguousarray(Y, dtype=np.int64)
    out = np.empty(X.shape[0], dtype=np.float64)
    _chk(lib().orc_zg_fbm_points_2d(octaves, pers, lac, f0, seed & 0xFFFFFFFF, _ip(X), _ip(Y), X.shape[0],
                                    _dp(out), nthreads))
    return out


# --- heights and weighted gradients (Sec. 3.1, Sec. 4 w) -------------------------

def height2_second(key: int) -> float:
    """Node height of the height-and-gradient model (the key's second word)."""
    return float(lib().orc_height2_second(key & 0xFFFFFFFF))


def hg_cell(smooth: int, h, grad, w: float, x: float, y: float) -> float:
    hh = np.ascontiguousarray(h, dtype=np.float64).reshape(4)
    g = np.ascontiguousarray(grad, dtype=np.float64).reshape(8)
    return float(lib().orc_hg_cell(smooth, _dp(hh), _dp(g), w, x, y))


def hg_fbm_2d(smooth, octaves, pers, lac, f0, w, seed, x0, y0, nx, ny, nthreads=0) -> np.ndarray:
    out = np.empty((ny, nx), dtype=np.float64)
    _chk(lib().orc_hg_fbm_2d(smooth, octaves, pers, lac, f0, w, seed & 0xFFFFFFFF, x0, y0, nx, ny, _dp(out),
                             nthreads))
    return out


def hg_fbm_points_2d(smooth, octaves, pers, lac, f0, w, seed, X, Y, nthreads=0) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.int64)
    Y = np.ascontiguousarray(Y, dtype=np.int64)
    out = np.empty(X.shape[0], dtype=np.float64)
    _chk(lib().orc_hg_fbm_points_2d(smooth, octaves, pers, lac, f0, w, seed & 0xFFFFFFFF, _ip(X), _ip(Y), X.shape[0],
                                    _dp(out), nthreads))
    return out


def simplex_at(ux: float, uy: float, octave: int, seed: int) -> float:
    """Simplex-lattice gradient noise of one octave at lattice coordinates (ux, uy)."""
    return float(lib().orc_simplex_at(ux, uy, octave, seed & 0xFFFFFFFF))


def simplex_2d(octaves, pers, lac, f0, seed, x0, y0, nx, ny, nthreads=0) -> np.ndarray:
    out = np.empty((ny, nx), dtype=np.float64)
    _chk(lib().orc_simplex_2d(octaves, pers, lac, f0, seed & 0xFFFFFFFF, x0, y0, nx, ny, _dp(out), nthreads))
    return out


def height3(key: int) -> float:
    """Node height of the 3D height-and-gradient model (the key's third word)."""
    return float(lib().orc_height3(key & 0xFFFFFFFF))


def hg_cell_3d(smooth: int, h, grad, w: float, x: float, y: float, z: float) -> float:
    hh = np.ascontiguousarray(h, dtype=np.float64).reshape(8)
    g = np.ascontiguousarray(grad, dtype=np.float64).reshape(24)
    return float(lib().orc_hg_cell_3d(smooth, _dp(hh), _dp(g), w, x, y, z))


def hg_fbm_3d(smooth, octaves, pers, lac, f0, w, seed, x0, y0, z0, nx, ny, nz, nthreads=0) -> np.ndarray:
    out = np.empty((nz, ny, nx), dtype=np.float64)
    _chk(lib().orc_hg_fbm_3d(smooth, octaves, pers, lac, f0, w, seed & 0xFFFFFFFF, x0, y0, z0, nx, ny, nz, _dp(out),
                             nthreads))
    return out


def hg_fbm_points_3d(smooth, octaves, pers, lac, f0, w, seed, X, Y, Z, nthreads=0) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.int64)
    Y = np.ascontiguousarray(Y, dtype=np.int64)
    Z = np.ascontiguousarray(Z, dtype=np.int64)
    out = np.empty(X.shape[0], dtype=np.float64)
    _chk(lib().orc_hg_fbm_points_3d(smooth, octaves, pers, lac, f0, w, seed & 0xFFFFFFFF, _ip(X), _ip(Y), _ip(Z),
                                    X.shape[0], _dp(out), nthreads))
    return out


# --- analytic gradient (Sec. 5.1 gradient maps) ----------------------------------

MODELS = {"gradient": 0, "zero_gradient": 1, "height_gradient": 2}


def basis_deriv(smooth: int, t: float):
    db0 = np.zeros(2)
    db1 = np.zeros(2)
    lib().orc_basis_deriv(smooth, t, _dp(db0), _dp(db1))
    return db0, db1


def cell_2d_grad(model, smooth, h, grad, w, x, y) -> np.ndarray:
    """(value, d/dtx, d/dty) of one cell of the model."""
    hh = np.ascontiguousarray(h, dtype=np.float64).reshape(4)
    g = np.ascontiguousarray(grad, dtype=np.float64).reshape(8)
    out = np.zeros(3)
    lib().orc_cell_2d_grad(MODELS.get(model, model), smooth, _dp(hh), _dp(g), w, x, y, _dp(out))
    return out


def fbm_2d_grad(model, smooth, octaves, pers, lac, f0, w, seed, x0, y0, nx, ny, nthreads=0):
    """(H, dH/dX, dH/dY), each (ny, nx)."""
    outs = [np.empty((ny, nx), dtype=np.float64) for _ in range(3)]
    _chk(lib().orc_fbm_2d_grad(MODELS.get(model, model), smooth, octaves, pers, lac, f0, w, seed & 0xFFFFFFFF, x0, y0,
                               nx, ny, _dp(outs[0]), _dp(outs[1]), _dp(outs[2]), nthreads))
    return tuple(outs)


def max_threads() -> int:
    return int(lib().orc_max_threads())

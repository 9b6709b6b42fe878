"""GPU parity: every stage of the HIP path against the FP64 oracle, through the C ABI.

Bar (fixed in advance from the arithmetic):
* coordinate step: int64 cells bit-exact, FP32 fractions equal to the oracle's FP64
  fraction rounded to FP32 (same FP64 operations on both sides);
* lattice: uint32 keys bit-exact; gradients within 2^-20 of the FP64 map;
* per-cell coefficients: within 2e-6 * (sum of |terms|) of the FP64 expansion;
* fields: max |H_gpu - H_oracle| <= 1e-5 * A, A = sum_o p^o (total amplitude).
"""
import math

import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
import paper_1610_03525_amd as ptg  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _amp_total(p, n):
    return sum(p ** o for o in range(n))


def _sync():
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------------
# a1 coordinate step
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("f0,lac,x0", [
    (1 / 512, 2.0, 0), (1 / 512, 2.0, -3 * 2 ** 20 - 7), (8 / 256, 2.0, 2 ** 33 + 5),
    (0.013, 1.87, -123456789), (1 / 16384 * 32, 2.0, (2 ** 24 - 3) * 512),
])
def test_coords_bit_exact(f0, lac, x0):
    n, octs = 777, 8
    cells = torch.empty((octs, n), dtype=torch.int64, device=DEV)
    frac = torch.empty((octs, n), dtype=torch.float32, device=DEV)
    ptg.coords(f0, lac, octs, x0, cells, frac)
    _sync()
    cells, frac = cells.cpu().numpy(), frac.cpu().numpy()
    freq, _ = O.octave_params(f0, lac, 0.5, octs)
    for o in range(octs):
        for i in range(0, n, 7):
            c, t = O.coord(x0 + i, freq[o])
            assert cells[o, i] == c
            assert frac[o, i] == np.float32(t)


# ---------------------------------------------------------------------------------
# a2 lattice hash (K1)
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("seed,octave,ix0,iy0", [
    (1, 0, 0, 0), (2, 3, -40, -17), (0xDEADBEEF, 9, -3 * 2 ** 20 - 7, 2 ** 33 + 5),
    (3, 15, (2 ** 24 - 3), -(2 ** 24 - 5)), (0, 2, -(2 ** 46), 2 ** 46 - 64),
])
def test_lattice2d_keys_bit_exact(seed, octave, ix0, iy0):
    nx, ny = 37, 29
    keys = torch.empty((ny, nx), dtype=torch.int32, device=DEV)
    grad = torch.empty((2, ny, nx), dtype=torch.float32, device=DEV)
    ptg.lattice_2d(seed, octave, ix0, iy0, keys, grad)
    _sync()
    k = keys.cpu().numpy().view(np.uint32)
    g = grad.cpu().numpy()
    ref = O.keys2_box(ix0, iy0, nx, ny, octave, seed)
    np.testing.assert_array_equal(k, ref)
    worst = 0.0
    for j in range(ny):
        for i in range(nx):
            gr = O.grad2(int(ref[j, i]))
            worst = max(worst, abs(g[0, j, i] - gr[0]), abs(g[1, j, i] - gr[1]))
    assert worst <= 2 ** -20, worst


@pytest.mark.parametrize("seed,octave,ix0,iy0,iz0", [
    (1, 0, 0, 0, 0), (7, 5, -9, 13, -2 ** 33), (0xFFFFFFFF, 12, 2 ** 40, -(2 ** 40), 77),
])
def test_lattice3d_keys_bit_exact(seed, octave, ix0, iy0, iz0):
    nx, ny, nz = 11, 7, 5
    keys = torch.empty((nz, ny, nx), dtype=torch.int32, device=DEV)
    sec = torch.empty((nz, ny, nx), dtype=torch.int32, device=DEV)
    grad = torch.empty((3, nz, ny, nx), dtype=torch.float32, device=DEV)
    ptg.lattice_3d(seed, octave, ix0, iy0, iz0, keys, sec, grad)
    _sync()
    k = keys.cpu().numpy().view(np.uint32)
    s = sec.cpu().numpy().view(np.uint32)
    g = grad.cpu().numpy()
    ref = O.keys3_box(ix0, iy0, iz0, nx, ny, nz, octave, seed)
    np.testing.assert_array_equal(k, ref)
    worst = 0.0
    for q in np.ndindex(nz, ny, nx):
        assert s[q] == O.key3_second(int(ref[q]))
        gr = O.grad3(int(ref[q]))
        worst = max(worst, max(abs(g[(a,) + q] - gr[a]) for a in range(3)))
    assert worst <= 2 ** -20, worst


# ---------------------------------------------------------------------------------
# a3 per-cell coefficients (K2)
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("smooth", [1, 2])
def test_cells2d_against_oracle(smooth):
    seed, octave, ix0, iy0, nnx, nny = 5, 2, -21, 1000, 35, 19
    amp = 0.25
    grad = torch.empty((2, nny, nnx), dtype=torch.float32, device=DEV)
    ptg.lattice_2d(seed, octave, ix0, iy0, None, grad)
    n1 = 2 * smooth + 2
    coeff = torch.empty((nny - 1, nnx - 1, n1, n1), dtype=torch.float32, device=DEV)
    ptg.cells_2d(smooth, grad, amp, coeff)
    _sync()
    c = coeff.cpu().numpy()
    for cj in range(nny - 1):
        for ci in range(nnx - 1):
            g = np.array([O.grad2(O.key2(ix0 + ci + dx, iy0 + cj + dy, octave, seed))
                          for dy in (0, 1) for dx in (0, 1)])
            ref = amp * O.coeffs_2d(smooth, g)
            tol = 2e-6 * amp * (16 if smooth == 1 else 200)
            assert np.max(np.abs(c[cj, ci] - ref)) <= tol


@pytest.mark.parametrize("smooth", [1, 2])
def test_cells3d_against_oracle(smooth):
    seed, octave, ix0, iy0, iz0, nn = 9, 1, 3, -4, 5, 6
    grad = torch.empty((3, nn, nn, nn), dtype=torch.float32, device=DEV)
    ptg.lattice_3d(seed, octave, ix0, iy0, iz0, None, None, grad)
    n1 = 2 * smooth + 2
    coeff = torch.empty((nn - 1, nn - 1, nn - 1, n1, n1, n1), dtype=torch.float32, device=DEV)
    ptg.cells_3d(smooth, grad, 1.0, coeff)
    _sync()
    c = coeff.cpu().numpy()
    for ck, cj, ci in [(0, 0, 0), (4, 4, 4), (2, 1, 3), (1, 4, 0)]:
        g = np.array([O.grad3(O.key3(ix0 + ci + dx, iy0 + cj + dy, iz0 + ck + dz, octave, seed))
                      for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)])
        ref = O.coeffs_3d(smooth, g)
        tol = 2e-6 * (64 if smooth == 1 else 3000)
        assert np.max(np.abs(c[ck, cj, ci] - ref)) <= tol


# Stage kernels over several workgroups: K1 covers 256 node columns x 16 node rows per
# workgroup (3D rows wrap from one j to the next k inside a workgroup), K2 64 x 4 cells
# (2D) and 64 x 2 x 2 cells (3D); ragged last workgroups on every axis, and K2 output
# buffers that are and are not 16-byte aligned (vector and scalar stores).
def test_lattice2d_multi_workgroup():
    seed, octave, ix0, iy0, nx, ny = 77, 4, -(2 ** 35) - 130, 2 ** 21 + 3, 300, 37
    keys = torch.empty((ny, nx), dtype=torch.int32, device=DEV)
    grad = torch.empty((2, ny, nx), dtype=torch.float32, device=DEV)
    ptg.lattice_2d(seed, octave, ix0, iy0, keys, grad)
    h = torch.empty((ny, nx), dtype=torch.float32, device=DEV)
    ptg.heights_2d(seed, octave, ix0, iy0, h)
    _sync()
    ref = O.keys2_box(ix0, iy0, nx, ny, octave, seed)
    np.testing.assert_array_equal(keys.cpu().numpy().view(np.uint32), ref)
    g, hh = grad.cpu().numpy(), h.cpu().numpy()
    worst = 0.0
    for j in range(0, ny, 3):
        for i in range(nx):
            gr = O.grad2(int(ref[j, i]))
            worst = max(worst, abs(g[0, j, i] - gr[0]), abs(g[1, j, i] - gr[1]))
            assert hh[j, i] == np.float32(O.height2(int(ref[j, i])))
    assert worst <= 2 ** -20, worst


def test_lattice3d_rows_wrap_inside_workgroup():
    seed, octave, ix0, iy0, iz0, nx, ny, nz = 0xC0FFEE, 3, 2 ** 33 - 100, -7, 2 ** 30, 260, 5, 7
    keys = torch.empty((nz, ny, nx), dtype=torch.int32, device=DEV)
    sec = torch.empty((nz, ny, nx), dtype=torch.int32, device=DEV)
    grad = torch.empty((3, nz, ny, nx), dtype=torch.float32, device=DEV)
    ptg.lattice_3d(seed, octave, ix0, iy0, iz0, keys, sec, grad)
    _sync()
    ref = O.keys3_box(ix0, iy0, iz0, nx, ny, nz, octave, seed)
    np.testing.assert_array_equal(keys.cpu().numpy().view(np.uint32), ref)
    s, g = sec.cpu().numpy().view(np.uint32), grad.cpu().numpy()
    worst = 0.0
    for q in np.ndindex(nz, ny, nx):
        if q[2] % 7 and q[2] < nx - 3:
            continue  # every 7th column and the last three
        assert s[q] == O.key3_second(int(ref[q]))
        gr = O.grad3(int(ref[q]))
        worst = max(worst, max(abs(g[(a,) + q] - gr[a]) for a in range(3)))
    assert worst <= 2 ** -20, worst


def _unaligned(n, dtype=torch.float32):
    """A contiguous device buffer of n elements whose address is 4 bytes past 16-byte alignment."""
    base = torch.empty(n + 4, dtype=dtype, device=DEV)
    assert base.data_ptr() % 16 == 0
    return base[1:1 + n]


@pytest.mark.parametrize("smooth", [1, 2])
@pytest.mark.parametrize("aligned", [True, False])
def test_cells2d_multi_workgroup(smooth, aligned):
    seed, octave, ix0, iy0, nnx, nny = 11, 5, 2 ** 40 - 70, -(2 ** 20), 140, 7
    amp = 0.125
    grad = torch.empty((2, nny, nnx), dtype=torch.float32, device=DEV)
    ptg.lattice_2d(seed, octave, ix0, iy0, None, grad)
    n1 = 2 * smooth + 2
    shape = (nny - 1, nnx - 1, n1, n1)
    n = int(np.prod(shape))
    coeff = (torch.empty(n, dtype=torch.float32, device=DEV) if aligned else _unaligned(n)).view(shape)
    assert (coeff.data_ptr() % 16 == 0) == aligned
    ptg.cells_2d(smooth, grad, amp, coeff)
    _sync()
    c = coeff.cpu().numpy()
    tol = 2e-6 * amp * (16 if smooth == 1 else 200)
    for cj in range(nny - 1):
        for ci in range(nnx - 1):
            g = np.array([O.grad2(O.key2(ix0 + ci + dx, iy0 + cj + dy, octave, seed))
                          for dy in (0, 1) for dx in (0, 1)])
            assert np.max(np.abs(c[cj, ci] - amp * O.coeffs_2d(smooth, g))) <= tol, (cj, ci)


@pytest.mark.parametrize("smooth", [1, 2])
@pytest.mark.parametrize("aligned", [True, False])
def test_cells3d_multi_workgroup(smooth, aligned):
    seed, octave, ix0, iy0, iz0, nnx, nny, nnz = 13, 2, -65, 2 ** 31, -(2 ** 33), 67, 4, 4
    amp = 0.5
    grad = torch.empty((3, nnz, nny, nnx), dtype=torch.float32, device=DEV)
    ptg.lattice_3d(seed, octave, ix0, iy0, iz0, None, None, grad)
    n1 = 2 * smooth + 2
    shape = (nnz - 1, nny - 1, nnx - 1, n1, n1, n1)
    n = int(np.prod(shape))
    coeff = (torch.empty(n, dtype=torch.float32, device=DEV) if aligned else _unaligned(n)).view(shape)
    ptg.cells_3d(smooth, grad, amp, coeff)
    _sync()
    c = coeff.cpu().numpy()
    tol = 2e-6 * amp * (64 if smooth == 1 else 3000)
    for ck in range(nnz - 1):
        for cj in range(nny - 1):
            for ci in list(range(0, nnx - 1, 5)) + [62, 63, 64, 65]:
                g = np.array([O.grad3(O.key3(ix0 + ci + dx, iy0 + cj + dy, iz0 + ck + dz, octave, seed))
                              for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)])
                assert np.max(np.abs(c[ck, cj, ci] - amp * O.coeffs_3d(smooth, g))) <= tol, (ck, cj, ci)


# ---------------------------------------------------------------------------------
# a1-a5 fields (K3)
# ---------------------------------------------------------------------------------
def _gpu_fbm2(nx, ny, x0, y0, dtype=torch.float32, pitch=None, **kw):
    if pitch is None:
        out = torch.empty((ny, nx), dtype=dtype, device=DEV)
    else:
        out = torch.full((ny, pitch), 7.0, dtype=dtype, device=DEV)[:, :nx]
    ptg.fbm_2d(out, x0=x0, y0=y0, **kw)
    _sync()
    return out


@pytest.mark.parametrize("smooth", [1, 2])
@pytest.mark.parametrize("seed", [1, 2, 3, 0xDEADBEEF])
@pytest.mark.parametrize("origin", [(0, 0), (-3 * 2 ** 20 - 7, 2 ** 33 + 5)])
def test_fbm2d_256_4oct_full_field(smooth, seed, origin):
    """2D 256x256, 4 octaves, base lattice 8x8, L = 2, p = 0.5 (the correctness workload)."""
    kw = dict(smoothness=smooth, octaves=4, persistence=0.5, lacunarity=2.0, base_freq=8 / 256, seed=seed)
    g = _gpu_fbm2(256, 256, *origin, **kw).cpu().numpy().astype(np.float64)
    ref = O.fbm_2d(smooth, 4, 0.5, 2.0, 8 / 256, seed, origin[0], origin[1], 256, 256)
    err = np.max(np.abs(g - ref))
    assert err <= 1e-5 * _amp_total(0.5, 4), err


@pytest.mark.parametrize("nx,ny,pitch", [(1, 1, None), (67, 45, None), (130, 3, 200), (5, 131, 9), (64, 64, 64)])
def test_fbm2d_ragged_edges_and_pitch(nx, ny, pitch):
    kw = dict(smoothness=1, octaves=5, persistence=0.5, lacunarity=2.0, base_freq=1 / 16, seed=11)
    out = _gpu_fbm2(nx, ny, -70, 33, pitch=pitch, **kw)
    g = out.cpu().numpy().astype(np.float64)
    ref = O.fbm_2d(1, 5, 0.5, 2.0, 1 / 16, 11, -70, 33, nx, ny)
    assert np.max(np.abs(g - ref)) <= 1e-5 * _amp_total(0.5, 5)
    if pitch is not None:
        full = out.as_strided((ny, pitch), (pitch, 1)).cpu().numpy()
        assert np.all(full[:, nx:] == 7.0)  # nothing written past the row


@pytest.mark.parametrize("smooth", [1, 2])
def test_fbm2d_non_dyadic_parameters(smooth):
    kw = dict(smoothness=smooth, octaves=6, persistence=0.61, lacunarity=1.87, base_freq=0.013, seed=77)
    x0, y0 = -123456789, 987654321
    g = _gpu_fbm2(150, 97, x0, y0, **kw).cpu().numpy().astype(np.float64)
    ref = O.fbm_2d(smooth, 6, 0.61, 1.87, 0.013, 77, x0, y0, 150, 97)
    assert np.max(np.abs(g - ref)) <= 1e-5 * _amp_total(0.61, 6)


def test_fbm2d_finest_lattice_one_cell_per_sample():
    kw = dict(smoothness=1, octaves=6, persistence=0.5, lacunarity=2.0, base_freq=1 / 32, seed=4)
    g = _gpu_fbm2(96, 80, 5, -5, **kw).cpu().numpy().astype(np.float64)
    ref = O.fbm_2d(1, 6, 0.5, 2.0, 1 / 32, 4, 5, -5, 96, 80)
    assert np.max(np.abs(g - ref)) <= 1e-5 * _amp_total(0.5, 6)


def test_fbm2d_sixteen_octaves_large_offset():
    kw = dict(smoothness=2, octaves=16, persistence=0.5, lacunarity=2.0, base_freq=2.0 ** -15, seed=12)
    x0, y0 = 2 ** 45 + 3, -(2 ** 44) - 1
    g = _gpu_fbm2(100, 70, x0, y0, **kw).cpu().numpy().astype(np.float64)
    ref = O.fbm_2d(2, 16, 0.5, 2.0, 2.0 ** -15, 12, x0, y0, 100, 70)
    assert np.max(np.abs(g - ref)) <= 1e-5 * _amp_total(0.5, 16)


def test_fbm2d_fp16_output():
    kw = dict(smoothness=1, octaves=4, persistence=0.5, lacunarity=2.0, base_freq=8 / 256, seed=1)
    g = _gpu_fbm2(256, 256, 0, 0, dtype=torch.float16, **kw).cpu().numpy().astype(np.float64)
    ref = O.fbm_2d(1, 4, 0.5, 2.0, 8 / 256, 1, 0, 0, 256, 256)
    # FP16 rounding of |H| < 1: half an ulp at [0.5, 1) is 2^-12
    assert np.max(np.abs(g - ref)) <= 2.0 ** -12 + 1e-5 * 1.875


def test_fbm2d_tiles_stitch_bit_exactly():
    """A tile equals the matching crop of a larger field (per-sample arithmetic does not
    depend on where the tile boundaries fall)."""
    kw = dict(smoothness=1, octaves=6, persistence=0.5, lacunarity=2.0, base_freq=1 / 64, seed=3)
    big = _gpu_fbm2(300, 200, -3 * 2 ** 20 - 7 - 5, 2 ** 33 + 5 - 9, **kw)
    small = _gpu_fbm2(130, 70, -3 * 2 ** 20 - 7, 2 ** 33 + 5, **kw)
    assert torch.equal(big[9:79, 5:135], small)


def test_fbm2d_8192_8oct_sampled():
    """2D 8192x8192, 8 octaves, base lattice 16x16 (the throughput workload): oracle at
    sampled samples + one full 64x64 tile + the last row/column."""
    kw = dict(smoothness=1, octaves=8, persistence=0.5, lacunarity=2.0, base_freq=16 / 8192, seed=1)
    out = _gpu_fbm2(8192, 8192, 0, 0, **kw)
    g = out.cpu().numpy()
    rng = np.random.default_rng(2024)
    X = rng.integers(0, 8192, size=20000)
    Y = rng.integers(0, 8192, size=20000)
    X = np.concatenate([X, np.arange(8192), np.full(8192, 8191), np.arange(4096, 4160).repeat(64)])
    Y = np.concatenate([Y, np.full(8192, 8191), np.arange(8192), np.tile(np.arange(1000, 1064), 64)])
    ref = O.fbm_points_2d(1, 8, 0.5, 2.0, 16 / 8192, 1, X, Y)
    err = np.max(np.abs(g[Y, X].astype(np.float64) - ref))
    assert err <= 1e-5 * _amp_total(0.5, 8), err


# ---------------------------------------------------------------------------------
# 3D
# ---------------------------------------------------------------------------------
def _gpu_fbm3(nx, ny, nz, x0, y0, z0, **kw):
    out = torch.empty((nz, ny, nx), dtype=torch.float32, device=DEV)
    ptg.fbm_3d(out, x0=x0, y0=y0, z0=z0, **kw)
    _sync()
    return out


@pytest.mark.parametrize("smooth", [1, 2])
@pytest.mark.parametrize("dims,origin", [((64, 40, 24), (0, 0, 0)), ((70, 9, 11), (-5, 2 ** 33 + 1, -(2 ** 20)))])
def test_fbm3d_full_field(smooth, dims, origin):
    kw = dict(smoothness=smooth, octaves=6, persistence=0.5, lacunarity=2.0, base_freq=1 / 64, seed=1)
    g = _gpu_fbm3(*dims, *origin, **kw).cpu().numpy().astype(np.float64)
    ref = O.fbm_3d(smooth, 6, 0.5, 2.0, 1 / 64, 1, *origin, *dims)
    err = np.max(np.abs(g - ref))
    assert err <= 1e-5 * _amp_total(0.5, 6), err


def test_fbm3d_512_6oct_c2_sampled():
    """3D 512^3, 6 octaves, base lattice 8^3, C2 quintic: sampled against the oracle."""
    kw = dict(smoothness=2, octaves=6, persistence=0.5, lacunarity=2.0, base_freq=8 / 512, seed=1)
    out = _gpu_fbm3(512, 512, 512, 0, 0, 0, **kw)
    rng = np.random.default_rng(7)
    n = 20000
    X, Y, Z = (rng.integers(0, 512, size=n) for _ in range(3))
    g = out[torch.from_numpy(Z).to(DEV), torch.from_numpy(Y).to(DEV), torch.from_numpy(X).to(DEV)].cpu().numpy()
    ref = O.fbm_points_3d(2, 6, 0.5, 2.0, 8 / 512, 1, X, Y, Z)
    err = np.max(np.abs(g.astype(np.float64) - ref))
    assert err <= 1e-5 * _amp_total(0.5, 6), err


def test_fbm3d_non_dyadic_and_ragged():
    kw = dict(smoothness=1, octaves=4, persistence=0.7, lacunarity=2.3, base_freq=0.021, seed=99)
    g = _gpu_fbm3(33, 17, 10, 1000, -2000, 3000, **kw).cpu().numpy().astype(np.float64)
    ref = O.fbm_3d(1, 4, 0.7, 2.3, 0.021, 99, 1000, -2000, 3000, 33, 17, 10)
    assert np.max(np.abs(g - ref)) <= 1e-5 * _amp_total(0.7, 4)


# Each dyadic ladder below selects a different specialisation of the 3D strip kernel
# (finest period 2, 4, 8, >= 16; no coarse octave; coarse octaves with and without a basis
# table) or its fallback (ladders reaching period 1); every field is an unaligned window
# with ragged edges against 64 x 8 x 16 blocks, several blocks deep in z.
@pytest.mark.parametrize("path", ["auto", "general"])
@pytest.mark.parametrize("smooth", [1, 2])
@pytest.mark.parametrize("f0,octs,origin,shape", [
    (1 / 64, 7, (-5, 2 ** 33 + 1, -(2 ** 20) + 3), (70, 19, 13)),   # periods 64..1
    (1 / 64, 6, (3, -11, 7), (129, 9, 6)),                          # periods 64..2
    (1 / 32, 4, (61, 5, -1), (67, 17, 9)),                          # periods 32..4
    (1 / 256, 6, (-300, 77, 1000), (130, 12, 5)),                   # periods 256..8
    (1 / 4, 3, (2, 3, 1), (65, 8, 4)),                              # periods 4..1, no coarse octave
    (2.0 ** -20, 5, (2 ** 40 + 9, -(2 ** 41) - 3, 2 ** 39), (66, 10, 3)),  # periods 2^20..2^16
    (1 / 2, 2, (0, 0, 0), (40, 6, 5)),                              # periods 2, 1: general kernel
    (1 / 8, 3, (5, -3, 17), (70, 19, 37)),                          # periods 8, 4, 2: no coarse octave
    (1 / 16, 4, (-100, 50, -33), (90, 25, 40)),                     # periods 16..2
    (1 / 512, 8, (7, -1000, 2 ** 36 + 5), (65, 9, 20)),            # periods 512..4 (512: no table)
    (1 / 128, 4, (-64, 8, 16), (128, 16, 32)),                      # periods 128..16, aligned blocks
])
def test_fbm3d_ladders_against_oracle(path, smooth, f0, octs, origin, shape):
    kw = dict(smoothness=smooth, octaves=octs, persistence=0.5, lacunarity=2.0, base_freq=f0, seed=21, path=path)
    g = _gpu_fbm3(*shape, *origin, **kw).cpu().numpy().astype(np.float64)
    ref = O.fbm_3d(smooth, octs, 0.5, 2.0, f0, 21, *origin, *shape)
    err = np.max(np.abs(g - ref))
    assert err <= 1e-5 * _amp_total(0.5, octs), err


def test_fbm3d_dyadic_path_rejects_ladders_it_cannot_take():
    out = torch.empty((4, 4, 4), dtype=torch.float32, device=DEV)
    with pytest.raises(ptg.PtgError):
        ptg.fbm_3d(out, base_freq=1 / 2, octaves=2, path="dyadic")
    with pytest.raises(ptg.PtgError):
        ptg.fbm_3d(out, base_freq=0.03, octaves=2, path="dyadic")


def test_fbm3d_fp16_output_and_crops():
    kw = dict(smoothness=2, octaves=6, persistence=0.5, lacunarity=2.0, base_freq=1 / 64, seed=4)
    big = _gpu_fbm3(100, 20, 10, 60, -9, 5, **kw)
    small = _gpu_fbm3(50, 7, 4, 70, -5, 8, **kw)
    assert torch.equal(big[3:7, 4:11, 10:60], small)
    h = torch.empty((10, 20, 100), dtype=torch.float16, device=DEV)
    ptg.fbm_3d(h, x0=60, y0=-9, z0=5, **kw)
    _sync()
    ref = O.fbm_3d(2, 6, 0.5, 2.0, 1 / 64, 4, 60, -9, 5, 100, 20, 10)
    assert np.max(np.abs(h.cpu().numpy().astype(np.float64) - ref)) <= 2.0 ** -12 + 1e-5 * _amp_total(0.5, 6)


def test_empty_fields_are_noops():
    out = torch.empty((0, 16), dtype=torch.float32, device=DEV)
    ptg.fbm_2d(out, base_freq=1 / 8, octaves=2)
    out3 = torch.empty((4, 0, 4), dtype=torch.float32, device=DEV)
    ptg.fbm_3d(out3, base_freq=1 / 8, octaves=2)
    _sync()


# ---------------------------------------------------------------------------------
# kernel choice: the general and the dyadic (matrix-core) K3 on the same dyadic fields
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("path", ["general", "dyadic"])
@pytest.mark.parametrize("smooth", [1, 2])
@pytest.mark.parametrize("f0,octs,origin,shape", [
    (8 / 256, 4, (-3 * 2 ** 20 - 7, 2 ** 33 + 5), (256, 256)),   # periods 32..4 (16x16x4 + 4x4x1)
    (1 / 8, 4, (13, -29), (97, 71)),                              # periods 8..1 (4x4x1 + VALU), ragged
    (2.0 ** -12, 13, (2 ** 40 + 3, -(2 ** 40) - 61), (130, 66)),  # periods 4096..1, unaligned window
])
def test_fbm2d_paths_against_oracle(path, smooth, f0, octs, origin, shape):
    kw = dict(smoothness=smooth, octaves=octs, persistence=0.5, lacunarity=2.0, base_freq=f0, seed=5, path=path)
    nx, ny = shape
    g = _gpu_fbm2(nx, ny, *origin, **kw).cpu().numpy().astype(np.float64)
    ref = O.fbm_2d(smooth, octs, 0.5, 2.0, f0, 5, origin[0], origin[1], nx, ny)
    err = np.max(np.abs(g - ref))
    assert err <= 1e-5 * _amp_total(0.5, octs), err


@pytest.mark.parametrize("smooth", [1, 2])
@pytest.mark.parametrize("f0,octs", [(2.0 ** -10, 8), (2.0 ** -11, 8), (2.0 ** -12, 8), (2.0 ** -13, 8),
                                     (2.0 ** -14, 6), (2.0 ** -6, 5), (2.0 ** -5, 6)])
def test_fbm2d_strip_finest_periods(smooth, f0, octs):
    """Finest period 8, 16, 32, 64, 512; a ladder from period 64 to 4; one from 32 to 1."""
    x0, y0, nx, ny = -77, 2 ** 35 + 13, 203, 131
    kw = dict(smoothness=smooth, octaves=octs, persistence=0.5, lacunarity=2.0, base_freq=f0, seed=3)
    g = _gpu_fbm2(nx, ny, x0, y0, **kw).cpu().numpy().astype(np.float64)
    ref = O.fbm_2d(smooth, octs, 0.5, 2.0, f0, 3, x0, y0, nx, ny)
    assert np.max(np.abs(g - ref)) <= 1e-5 * _amp_total(0.5, octs)


def test_fbm2d_dyadic_crops_bit_exact():
    kw = dict(smoothness=1, octaves=8, persistence=0.5, lacunarity=2.0, base_freq=1 / 256, seed=8, path="dyadic")
    big = _gpu_fbm2(333, 211, -1000 - 5, 5000 - 9, **kw)
    small = _gpu_fbm2(150, 77, -1000, 5000, **kw)
    assert torch.equal(big[9:86, 5:155], small)


def test_fbm2d_dyadic_rejects_non_dyadic():
    out = torch.empty((8, 8), dtype=torch.float32, device=DEV)
    with pytest.raises(ptg.PtgError):
        ptg.fbm_2d(out, base_freq=0.013, octaves=3, path="dyadic")
    with pytest.raises(ptg.PtgError):
        ptg.fbm_2d(out, base_freq=1 / 64, lacunarity=1.9, octaves=3, path="dyadic")


# ---------------------------------------------------------------------------------
# matrix-core precision form: every 4 rows x 64 columns one FP16 / BF16 MFMA with FP32
# accumulation (octaves of period >= 16 fused per quarter, the period-8 and period-4 cells);
# constant terms and periods 2, 1 in FP32; FP16 output
# ---------------------------------------------------------------------------------
# Bounds on max |err| / A and RMS / A over this window of the 16384^2 10-octave field:
# twice the full-field values measured on MI355X (tests/test_gpu_fullfield.py records them).
MFMA_BOUNDS = {("mfma_f16", "monomial"): (2.1e-4, 3.0e-5), ("mfma_f16", "centred"): (1.4e-4, 2.9e-5),
               ("mfma_f16", "hermite"): (1.4e-4, 2.9e-5), ("mfma_bf16", "monomial"): (1.2e-3, 7.8e-5),
               ("mfma_bf16", "centred"): (2.7e-4, 3.2e-5), ("mfma_bf16", "hermite"): (2.6e-4, 3.2e-5)}
# Other ladders: the a-priori bound of the form (operand rounding 2^-11 on terms of size <= 1
# times the number of terms, plus the FP16 output rounding), a factor ~4 above the estimate.
LADDER_BOUNDS = {"monomial": 2e-3, "centred": 2e-3, "hermite": 2e-3}


@pytest.mark.parametrize("form", ["mfma_f16", "mfma_bf16"])
@pytest.mark.parametrize("basis", ["monomial", "centred", "hermite"])
def test_fbm2d_vandermonde_form_error(form, basis):
    """2D fBm, 10 octaves, base lattice 32 x 32 over 16384 samples (periods 512..1), world
    offset (2^24 - 3) * 512, -(2^24 - 5) * 512 samples: a 512 x 384 window, FP16 output."""
    x0, y0 = (2 ** 24 - 3) * 512, -(2 ** 24 - 5) * 512
    nx, ny = 512, 384
    kw = dict(smoothness=1, octaves=10, persistence=0.5, lacunarity=2.0, base_freq=32 / 16384, seed=1,
              form=form, basis=basis)
    g = _gpu_fbm2(nx, ny, x0, y0, dtype=torch.float16, **kw).cpu().numpy().astype(np.float64)
    ref = O.fbm_2d(1, 10, 0.5, 2.0, 32 / 16384, 1, x0, y0, nx, ny)
    A = _amp_total(0.5, 10)
    err = np.abs(g - ref)
    mx, rms = float(err.max()) / A, float(np.sqrt(np.mean(err ** 2))) / A
    print(f"[{form}/{basis}] max/A = {mx:.3e}  rms/A = {rms:.3e}", flush=True)
    assert mx <= MFMA_BOUNDS[(form, basis)][0]
    assert rms <= MFMA_BOUNDS[(form, basis)][1]


@pytest.mark.parametrize("basis", ["monomial", "centred", "hermite"])
@pytest.mark.parametrize("f0,octs,origin,shape", [
    (1 / 64, 7, (-77, 2 ** 35 + 13), (203, 131)),      # periods 64..1, ragged window
    (1 / 256, 7, (5, -9), (130, 70)),                  # periods 256..4
    (1 / 512, 6, (2 ** 40 + 3, 64), (150, 64)),        # periods 512..16 (no period-8 / -4 cell)
    (1 / 32, 4, (13, -29), (97, 71)),                  # periods 32..4
])
def test_fbm2d_vandermonde_form_ladders(basis, f0, octs, origin, shape):
    """The precision form on ladders that reach (or stop above) periods 8, 4, 2, 1, ragged
    unaligned windows: FP16 error within the bound of the configuration above."""
    nx, ny = shape
    kw = dict(smoothness=1, octaves=octs, persistence=0.5, lacunarity=2.0, base_freq=f0, seed=7,
              form="mfma_f16", basis=basis)
    g = _gpu_fbm2(nx, ny, *origin, dtype=torch.float16, **kw).cpu().numpy().astype(np.float64)
    ref = O.fbm_2d(1, octs, 0.5, 2.0, f0, 7, origin[0], origin[1], nx, ny)
    assert np.max(np.abs(g - ref)) / _amp_total(0.5, octs) <= LADDER_BOUNDS[basis]


def test_fbm2d_vandermonde_form_crops_bit_exact():
    kw = dict(smoothness=1, octaves=9, persistence=0.5, lacunarity=2.0, base_freq=1 / 512, seed=8,
              form="mfma_bf16", basis="hermite")
    big = _gpu_fbm2(333, 211, -1000 - 5, 5000 - 9, dtype=torch.float16, **kw)
    small = _gpu_fbm2(150, 77, -1000, 5000, dtype=torch.float16, **kw)
    assert torch.equal(big[9:86, 5:155], small)


def test_fbm2d_vandermonde_form_rejects():
    out = torch.empty((8, 8), dtype=torch.float16, device=DEV)
    with pytest.raises(ptg.PtgError):
        ptg.fbm_2d(out, base_freq=0.013, octaves=3, form="mfma_f16")
    with pytest.raises(ptg.PtgError):
        ptg.fbm_2d(out, base_freq=1 / 64, octaves=3, smoothness=2, form="mfma_f16")
    with pytest.raises(ptg.PtgError):  # FP16 output only
        ptg.fbm_2d(torch.empty((8, 8), dtype=torch.float32, device=DEV), base_freq=1 / 64, octaves=3,
                   form="mfma_f16")

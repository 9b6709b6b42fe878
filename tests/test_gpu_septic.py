"""Septic cells (M = 3: derivatives up to third order constrained, C3 across faces) on the
2D strip kernel (every finest-period class) and the general kernels, and orders M = 4..6
(degree 9..13, the closed-form bases) on the general kernels, against the FP64 oracle: 2D
gradient and height-and-gradient models (dyadic and non-dyadic ladders, int64 offsets,
ragged windows), 3D, FP16 output, crops."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
import paper_1610_03525_amd as ptg  # noqa: E402

pytestmark = pytest.mark.gpu


def _amp(octaves, pers=0.5):
    return sum(pers ** o for o in range(octaves))


@pytest.mark.parametrize("path", ["auto", "general"])
@pytest.mark.parametrize("f0,lac,octaves", [
    (2.0 ** -5, 2.0, 6),    # periods 32..1 (strip: period 1 streamed)
    (2.0 ** -8, 2.0, 5),    # periods 256..16
    (2.0 ** -6, 2.0, 6),    # periods 64..2
    (2.0 ** -9, 2.0, 8),    # periods 512..4
    (2.0 ** -7, 2.0, 5),    # periods 128..8
    (2.0 ** -12, 2.0, 5),   # periods 4096..256: coarse octaves only
    (0.0137, 1.9, 5)])      # not dyadic: general kernel
def test_2d_gradient_model(path, f0, lac, octaves):
    nx, ny, x0, y0 = 190, 97, -(1 << 33) + 11, (1 << 25) + 3
    out = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    ptg.fbm_2d(out, x0=x0, y0=y0, smoothness=3, octaves=octaves, base_freq=f0, lacunarity=lac, seed=21, path=path)
    torch.cuda.synchronize()
    want = O.fbm_2d(3, octaves, 0.5, lac, f0, 21, x0, y0, nx, ny)
    assert np.max(np.abs(out.cpu().numpy() - want)) <= 1e-5 * _amp(octaves)


def test_2d_strip_kernel_takes_septic_ladders():
    assert ptg.tune_query((512, 512), smoothness=3, octaves=8, base_freq=1 / 512)[0] == "strip_2d"


def test_2d_benchmark_field_sampled():
    """8192^2, 8 octaves, base lattice 16^2, septic cells (strip kernel): sampled."""
    n = 8192
    out = torch.empty((n, n), dtype=torch.float32, device="cuda")
    ptg.fbm_2d(out, smoothness=3, octaves=8, base_freq=16 / n, seed=1)
    torch.cuda.synchronize()
    rng = np.random.default_rng(33)
    X, Y = rng.integers(0, n, 20000), rng.integers(0, n, 20000)
    got = out[torch.from_numpy(Y).cuda(), torch.from_numpy(X).cuda()].cpu().numpy()
    want = O.fbm_points_2d(3, 8, 0.5, 2.0, 16 / n, 1, X, Y)
    assert np.max(np.abs(got - want)) <= 1e-5 * _amp(8)


@pytest.mark.parametrize("path", ["auto", "general"])
@pytest.mark.parametrize("w", [0.01, 0.6])
def test_2d_height_gradient_model(path, w):
    nx, ny, x0, y0, f0, octaves = 170, 88, 5000, -77, 2.0 ** -6, 5
    out = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    ptg.fbm_2d(out, x0=x0, y0=y0, smoothness=3, octaves=octaves, base_freq=f0, seed=8, model="height_gradient",
               gradient_weight=w, path=path)
    torch.cuda.synchronize()
    want = O.hg_fbm_2d(3, octaves, 0.5, 2.0, f0, w, 8, x0, y0, nx, ny)
    assert np.max(np.abs(out.cpu().numpy() - want)) <= 1e-5 * _amp(octaves)


# Orders 4..6: the tensor Hermite cells of degree 9, 11, 13 (general kernels).
@pytest.mark.parametrize("M", [4, 5, 6])
@pytest.mark.parametrize("f0,lac,octaves", [(2.0 ** -5, 2.0, 5), (0.0137, 1.9, 4)])
def test_2d_higher_orders(M, f0, lac, octaves):
    nx, ny, x0, y0 = 150, 70, (1 << 33) - 7, -(1 << 20) + 5
    out = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    ptg.fbm_2d(out, x0=x0, y0=y0, smoothness=M, octaves=octaves, base_freq=f0, lacunarity=lac, seed=12)
    torch.cuda.synchronize()
    want = O.fbm_2d(M, octaves, 0.5, lac, f0, 12, x0, y0, nx, ny)
    assert np.max(np.abs(out.cpu().numpy() - want)) <= 1e-5 * _amp(octaves)


@pytest.mark.parametrize("M", [4, 6])
def test_higher_orders_height_gradient_and_3d(M):
    nx, ny, f0, octaves = 100, 40, 2.0 ** -4, 4
    out = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    ptg.fbm_2d(out, x0=-9, y0=13, smoothness=M, octaves=octaves, base_freq=f0, seed=3, model="height_gradient",
               gradient_weight=0.3)
    vol = torch.empty((9, 12, 70), dtype=torch.float32, device="cuda")
    ptg.fbm_3d(vol, x0=5, y0=-3, z0=2 ** 30, smoothness=M, octaves=octaves, base_freq=f0, seed=3)
    torch.cuda.synchronize()
    want = O.hg_fbm_2d(M, octaves, 0.5, 2.0, f0, 0.3, 3, -9, 13, nx, ny)
    assert np.max(np.abs(out.cpu().numpy() - want)) <= 1e-5 * _amp(octaves)
    want3 = O.fbm_3d(M, octaves, 0.5, 2.0, f0, 3, 5, -3, 2 ** 30, 70, 12, 9)
    assert np.max(np.abs(vol.cpu().numpy() - want3)) <= 1e-5 * _amp(octaves)


def test_3d():
    nx, ny, nz, octaves, f0 = 70, 19, 13, 4, 2.0 ** -4
    x0, y0, z0 = -(1 << 32) + 5, 3, (1 << 20) - 1
    out = torch.empty((nz, ny, nx), dtype=torch.float32, device="cuda")
    ptg.fbm_3d(out, x0=x0, y0=y0, z0=z0, smoothness=3, octaves=octaves, base_freq=f0, seed=5)
    torch.cuda.synchronize()
    want = O.fbm_3d(3, octaves, 0.5, 2.0, f0, 5, x0, y0, z0, nx, ny, nz)
    assert np.max(np.abs(out.cpu().numpy() - want)) <= 1e-5 * _amp(octaves)


def test_fp16_and_crops():
    kw = dict(smoothness=3, octaves=5, base_freq=2.0 ** -5, seed=2)
    full = torch.empty((128, 192), dtype=torch.float32, device="cuda")
    ptg.fbm_2d(full, x0=-64, y0=32, **kw)
    crop = torch.empty((50, 70), dtype=torch.float32, device="cuda")
    ptg.fbm_2d(crop, x0=-64 + 33, y0=32 + 17, **kw)
    half = torch.empty((128, 192), dtype=torch.float16, device="cuda")
    ptg.fbm_2d(half, x0=-64, y0=32, **kw)
    torch.cuda.synchronize()
    assert torch.equal(crop, full[17:67, 33:103])
    want = O.fbm_2d(3, 5, 0.5, 2.0, 2.0 ** -5, 2, -64, 32, 192, 128)
    got = half.float().cpu().numpy()
    assert np.all(np.abs(got - want) <= np.abs(want) * 2.0 ** -11 + 1e-5 * _amp(5))

"""Height-and-gradient model (tensor Hermite cells with random node heights and
w-weighted lattice gradients; Sec. 3.1 heights, Sec. 4 w) on the GPU against the FP64
oracle: fields within 1e-5 * A for C1 and C2 cells on the strip kernel (every
finest-period specialisation) and the general kernel, weights 0 (smoothstep value
noise), the paper's 0.01 and 0.5, FP16 output, crops equal to the full field bit for
bit, and sampled outputs of an 8192^2 8-octave field."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
import paper_1610_03525_amd as ptg  # noqa: E402

pytestmark = pytest.mark.gpu


def _field(nx, ny, x0, y0, dtype=torch.float32, **kw):
    out = torch.empty((ny, nx), dtype=dtype, device="cuda")
    ptg.fbm_2d(out, x0=x0, y0=y0, model="height_gradient", **kw)
    torch.cuda.synchronize()
    return out


def _amp(octaves, pers=0.5):
    return sum(pers ** o for o in range(octaves))


LADDERS = [(2.0 ** -5, 6), (2.0 ** -5, 5), (2.0 ** -5, 4), (2.0 ** -6, 4), (2.0 ** -6, 3), (2.0 ** -6, 2),
           (2.0 ** -8, 3)]


@pytest.mark.parametrize("M", [1, 2])
@pytest.mark.parametrize("f0,octaves", LADDERS)
@pytest.mark.parametrize("path", ["dyadic", "general"])
def test_field_matches_oracle(M, f0, octaves, path):
    nx, ny, x0, y0, seed, w = 200, 131, (1 << 33) - 29, -(1 << 22) + 3, 99, 0.01
    got = _field(nx, ny, x0, y0, smoothness=M, octaves=octaves, base_freq=f0, seed=seed, gradient_weight=w,
                 path=path).cpu().numpy()
    want = O.hg_fbm_2d(M, octaves, 0.5, 2.0, f0, w, seed, x0, y0, nx, ny)
    assert np.max(np.abs(got - want)) <= 1e-5 * _amp(octaves)


@pytest.mark.parametrize("M", [1, 2])
@pytest.mark.parametrize("w", [0.0, 0.5, -1.3])
@pytest.mark.parametrize("path", ["dyadic", "general"])
def test_gradient_weights(M, w, path):
    nx, ny, f0, octaves = 130, 70, 2.0 ** -5, 4
    got = _field(nx, ny, -5, 17, smoothness=M, octaves=octaves, base_freq=f0, seed=3, gradient_weight=w,
                 path=path).cpu().numpy()
    want = O.hg_fbm_2d(M, octaves, 0.5, 2.0, f0, w, 3, -5, 17, nx, ny)
    assert np.max(np.abs(got - want)) <= 1e-5 * _amp(octaves) * max(1.0, abs(w))


@pytest.mark.parametrize("M", [1, 2])
def test_general_ladders_match_oracle(M):
    nx, ny, x0, y0, f0, lac, pers, octaves = 150, 77, 12345, -(1 << 30) + 1, 0.0137, 1.9, 0.55, 5
    got = _field(nx, ny, x0, y0, smoothness=M, octaves=octaves, base_freq=f0, lacunarity=lac, persistence=pers,
                 seed=7).cpu().numpy()
    want = O.hg_fbm_2d(M, octaves, pers, lac, f0, 0.01, 7, x0, y0, nx, ny)
    assert np.max(np.abs(got - want)) <= 1e-5 * _amp(octaves, pers)


def test_dyadic_path_rejects_ladders_the_strip_kernel_does_not_take():
    with pytest.raises(ptg.PtgError) as e:
        _field(64, 64, 0, 0, octaves=4, base_freq=2.0 ** -4, path="dyadic")  # periods 16..2
    assert e.value.code == ptg.PTG_EINVAL
    auto = _field(64, 64, 0, 0, octaves=4, base_freq=2.0 ** -4).cpu().numpy()  # general kernel
    want = O.hg_fbm_2d(1, 4, 0.5, 2.0, 2.0 ** -4, 0.01, 1, 0, 0, 64, 64)
    assert np.max(np.abs(auto - want)) <= 1e-5 * _amp(4)


def test_fp16_output_within_its_rounding():
    nx, ny, f0, octaves = 256, 64, 2.0 ** -6, 5
    got = _field(nx, ny, 0, 0, dtype=torch.float16, octaves=octaves, base_freq=f0, seed=3).float().cpu().numpy()
    want = O.hg_fbm_2d(1, octaves, 0.5, 2.0, f0, 0.01, 3, 0, 0, nx, ny)
    assert np.all(np.abs(got - want) <= np.abs(want) * 2.0 ** -11 + 1e-5 * _amp(octaves))


@pytest.mark.parametrize("M", [1, 2])
def test_crops_equal_the_full_field(M):
    kw = dict(smoothness=M, octaves=6, base_freq=2.0 ** -5, seed=11, gradient_weight=0.2)
    full = _field(256, 192, -64, 128, **kw)
    for (cx, cy, w, h) in ((0, 0, 256, 192), (3, 5, 77, 61), (64, 64, 128, 64), (200, 150, 56, 42)):
        crop = _field(w, h, -64 + cx, 128 + cy, **kw)
        assert torch.equal(crop, full[cy:cy + h, cx:cx + w])


def test_benchmark_size_field_sampled():
    n, octaves, f0 = 8192, 8, 16 / 8192
    out = _field(n, n, 0, 0, octaves=octaves, base_freq=f0, seed=1)
    rng = np.random.default_rng(9)
    i = rng.integers(0, n, 4000)
    j = rng.integers(0, n, 4000)
    got = out[torch.as_tensor(j, device="cuda"), torch.as_tensor(i, device="cuda")].cpu().numpy()
    want = O.hg_fbm_points_2d(1, octaves, 0.5, 2.0, f0, 0.01, 1, i, j)
    assert np.max(np.abs(got - want)) <= 1e-5 * _amp(octaves)

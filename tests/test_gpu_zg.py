"""Zero-gradient D2M1N3 model (Sec. 3.3) on the GPU against the FP64 oracle: node
heights bit for bit (K1), fields within 1e-5 * A on the strip kernel (every finest-period
specialisation, ragged windows, int64 offsets) and the general kernel (any base
frequency and lacunarity), FP16 output within its rounding, crops equal to the full
field bit for bit, and sampled outputs of the 8192^2 8-octave field."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
import paper_1610_03525_amd as ptg  # noqa: E402

pytestmark = pytest.mark.gpu


def _field(nx, ny, x0, y0, dtype=torch.float32, **kw):
    out = torch.empty((ny, nx), dtype=dtype, device="cuda")
    ptg.fbm_2d(out, x0=x0, y0=y0, model="zero_gradient", **kw)
    torch.cuda.synchronize()
    return out


def _amp(octaves, pers=0.5):
    return sum(pers ** o for o in range(octaves))


def test_node_heights_bit_exact():
    ix0, iy0 = -(1 << 40) + 3, (1 << 35) - 17
    h = torch.empty((37, 70), dtype=torch.float32, device="cuda")
    for octave, seed in ((0, 1), (5, 0xDEADBEEF)):
        ptg.heights_2d(seed, octave, ix0, iy0, h)
        got = h.cpu().numpy().astype(np.float64)
        want = np.array([[O.height2(O.key2(ix0 + i, iy0 + j, octave, seed)) for i in range(70)] for j in range(37)])
        assert np.array_equal(got, want)


# (base frequency, octaves): finest periods 1, 2, 4, 8, 16, 32 and only periods >= 64
LADDERS = [(2.0 ** -5, 6), (2.0 ** -5, 5), (2.0 ** -5, 4), (2.0 ** -6, 4), (2.0 ** -6, 3), (2.0 ** -6, 2),
           (2.0 ** -8, 3)]


@pytest.mark.parametrize("f0,octaves", LADDERS)
@pytest.mark.parametrize("path", ["dyadic", "general"])
def test_field_matches_oracle(f0, octaves, path):
    nx, ny, x0, y0, seed = 200, 131, -(1 << 33) + 37, (1 << 20) - 5, 1610
    got = _field(nx, ny, x0, y0, octaves=octaves, base_freq=f0, seed=seed, path=path).cpu().numpy()
    want = O.zg_fbm_2d(octaves, 0.5, 2.0, f0, seed, x0, y0, nx, ny)
    assert np.max(np.abs(got - want)) <= 1e-5 * _amp(octaves)


@pytest.mark.parametrize("f0,lac,pers,octaves", [(0.0137, 1.9, 0.55, 5), (0.003, 2.3, 0.4, 4), (0.21, 1.5, 0.6, 3)])
def test_general_ladders_match_oracle(f0, lac, pers, octaves):
    nx, ny, x0, y0, seed = 150, 77, 12345, -(1 << 30) + 1, 7
    got = _field(nx, ny, x0, y0, octaves=octaves, base_freq=f0, lacunarity=lac, persistence=pers,
                 seed=seed).cpu().numpy()
    want = O.zg_fbm_2d(octaves, pers, lac, f0, seed, x0, y0, nx, ny)
    assert np.max(np.abs(got - want)) <= 1e-5 * _amp(octaves, pers)


def test_fp16_output_within_its_rounding():
    nx, ny, f0, octaves = 256, 64, 2.0 ** -6, 5
    got = _field(nx, ny, 0, 0, dtype=torch.float16, octaves=octaves, base_freq=f0, seed=3).float().cpu().numpy()
    want = O.zg_fbm_2d(octaves, 0.5, 2.0, f0, 3, 0, 0, nx, ny)
    assert np.all(np.abs(got - want) <= np.abs(want) * 2.0 ** -11 + 1e-5 * _amp(octaves))


def test_crops_equal_the_full_field():
    kw = dict(octaves=6, base_freq=2.0 ** -5, seed=11)
    full = _field(256, 192, -64, 128, **kw)
    for (cx, cy, w, h) in ((0, 0, 256, 192), (3, 5, 77, 61), (64, 64, 128, 64), (200, 150, 56, 42)):
        crop = _field(w, h, -64 + cx, 128 + cy, **kw)
        assert torch.equal(crop, full[cy:cy + h, cx:cx + w])


def test_benchmark_field_sampled():
    """8192^2, 8 octaves, base lattice 16^2 (periods 512..4): the strip kernel's workload."""
    n, octaves, f0 = 8192, 8, 16 / 8192
    out = _field(n, n, 0, 0, octaves=octaves, base_freq=f0, seed=1)
    rng = np.random.default_rng(8)
    i = rng.integers(0, n, 4000)
    j = rng.integers(0, n, 4000)
    got = out[torch.as_tensor(j, device="cuda"), torch.as_tensor(i, device="cuda")].cpu().numpy()
    want = O.zg_fbm_points_2d(octaves, 0.5, 2.0, f0, 1, i, j)
    assert np.max(np.abs(got - want)) <= 1e-5 * _amp(octaves)
    assert float(out.abs().max()) <= _amp(octaves)

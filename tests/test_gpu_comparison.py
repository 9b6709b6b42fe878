"""The comparison paths on the GPU against the FP64 oracle: Perlin's gradient noise
(Sec. 3.2, fade S3 and S5, the same hashed unit gradients) and the simplex-lattice gradient
noise standing for the paper's OpenSimplex timings (parity against the oracle only: the
oracle's simplex noise is itself unpinned against any outside implementation).  Fields
within 1e-5 * A on dyadic and non-dyadic ladders at int64 offsets, FP16 output, crops
equal to the full field bit for bit."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
import paper_1610_03525_amd as ptg  # noqa: E402

pytestmark = pytest.mark.gpu


def _amp(octaves, pers=0.5):
    return sum(pers ** o for o in range(octaves))


def _field(nx, ny, x0, y0, dtype=torch.float32, **kw):
    out = torch.empty((ny, nx), dtype=dtype, device="cuda")
    ptg.fbm_2d(out, x0=x0, y0=y0, **kw)
    torch.cuda.synchronize()
    return out


LADDERS = [(2.0 ** -5, 2.0, 6), (2.0 ** -9, 2.0, 8), (0.0137, 1.9, 5), (0.45, 2.0, 2)]


@pytest.mark.parametrize("smooth,order", [(1, 3), (2, 5)])
@pytest.mark.parametrize("f0,lac,octaves", LADDERS)
def test_perlin_matches_oracle(smooth, order, f0, lac, octaves):
    nx, ny, x0, y0 = 150, 77, -(1 << 33) + 5, (1 << 21) + 9
    got = _field(nx, ny, x0, y0, model="perlin", smoothness=smooth, octaves=octaves, base_freq=f0, lacunarity=lac,
                 seed=13).cpu().numpy()
    want = O.perlin_2d(order, octaves, 0.5, lac, f0, 13, x0, y0, nx, ny)
    assert np.max(np.abs(got - want)) <= 1e-5 * _amp(octaves)


@pytest.mark.parametrize("f0,lac,octaves", LADDERS + [(1.0, 0.5, 3)])
def test_simplex_matches_oracle(f0, lac, octaves):
    nx, ny, x0, y0 = 150, 77, -(1 << 33) + 5, (1 << 21) + 9
    got = _field(nx, ny, x0, y0, model="simplex", octaves=octaves, base_freq=f0, lacunarity=lac,
                 seed=13).cpu().numpy()
    want = O.simplex_2d(octaves, 0.5, lac, f0, 13, x0, y0, nx, ny)
    assert np.max(np.abs(got - want)) <= 1e-5 * _amp(octaves)


@pytest.mark.parametrize("model", ["perlin", "simplex"])
def test_fp16_output_and_crops(model):
    kw = dict(model=model, octaves=6, base_freq=1 / 64, seed=2)
    full = _field(192, 128, -64, 32, **kw)
    crop = _field(70, 50, -64 + 33, 32 + 17, **kw)
    assert torch.equal(crop, full[17:67, 33:103])
    half = _field(192, 128, -64, 32, dtype=torch.float16, **kw).float().cpu().numpy()
    want = (O.perlin_2d(3, 6, 0.5, 2.0, 1 / 64, 2, -64, 32, 192, 128) if model == "perlin"
            else O.simplex_2d(6, 0.5, 2.0, 1 / 64, 2, -64, 32, 192, 128))
    assert np.all(np.abs(half - want) <= np.abs(want) * 2.0 ** -11 + 1e-5 * _amp(6))


def test_benchmark_field_sampled():
    n = 8192
    for model, ref in (("perlin", lambda X, Y: None), ("simplex", None)):
        out = _field(n, n, 0, 0, model=model, octaves=8, base_freq=16 / n, seed=1)
        rng = np.random.default_rng(4)
        X, Y = rng.integers(0, n, 400), rng.integers(0, n, 400)
        got = out[torch.from_numpy(Y).cuda(), torch.from_numpy(X).cuda()].cpu().numpy()
        for k in range(0, 400, 40):  # the oracle one sample at a time
            x, y = int(X[k]), int(Y[k])
            want = (O.perlin_2d(3, 8, 0.5, 2.0, 16 / n, 1, x, y, 1, 1) if model == "perlin"
                    else O.simplex_2d(8, 0.5, 2.0, 16 / n, 1, x, y, 1, 1))[0, 0]
            assert abs(got[k] - want) <= 1e-5 * _amp(8)

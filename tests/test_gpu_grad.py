"""Analytic gradient output (ptg_fbm_2d_grad; the gradient maps of Sec. 5.1) against the
FP64 oracle for the three cell models and cubic to septic cells, dyadic and non-dyadic
ladders at int64 offsets; its height output equals the general kernel's bit for bit."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
import paper_1610_03525_amd as ptg  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [("gradient", 1), ("gradient", 2), ("gradient", 3), ("zero_gradient", 1), ("height_gradient", 1),
         ("height_gradient", 2), ("height_gradient", 3)]


@pytest.mark.parametrize("model,M", CASES)
@pytest.mark.parametrize("f0,lac,octaves", [(2.0 ** -5, 2.0, 6), (0.0137, 1.9, 5)])
def test_gradient_matches_oracle(model, M, f0, lac, octaves):
    ptg.tune_reset()
    nx, ny, x0, y0, seed, w, pers = 150, 97, -(1 << 33) + 21, (1 << 24) - 7, 31, 0.3, 0.5
    kw = dict(smoothness=M, octaves=octaves, base_freq=f0, lacunarity=lac, persistence=pers, seed=seed,
              model=model, gradient_weight=w)
    h, dx, dy = (torch.empty((ny, nx), dtype=torch.float32, device="cuda") for _ in range(3))
    ptg.fbm_2d_grad(h, dx, dy, x0=x0, y0=y0, **kw)
    ref = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    ptg.fbm_2d(ref, x0=x0, y0=y0, path="general", **kw)
    torch.cuda.synchronize()
    assert torch.equal(h, ref)
    H, HX, HY = O.fbm_2d_grad(model, M, octaves, pers, lac, f0, w, seed, x0, y0, nx, ny)
    amp = sum(pers ** o for o in range(octaves))
    gscale = sum(pers ** o * f0 * lac ** o for o in range(octaves))  # sum a_o f_o
    assert np.max(np.abs(h.cpu().numpy() - H)) <= 1e-5 * amp
    assert np.max(np.abs(dx.cpu().numpy() - HX)) <= 4e-5 * gscale
    assert np.max(np.abs(dy.cpu().numpy() - HY)) <= 4e-5 * gscale


def test_fp16_outputs_and_validation():
    kw = dict(octaves=4, base_freq=2.0 ** -4, seed=2)
    h, dx, dy = (torch.empty((64, 96), dtype=torch.float16, device="cuda") for _ in range(3))
    ptg.fbm_2d_grad(h, dx, dy, x0=10, y0=-3, **kw)
    torch.cuda.synchronize()
    H, HX, HY = O.fbm_2d_grad("gradient", 1, 4, 0.5, 2.0, 2.0 ** -4, 0.01, 2, 10, -3, 96, 64)
    for got, want in ((h, H), (dx, HX), (dy, HY)):
        g = got.float().cpu().numpy()
        assert np.all(np.abs(g - want) <= np.abs(want) * 2.0 ** -11 + 1e-4)
    with pytest.raises(ptg.PtgError):
        ptg.fbm_2d_grad(h, dx, dy, form="mfma_f16", **kw)

"""Analytic gradient output (ptg_fbm_2d_grad; the gradient maps of Sec. 5.1) against the
FP64 oracle for the three cell models and cubic to septic cells, dyadic ladders (the strip
kernel, finest periods 1, 4 and >= 64) and a non-dyadic one (the general kernel) at int64
offsets with ragged edges; its height output equals ptg_fbm_2d's bit for bit, and the
strip kernel's derivatives agree with the general kernel's."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
import paper_1610_03525_amd as ptg  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [("gradient", 1), ("gradient", 2), ("gradient", 3), ("zero_gradient", 1), ("height_gradient", 1),
         ("height_gradient", 2), ("height_gradient", 3)]


LADDERS = [(2.0 ** -5, 2.0, 6), (2.0 ** -9, 2.0, 8), (2.0 ** -12, 2.0, 4), (0.0137, 1.9, 5)]


@pytest.mark.parametrize("model,M", CASES)
@pytest.mark.parametrize("f0,lac,octaves", LADDERS)
def test_gradient_matches_oracle(model, M, f0, lac, octaves):
    ptg.tune_reset()
    nx, ny, x0, y0, seed, w, pers = 150, 97, -(1 << 33) + 21, (1 << 24) - 7, 31, 0.3, 0.5
    kw = dict(smoothness=M, octaves=octaves, base_freq=f0, lacunarity=lac, persistence=pers, seed=seed,
              model=model, gradient_weight=w)
    print(f"[grad] {model} C{M} f0={f0} lac={lac} oct={octaves}", flush=True)
    h, dx, dy = (torch.empty((ny, nx), dtype=torch.float32, device="cuda") for _ in range(3))
    ptg.fbm_2d_grad(h, dx, dy, x0=x0, y0=y0, **kw)
    ref = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    ptg.fbm_2d(ref, x0=x0, y0=y0, **kw)  # the same plan: strip kernel for dyadic ladders
    gh, gx, gy = (torch.empty((ny, nx), dtype=torch.float32, device="cuda") for _ in range(3))
    ptg.fbm_2d_grad(gh, gx, gy, x0=x0, y0=y0, path="general", **kw)
    torch.cuda.synchronize()
    assert torch.equal(h, ref)
    H, HX, HY = O.fbm_2d_grad(model, M, octaves, pers, lac, f0, w, seed, x0, y0, nx, ny)
    amp = sum(pers ** o for o in range(octaves))
    gscale = sum(pers ** o * f0 * lac ** o for o in range(octaves))  # sum a_o f_o
    assert np.max(np.abs(h.cpu().numpy() - H)) <= 1e-5 * amp
    for d, ref_d, gen in ((dx, HX, gx), (dy, HY, gy)):
        assert np.max(np.abs(d.cpu().numpy() - ref_d)) <= 4e-5 * gscale
        assert np.max(np.abs(gen.cpu().numpy() - ref_d)) <= 4e-5 * gscale


@pytest.mark.parametrize("M", [1, 2])
def test_strip_gradient_full_size_sampled(M):
    """The 8192^2 8-octave field (base lattice 16^2) on the strip kernel, as timed: sampled
    rows and columns of dH/dX and dH/dY against the oracle, and the field bit for bit."""
    n, f0, octaves = 8192, 16 / 8192, 8
    kw = dict(smoothness=M, octaves=octaves, base_freq=f0, seed=1)
    print(f"[grad] 8192^2 C{M}", flush=True)
    h, dx, dy = (torch.empty((n, n), dtype=torch.float32, device="cuda") for _ in range(3))
    ptg.fbm_2d_grad(h, dx, dy, **kw)
    ref = torch.empty((n, n), dtype=torch.float32, device="cuda")
    ptg.fbm_2d(ref, **kw)
    torch.cuda.synchronize()
    assert torch.equal(h, ref)
    del ref
    gscale = sum(0.5 ** o * f0 * 2.0 ** o for o in range(octaves))
    for y0, x0, ny, nx in ((0, 0, 3, n), (4093, 0, 2, n), (n - 2, 0, 2, n), (0, 4095, n, 2), (0, n - 1, n, 1)):
        _, HX, HY = O.fbm_2d_grad("gradient", M, octaves, 0.5, 2.0, f0, 0.01, 1, x0, y0, nx, ny)
        assert np.max(np.abs(dx[y0:y0 + ny, x0:x0 + nx].cpu().numpy() - HX)) <= 4e-5 * gscale
        assert np.max(np.abs(dy[y0:y0 + ny, x0:x0 + nx].cpu().numpy() - HY)) <= 4e-5 * gscale


@pytest.mark.parametrize("M", [1, 2, 3])
def test_strip_gradient_fp16_outputs(M):
    """FP16 outputs of the one-launch strip gradient (a dyadic ladder with ragged edges):
    the field equals ptg_fbm_2d's FP16 output bit for bit, the derivatives match the oracle
    within their FP16 rounding."""
    kw = dict(smoothness=M, octaves=6, base_freq=2.0 ** -7, seed=5)
    nx, ny, x0, y0 = 200, 131, -(1 << 30) + 33, 77
    h, dx, dy = (torch.empty((ny, nx), dtype=torch.float16, device="cuda") for _ in range(3))
    ptg.fbm_2d_grad(h, dx, dy, x0=x0, y0=y0, **kw)
    ref = torch.empty((ny, nx), dtype=torch.float16, device="cuda")
    ptg.fbm_2d(ref, x0=x0, y0=y0, **kw)
    torch.cuda.synchronize()
    assert torch.equal(h, ref)
    _, HX, HY = O.fbm_2d_grad("gradient", M, 6, 0.5, 2.0, 2.0 ** -7, 0.01, 5, x0, y0, nx, ny)
    gscale = sum(0.5 ** o * 2.0 ** -7 * 2.0 ** o for o in range(6))
    for got, want in ((dx, HX), (dy, HY)):
        g = got.float().cpu().numpy()
        assert np.all(np.abs(g - want) <= np.abs(want) * 2.0 ** -11 + 4e-5 * gscale)


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

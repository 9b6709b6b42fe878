"""3D height-and-gradient model (D3M1N3 / D3M2N5 with random node heights from the key's
third word and w-weighted lattice gradients; Sec. 3.1 heights, Sec. 3.4, Sec. 4 w) on the
GPU against the FP64 oracle: volumes within 1e-5 * A (times max(1, |w|)) for C1 and C2
cells on the 3D strip kernel (every fine-period class) and the general kernel, weights 0
(smoothstep value noise), the paper's 0.01, 0.5 and -1.3, FP16 output, and crops equal to
the full volume bit for bit."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
import paper_1610_03525_amd as ptg  # noqa: E402

pytestmark = pytest.mark.gpu


def _vol(nx, ny, nz, x0, y0, z0, dtype=torch.float32, **kw):
    out = torch.empty((nz, ny, nx), dtype=dtype, device="cuda")
    ptg.fbm_3d(out, x0=x0, y0=y0, z0=z0, model="height_gradient", **kw)
    torch.cuda.synchronize()
    return out


def _amp(octaves, pers=0.5):
    return sum(pers ** o for o in range(octaves))


# (base frequency, octaves): finest periods 2, 4, 8, 16 and a ladder without coarse octaves
LADDERS = [(2.0 ** -6, 6), (2.0 ** -6, 5), (2.0 ** -6, 4), (2.0 ** -7, 4), (2.0 ** -3, 3)]


@pytest.mark.parametrize("M", [1, 2])
@pytest.mark.parametrize("f0,octaves", LADDERS)
@pytest.mark.parametrize("path", ["dyadic", "general"])
def test_volume_matches_oracle(M, f0, octaves, path):
    nx, ny, nz, x0, y0, z0, seed, w = 70, 19, 21, (1 << 33) - 29, -(1 << 22) + 3, 45, 99, 0.01
    got = _vol(nx, ny, nz, x0, y0, z0, smoothness=M, octaves=octaves, base_freq=f0, seed=seed, gradient_weight=w,
               path=path).cpu().numpy()
    want = O.hg_fbm_3d(M, octaves, 0.5, 2.0, f0, w, seed, x0, y0, z0, nx, ny, nz)
    assert np.max(np.abs(got - want)) <= 1e-5 * _amp(octaves)


@pytest.mark.parametrize("M", [1, 2])
@pytest.mark.parametrize("w", [0.0, 0.5, -1.3])
@pytest.mark.parametrize("path", ["dyadic", "general"])
def test_gradient_weights(M, w, path):
    nx, ny, nz, f0, octaves = 66, 10, 18, 2.0 ** -5, 4
    got = _vol(nx, ny, nz, -5, 17, -20, smoothness=M, octaves=octaves, base_freq=f0, seed=3, gradient_weight=w,
               path=path).cpu().numpy()
    want = O.hg_fbm_3d(M, octaves, 0.5, 2.0, f0, w, 3, -5, 17, -20, nx, ny, nz)
    assert np.max(np.abs(got - want)) <= 1e-5 * _amp(octaves) * max(1.0, abs(w))


@pytest.mark.parametrize("M", [1, 2])
def test_general_ladders_match_oracle(M):
    nx, ny, nz, f0, lac, pers, octaves = 40, 12, 9, 0.0137, 1.9, 0.55, 4
    got = _vol(nx, ny, nz, 12345, -(1 << 30) + 1, 77, smoothness=M, octaves=octaves, base_freq=f0, lacunarity=lac,
               persistence=pers, seed=7).cpu().numpy()
    want = O.hg_fbm_3d(M, octaves, pers, lac, f0, 0.01, 7, 12345, -(1 << 30) + 1, 77, nx, ny, nz)
    assert np.max(np.abs(got - want)) <= 1e-5 * _amp(octaves, pers)


def test_fp16_output_and_crops():
    kw = dict(smoothness=2, octaves=6, base_freq=1 / 64, seed=4, gradient_weight=0.3)
    big = _vol(100, 20, 30, 60, -9, 5, **kw)
    small = _vol(50, 7, 17, 70, -5, 8, **kw)
    assert torch.equal(big[3:20, 4:11, 10:60], small)
    h = _vol(100, 20, 30, 60, -9, 5, dtype=torch.float16, **kw)
    want = O.hg_fbm_3d(2, 6, 0.5, 2.0, 1 / 64, 0.3, 4, 60, -9, 5, 100, 20, 30)
    # FP16 output: round to nearest even, relative 2^-11 of |H| <= A
    assert np.max(np.abs(h.cpu().numpy().astype(np.float64) - want)) <= 2.0 ** -11 * _amp(6) + 1e-5 * _amp(6)


@pytest.mark.parametrize("M", [1, 2])
def test_full_size_volume_slabs(M):
    """The 512^3 6-octave volume as the benchmark times it (base lattice 8^3, w = 0.01): every
    sample of z-slabs that cross block boundaries inside a wave's run of consecutive blocks
    (whose fine node planes are carried from one block to the next) and at its start and end."""
    n, octaves, f0, seed, w = 512, 6, 8 / 512, 1, 0.01
    got = _vol(n, n, n, 0, 0, 0, smoothness=M, octaves=octaves, base_freq=f0, seed=seed, gradient_weight=w)
    for z0, nz in ((0, 32), (232, 32), (496, 16)):
        want = O.hg_fbm_3d(M, octaves, 0.5, 2.0, f0, w, seed, 0, 0, z0, n, n, nz)
        err = np.max(np.abs(got[z0:z0 + nz].cpu().numpy() - want))
        assert err <= 1e-5 * _amp(octaves), (z0, err)

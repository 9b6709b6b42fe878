"""The oracle's comparison paths, pinned by what their definitions fix.

Perlin's gradient noise (Sec. 3.2): the fBm of perlin_2d is the octave sum of Perlin cells
at the sample centres, the cell is the textbook lerp of corner dot products, and it is 0 at
the nodes with gradient g there.

Simplex-lattice gradient noise (the stand-in for the paper's OpenSimplex timings; PARITY
UNPINNED against any outside implementation): zero at every lattice point, gradient
70 (1/2)^4 g at a lattice point (only that corner's kernel is non-zero there), continuous
with a continuous gradient across the triangle edges and cell boundaries, and the fBm is
the octave sum at the sample centres."""
import math

import numpy as np
import pytest

import oracle as O

F2 = 0.5 * (math.sqrt(3.0) - 1.0)
G2 = (3.0 - math.sqrt(3.0)) / 6.0


def _lattice_point(i, j):
    t = (i + j) * G2
    return i - t, j - t


@pytest.mark.parametrize("i,j", [(0, 0), (3, 5), (-7, 2), (1 << 20, -(1 << 19)), (-1, -1)])
def test_simplex_zero_and_gradient_at_lattice_points(i, j):
    octave, seed = 2, 77
    ux, uy = _lattice_point(i, j)
    assert abs(O.simplex_at(ux, uy, octave, seed)) < 1e-12
    e = 1e-4  # central differences: O(e^2) truncation, FP64 rounding of |u| ~ 2^20 stays below 1e-9 / e
    gx = (O.simplex_at(ux + e, uy, octave, seed) - O.simplex_at(ux - e, uy, octave, seed)) / (2 * e)
    gy = (O.simplex_at(ux, uy + e, octave, seed) - O.simplex_at(ux, uy - e, octave, seed)) / (2 * e)
    g = O.grad2(O.key2(i, j, octave, seed))
    scale = 70.0 * 0.5 ** 4
    assert gx == pytest.approx(scale * g[0], abs=1e-5) and gy == pytest.approx(scale * g[1], abs=1e-5)


def test_simplex_continuous_with_continuous_gradient():
    rng = np.random.default_rng(3)
    e, h = 1e-9, 1e-5
    for _ in range(200):
        i, j = (int(v) for v in rng.integers(-1000, 1000, 2))
        # a point on the triangle edge x0 = y0 inside cell (i, j), and one on the cell's lower edge
        a = rng.uniform(0.05, 0.95)
        bx, by = _lattice_point(i, j)
        for px, py, nx, ny in ((bx + a * (1 - 2 * G2), by + a * (1 - 2 * G2), 1.0, -1.0),
                               (bx + a * (1 - G2), by - a * G2, a * G2, 1 - G2 * a)):
            nrm = math.hypot(nx, ny)
            nx, ny = nx / nrm, ny / nrm
            f = lambda s: O.simplex_at(px + s * nx, py + s * ny, 0, 5)  # noqa: E731
            assert f(e) == pytest.approx(f(-e), abs=1e-7)
            dl = (f(0.0) - f(-h)) / h
            dr = (f(h) - f(0.0)) / h
            assert dl == pytest.approx(dr, abs=1e-3)


def test_simplex_fbm_sums_the_octaves():
    f0, lac, pers, seed, n = 0.013, 2.0, 0.5, 9, 4
    x0, y0 = -(1 << 30) + 3, 12345
    got = O.simplex_2d(n, pers, lac, f0, seed, x0, y0, 7, 5)
    for jj in range(5):
        for ii in range(7):
            want, f, a = 0.0, f0, 1.0
            for o in range(n):
                want += a * O.simplex_at((x0 + ii + 0.5) * f, (y0 + jj + 0.5) * f, o, seed)
                f *= lac
                a *= pers
            assert got[jj, ii] == want
    assert np.max(np.abs(got)) < 2.0


@pytest.mark.parametrize("order", [3, 5])
def test_perlin_fbm_sums_textbook_cells(order):
    f0, lac, pers, seed, n = 0.021, 2.0, 0.5, 4, 3
    x0, y0 = 1000, -(1 << 33) - 9
    got = O.perlin_2d(order, n, pers, lac, f0, seed, x0, y0, 6, 4)
    fade = (lambda t: t * t * (3 - 2 * t)) if order == 3 else (lambda t: t ** 3 * (10 - 15 * t + 6 * t * t))
    for jj in range(4):
        for ii in range(6):
            want, f, a = 0.0, f0, 1.0
            for o in range(n):
                cx, tx = O.coord(x0 + ii, f)
                cy, ty = O.coord(y0 + jj, f)
                g = {(dx, dy): O.grad2(O.key2(cx + dx, cy + dy, o, seed)) for dx in (0, 1) for dy in (0, 1)}
                v = {k: g[k][0] * (tx - k[0]) + g[k][1] * (ty - k[1]) for k in g}
                sx, sy = fade(tx), fade(ty)
                h0 = v[0, 0] + sx * (v[1, 0] - v[0, 0])
                h1 = v[0, 1] + sx * (v[1, 1] - v[0, 1])
                want += a * (h0 + sy * (h1 - h0))
                f *= lac
                a *= pers
            assert got[jj, ii] == pytest.approx(want, abs=1e-14)

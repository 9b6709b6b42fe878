"""Height-and-gradient model in the oracle (Sec. 3.1 with non-zero corner heights, the
gradient weight w of Sec. 4, tensor Hermite form), pinned against what the mathematics
fixes: a brute-force solve of the corner conditions (value h, gradient w g, every other
mixed derivative up to M zero) for cubic and quintic cells, the smoothstep value noise it
reduces to at w = 0, C1 / C2 continuity across shared faces, the node-height map and its
independence from the gradient angle, and the fBm assembly of cells."""
import itertools
import math

import numpy as np
import pytest

import oracle as O


def _dmono(a, d, s):
    if d > a:
        return 0.0
    return math.factorial(a) / math.factorial(a - d) * (s ** (a - d) if a - d > 0 else 1.0)


def _brute(M, h, g, w):
    """Coefficients c[i][j] of x^i y^j from: at each corner h^(a,b) = value h for (0,0),
    w gx for (1,0), w gy for (0,1), and 0 for every other a, b <= M."""
    n1 = 2 * M + 2
    monos = list(itertools.product(range(n1), repeat=2))
    rows, rhs = [], []
    for c, (cx, cy) in enumerate([(0, 0), (1, 0), (0, 1), (1, 1)]):
        for a in range(M + 1):
            for b in range(M + 1):
                rows.append([_dmono(i, a, cx) * _dmono(j, b, cy) for i, j in monos])
                rhs.append(h[c] if (a, b) == (0, 0) else w * g[c][0] if (a, b) == (1, 0)
                           else w * g[c][1] if (a, b) == (0, 1) else 0.0)
    A = np.array(rows)
    assert np.linalg.matrix_rank(A) == n1 * n1
    return np.linalg.solve(A, np.array(rhs)).reshape(n1, n1)


def _poly(c, x, y, dx=0, dy=0):
    return sum(c[i, j] * _dmono(i, dx, x) * _dmono(j, dy, y) for i in range(c.shape[0]) for j in range(c.shape[1]))


@pytest.mark.parametrize("M", [1, 2])
def test_cell_is_the_brute_force_hermite_interpolant(M):
    rng = np.random.default_rng(20 + M)
    for _ in range(6):
        h = rng.uniform(-1, 1, 4)
        ang = rng.uniform(0, 2 * np.pi, 4)
        g = np.stack([np.cos(ang), np.sin(ang)], axis=1)
        w = float(rng.choice([0.0, 0.01, 0.7]))
        c = _brute(M, h, g, w)
        for x, y in rng.uniform(0, 1, (12, 2)):
            assert abs(O.hg_cell(M, h, g, w, x, y) - _poly(c, x, y)) < 1e-11


@pytest.mark.parametrize("M,S", [(1, lambda t: t * t * (3 - 2 * t)),
                                 (2, lambda t: t ** 3 * (10 - 15 * t + 6 * t * t))])
def test_zero_weight_is_smoothstep_value_noise(M, S):
    h = np.array([0.3, -0.8, 0.55, 0.1])
    g = np.ones((4, 2))
    for x, y in ((0.2, 0.7), (0.5, 0.5), (0.9, 0.05)):
        want = h[0] + S(x) * (h[1] - h[0]) + S(y) * (h[2] - h[0]) + S(x) * S(y) * (h[3] + h[0] - h[1] - h[2])
        assert O.hg_cell(M, h, g, 0.0, x, y) == pytest.approx(want, abs=1e-14)


@pytest.mark.parametrize("M", [1, 2])
def test_continuity_across_shared_faces(M):
    rng = np.random.default_rng(30 + M)
    H = rng.uniform(-1, 1, (4, 4))
    ang = rng.uniform(0, 2 * np.pi, (4, 4))
    G = np.stack([np.cos(ang), np.sin(ang)], axis=-1)
    w = 0.3

    def cell(i, j):
        hh = [H[j, i], H[j, i + 1], H[j + 1, i], H[j + 1, i + 1]]
        gg = [G[j, i], G[j, i + 1], G[j + 1, i], G[j + 1, i + 1]]
        return hh, np.array(gg)

    e = 1e-4  # central differences of each cell's polynomial at the face (it extends past it)
    for j in range(2):
        for i in range(2):
            hl, gl = cell(i, j)
            hr, gr = cell(i + 1, j)
            for t in rng.uniform(0.1, 0.9, 4):
                f = lambda hh, gg, x, y: O.hg_cell(M, hh, gg, w, x, y)  # noqa: E731
                assert f(hl, gl, 1.0, t) == pytest.approx(f(hr, gr, 0.0, t), abs=1e-13)
                dl = (f(hl, gl, 1.0 + e, t) - f(hl, gl, 1.0 - e, t)) / (2 * e)
                dr = (f(hr, gr, e, t) - f(hr, gr, -e, t)) / (2 * e)
                assert dl == pytest.approx(dr, abs=1e-6)  # first derivative continuous
                if M == 2:
                    sl = (f(hl, gl, 1.0 + e, t) - 2 * f(hl, gl, 1.0, t) + f(hl, gl, 1.0 - e, t)) / e ** 2
                    sr = (f(hr, gr, e, t) - 2 * f(hr, gr, 0.0, t) + f(hr, gr, -e, t)) / e ** 2
                    assert sl == pytest.approx(sr, abs=1e-4)  # second derivative continuous


def test_node_heights_use_the_second_word():
    for key in (0, 1, 0x12345678, 0xFFFFFFFF):
        second = O.key3_second(key)
        assert O.height2_second(key) == (second >> 8) / 2.0 ** 23 - 1.0
    keys = [O.key2(i, 5 - 2 * i, 1, 4242) for i in range(20000)]
    h = np.array([O.height2_second(k) for k in keys])
    ang = np.array([math.atan2(*O.grad2(k)[::-1]) for k in keys])
    assert abs(h.mean()) < 0.02 and abs(h.var() - 1 / 3) < 0.02
    assert abs(np.corrcoef(h, np.cos(ang))[0, 1]) < 0.03 and abs(np.corrcoef(h, np.sin(ang))[0, 1]) < 0.03


@pytest.mark.parametrize("M", [1, 2])
def test_fbm_sums_the_octave_cells(M):
    f0, lac, pers, w, seed, n = 0.043, 2.0, 0.5, 0.01, 5, 3
    x0, y0 = (1 << 34) + 7, -(1 << 28) - 3
    got = O.hg_fbm_2d(M, n, pers, lac, f0, w, seed, x0, y0, 11, 7)
    for j in range(7):
        for i in range(11):
            want, f, a = 0.0, f0, 1.0
            for o in range(n):
                cx, tx = O.coord(x0 + i, f)
                cy, ty = O.coord(y0 + j, f)
                keys = [O.key2(cx + dx, cy + dy, o, seed) for dy in (0, 1) for dx in (0, 1)]
                hh = [O.height2_second(k) for k in keys]
                gg = np.array([O.grad2(k) for k in keys])
                want += a * O.hg_cell(M, hh, gg, w, tx, ty)
                f *= lac
                a *= pers
            assert got[j, i] == want
    pts = O.hg_fbm_points_2d(M, n, pers, lac, f0, w, seed, x0 + np.array([3, 10]), y0 + np.array([6, 0]))
    assert np.array_equal(pts, got[[6, 0], [3, 10]])


# ---- 3D: D3M1N3 / D3M2N5 with node heights (Sec. 3.4 with Sec. 3.1 heights, Sec. 4 w) ----

def _brute3(M, h, g, w):
    """Coefficients c[i][j][k] of x^i y^j z^k from: at each corner the mixed derivative
    (a, b, c) = value h for (0,0,0), w gx / w gy / w gz for the unit orders, 0 for every other
    a, b, c <= M."""
    n1 = 2 * M + 2
    monos = list(itertools.product(range(n1), repeat=3))
    rows, rhs = [], []
    corners = [(cx, cy, cz) for cz in (0, 1) for cy in (0, 1) for cx in (0, 1)]
    unit = {(1, 0, 0): 0, (0, 1, 0): 1, (0, 0, 1): 2}
    for c, (cx, cy, cz) in enumerate(corners):
        for d in itertools.product(range(M + 1), repeat=3):
            rows.append([_dmono(i, d[0], cx) * _dmono(j, d[1], cy) * _dmono(k, d[2], cz) for i, j, k in monos])
            rhs.append(h[c] if d == (0, 0, 0) else w * g[c][unit[d]] if d in unit else 0.0)
    A = np.array(rows)
    return np.linalg.solve(A, np.array(rhs)).reshape(n1, n1, n1)


def _poly3(c, x, y, z):
    n1 = c.shape[0]
    vx, vy, vz = (np.array([t ** e for e in range(n1)]) for t in (x, y, z))
    return float(np.einsum("ijk,i,j,k->", c, vx, vy, vz))


def _unit3(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("M", [1, 2])
def test_cell_3d_is_the_brute_force_hermite_interpolant(M):
    rng = np.random.default_rng(40 + M)
    for _ in range(3):
        h = rng.uniform(-1, 1, 8)
        g = _unit3(rng, 8)
        w = float(rng.choice([0.0, 0.01, 0.7]))
        c = _brute3(M, h, g, w)
        for x, y, z in rng.uniform(0, 1, (8, 3)):
            assert abs(O.hg_cell_3d(M, h, g, w, x, y, z) - _poly3(c, x, y, z)) < 1e-10


@pytest.mark.parametrize("M,S", [(1, lambda t: t * t * (3 - 2 * t)),
                                 (2, lambda t: t ** 3 * (10 - 15 * t + 6 * t * t))])
def test_cell_3d_zero_weight_is_smoothstep_value_noise(M, S):
    h = np.array([0.3, -0.8, 0.55, 0.1, -0.45, 0.9, 0.0, -0.2])
    g = np.ones((8, 3))
    lerp = lambda a, b, t: a + (b - a) * t  # noqa: E731
    for x, y, z in ((0.2, 0.7, 0.4), (0.5, 0.5, 0.5), (0.9, 0.05, 0.66)):
        sx, sy, sz = S(x), S(y), S(z)
        want = lerp(lerp(lerp(h[0], h[1], sx), lerp(h[2], h[3], sx), sy),
                    lerp(lerp(h[4], h[5], sx), lerp(h[6], h[7], sx), sy), sz)
        assert O.hg_cell_3d(M, h, g, 0.0, x, y, z) == pytest.approx(want, abs=1e-14)


@pytest.mark.parametrize("M", [1, 2])
def test_cell_3d_continuity_across_shared_faces(M):
    """Two cells sharing the face x = 1 | x = 0 (and likewise in y and z): value and normal
    derivative (and for M = 2 the second normal derivative) agree on the face."""
    rng = np.random.default_rng(50 + M)
    H = rng.uniform(-1, 1, (3, 3, 3))
    G = _unit3(rng, 27).reshape(3, 3, 3, 3)
    w = 0.4

    def cell(i, j, k):
        idx = [(i + dx, j + dy, k + dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
        return [H[c[2], c[1], c[0]] for c in idx], np.array([G[c[2], c[1], c[0]] for c in idx])

    e = 1e-4
    for axis in range(3):
        lo = cell(0, 0, 0)
        hi = cell(*[1 if a == axis else 0 for a in range(3)])
        for s, t in rng.uniform(0.1, 0.9, (3, 2)):
            def at(cl, n):  # point on the face with normal coordinate n
                p = [s, t]
                p.insert(axis, n)
                return O.hg_cell_3d(M, cl[0], cl[1], w, *p)
            assert at(lo, 1.0) == pytest.approx(at(hi, 0.0), abs=1e-13)
            dl = (at(lo, 1.0 + e) - at(lo, 1.0 - e)) / (2 * e)
            dr = (at(hi, e) - at(hi, -e)) / (2 * e)
            assert dl == pytest.approx(dr, abs=1e-6)
            if M == 2:
                sl = (at(lo, 1.0 + e) - 2 * at(lo, 1.0) + at(lo, 1.0 - e)) / e ** 2
                sr = (at(hi, e) - 2 * at(hi, 0.0) + at(hi, -e)) / e ** 2
                assert sl == pytest.approx(sr, abs=1e-4)


def test_node_heights_3d_use_the_third_word():
    for key in (0, 1, 0x12345678, 0xFFFFFFFF):
        third = O.key3_second(O.key3_second(key))
        assert O.height3(key) == (third >> 8) / 2.0 ** 23 - 1.0
    keys = [O.key3(i, 5 - 2 * i, 3 * i + 1, 1, 4242) for i in range(20000)]
    h = np.array([O.height3(k) for k in keys])
    g = np.array([O.grad3(k) for k in keys])
    assert abs(h.mean()) < 0.02 and abs(h.var() - 1 / 3) < 0.02
    for a in range(3):
        assert abs(np.corrcoef(h, g[:, a])[0, 1]) < 0.03


@pytest.mark.parametrize("M", [1, 2])
def test_fbm_3d_sums_the_octave_cells(M):
    f0, lac, pers, w, seed, n = 0.071, 2.0, 0.5, 0.01, 9, 3
    x0, y0, z0 = (1 << 34) + 7, -(1 << 28) - 3, 5
    got = O.hg_fbm_3d(M, n, pers, lac, f0, w, seed, x0, y0, z0, 5, 4, 3)
    for k in range(3):
        for j in range(4):
            for i in range(5):
                want, f, a = 0.0, f0, 1.0
                for o in range(n):
                    (cx, tx), (cy, ty), (cz, tz) = (O.coord(v, f) for v in (x0 + i, y0 + j, z0 + k))
                    keys = [O.key3(cx + dx, cy + dy, cz + dz, o, seed)
                            for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
                    hh = [O.height3(q) for q in keys]
                    gg = np.array([O.grad3(q) for q in keys])
                    want += a * O.hg_cell_3d(M, hh, gg, w, tx, ty, tz)
                    f *= lac
                    a *= pers
                assert got[k, j, i] == want
    pts = O.hg_fbm_points_3d(M, n, pers, lac, f0, w, seed, x0 + np.array([3, 0]), y0 + np.array([2, 3]),
                             z0 + np.array([1, 2]))
    assert np.array_equal(pts, got[[1, 2], [2, 3], [3, 0]])

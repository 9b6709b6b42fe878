"""Zero-gradient D2M1N3 in the oracle (Sec. 3.3, eq. zg), pinned against what the paper
and the mathematics fix: the general D2M1N3 system of Sec. 3.1 (twelve corner
conditions on the twelve monomials it keeps) solved by brute force with zero gradients,
the corner values and gradients themselves, the sign of the xy term (the printed +xy
breaks the (1, 1) corner), value continuity across shared faces, the node-height map,
and the fBm assembly of cells."""
import numpy as np
import pytest

import oracle as O

# Sec. 3.1: h = sum c_ij x^i y^j, 0 <= i, j <= 3, with c22 = c33 = c32 = c23 = 0
MONO = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3), (3, 1), (1, 3)]
CORNERS = [(0, 0), (1, 0), (0, 1), (1, 1)]


def _d2m1n3(h, f, g):
    """Coefficients of the Sec. 3.1 polynomial from corner heights h, x-gradients f and
    y-gradients g (corner order 00, 10, 01, 11), by a dense linear solve."""
    rows, rhs = [], []
    for (cx, cy), hv, fv, gv in zip(CORNERS, h, f, g):
        rows.append([float(cx ** i * cy ** j) for i, j in MONO])
        rhs.append(hv)
        rows.append([float(i * cx ** (i - 1) * cy ** j) if i else 0.0 for i, j in MONO])
        rhs.append(fv)
        rows.append([float(j * cx ** i * cy ** (j - 1)) if j else 0.0 for i, j in MONO])
        rhs.append(gv)
    A = np.array(rows)
    assert np.linalg.matrix_rank(A) == 12
    return np.linalg.solve(A, np.array(rhs))


def _poly(c, x, y):
    return sum(ci * x ** i * y ** j for ci, (i, j) in zip(c, MONO))


def test_zero_gradient_cell_is_the_general_d2m1n3_with_zero_gradients():
    rng = np.random.default_rng(3)
    for _ in range(25):
        h = rng.uniform(-1, 1, 4)
        c = _d2m1n3(h, np.zeros(4), np.zeros(4))
        for x, y in rng.uniform(0, 1, (20, 2)):
            assert abs(O.zg_cell(h, x, y) - _poly(c, x, y)) < 1e-13


def test_corner_heights_and_zero_corner_gradients():
    rng = np.random.default_rng(4)
    e = 1e-6
    for _ in range(25):
        h = rng.uniform(-1, 1, 4)
        for (cx, cy), hv in zip(CORNERS, h):
            assert O.zg_cell(h, cx, cy) == pytest.approx(hv, abs=1e-15)
            gx = (O.zg_cell(h, cx + e, cy) - O.zg_cell(h, cx - e, cy)) / (2 * e)
            gy = (O.zg_cell(h, cx, cy + e) - O.zg_cell(h, cx, cy - e)) / (2 * e)
            assert abs(gx) < 1e-9 and abs(gy) < 1e-9


def test_printed_plus_xy_term_breaks_the_far_corner():
    """The form printed in Sec. 3.3 (+xy) gives h(1, 1) = h11 + 2A; the oracle's -xy
    form gives h11 (reading: the Sec. 3.1 coefficients decide the sign)."""
    h = np.array([0.3, -0.2, 0.5, 0.9])
    A = h[3] + h[0] - h[1] - h[2]
    s3 = lambda t: t * t * (3 - 2 * t)  # noqa: E731

    def printed(x, y):
        return h[0] + s3(x) * (h[1] - h[0]) + s3(y) * (h[2] - h[0]) + A * (s3(x) * y + s3(y) * x + x * y)

    assert printed(1.0, 1.0) == pytest.approx(h[3] + 2 * A)
    assert abs(printed(1.0, 1.0) - h[3]) > 0.1
    assert O.zg_cell(h, 1.0, 1.0) == pytest.approx(h[3], abs=1e-15)


def test_shared_faces_agree_in_value():
    """Neighbouring cells use only the face's two nodes on a shared face, so the field is
    continuous; its normal derivative there depends on A and is not (C0 model)."""
    rng = np.random.default_rng(5)
    H = rng.uniform(-1, 1, (5, 5))  # node heights H[j, i]

    def cell(i, j):
        return [H[j, i], H[j, i + 1], H[j + 1, i], H[j + 1, i + 1]]

    jumps = []
    for j in range(3):
        for i in range(3):
            for t in rng.uniform(0, 1, 7):
                assert O.zg_cell(cell(i, j), 1.0, t) == pytest.approx(O.zg_cell(cell(i + 1, j), 0.0, t), abs=1e-14)
                assert O.zg_cell(cell(i, j), t, 1.0) == pytest.approx(O.zg_cell(cell(i, j + 1), t, 0.0), abs=1e-14)
                e = 1e-6
                dl = (O.zg_cell(cell(i, j), 1.0, t) - O.zg_cell(cell(i, j), 1.0 - e, t)) / e
                dr = (O.zg_cell(cell(i + 1, j), e, t) - O.zg_cell(cell(i + 1, j), 0.0, t)) / e
                jumps.append(abs(dl - dr))
    assert max(jumps) > 1e-3  # gradients are pinned at the nodes only


def test_node_heights_are_the_top_24_key_bits_on_minus_one_to_one():
    for m in (0, 1, 1 << 23, (1 << 24) - 1):
        for low in (0, 0xFF):
            assert O.height2((m << 8) | low) == m / 2.0 ** 23 - 1.0
    keys = [O.key2(i, 3 * i - 7, 2, 99) for i in range(20000)]
    h = np.array([O.height2(k) for k in keys])
    assert h.min() >= -1.0 and h.max() < 1.0
    assert abs(h.mean()) < 0.02 and abs(h.var() - 1 / 3) < 0.02


def test_zero_gradient_fbm_sums_the_octave_cells():
    f0, lac, pers, seed, n = 0.071, 2.0, 0.5, 77, 3
    x0, y0 = -(1 << 33) - 5, (1 << 31) + 9
    got = O.zg_fbm_2d(n, pers, lac, f0, seed, x0, y0, 13, 9)
    for j in range(9):
        for i in range(13):
            want, f, a = 0.0, f0, 1.0
            for o in range(n):
                cx, tx = O.coord(x0 + i, f)
                cy, ty = O.coord(y0 + j, f)
                h = [O.height2(O.key2(cx + dx, cy + dy, o, seed)) for dy in (0, 1) for dx in (0, 1)]
                want += a * O.zg_cell(h, tx, ty)
                f *= lac
                a *= pers
            assert got[j, i] == want
    pts = O.zg_fbm_points_2d(n, pers, lac, f0, seed, x0 + np.array([0, 12, 5]), y0 + np.array([0, 8, 3]))
    assert np.array_equal(pts, got[[0, 8, 3], [0, 12, 5]])

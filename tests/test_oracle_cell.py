"""Pins of the oracle's cell polynomial against the paper's model (CPU only).

The oracle evaluates a closed (tensor Hermite) form.  These tests check it against
things it does not compute itself:

* a brute-force solve of the square linear system that the corner constraints
  define (Sec. 2, eqs. mixedderiv / polynomial / nconstraints), built here from
  the derivative rule for monomials;
* the smoothstep functions the paper names (S3 in Sec. 3.2 / 3.4, S5 in Sec. 5.1);
* C1 / C2 continuity across shared faces (the edge boundary condition,
  eq. independance, and the smoothness the method is for);
* the paper's own D2M1N3 member (Sec. 3.1) as a negative control, and the
  zero-gradient reduction (eq. zg) with its sign reading.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O


def _dmono(a, d, s):
    """d-th derivative of s^a (one axis), with 0^0 = 1."""
    if d > a:
        return 0.0
    return math.factorial(a) / math.factorial(a - d) * (s ** (a - d) if a - d > 0 else 1.0)


def _brute_coeffs(D, M, grads):
    """Solve for the (n+1)^D monomial coefficients from the corner conditions:
    h^d(s) = 0 for every d in {0..M}^D except d = e_a, where h^{e_a}(s) = g_a(s)."""
    n1 = 2 * M + 2
    monos = list(itertools.product(range(n1), repeat=D))
    rows, rhs = [], []
    for ci, corner in enumerate(itertools.product((0, 1), repeat=D)):
        corner = corner[::-1]  # corner index c = cx + 2 cy (+ 4 cz): x fastest
        for d in itertools.product(range(M + 1), repeat=D):
            row = [np.prod([_dmono(a[k], d[k], corner[k]) for k in range(D)]) for a in monos]
            rows.append(row)
            if sum(d) == 1:
                rhs.append(grads[ci][d.index(1)])
            else:
                rhs.append(0.0)
    A = np.array(rows)
    assert A.shape == (n1 ** D, n1 ** D)  # square system: (M+1)^D conditions per corner
    b = np.array(rhs)
    c = np.linalg.solve(A, b)
    return c.reshape((n1,) * D), A, b


def _poly_eval(c, pts, deriv=None):
    """Evaluate sum c[a] prod x_k^a_k (optionally a mixed derivative) at points."""
    D = c.ndim
    deriv = deriv or (0,) * D
    out = 0.0
    for a in itertools.product(range(c.shape[0]), repeat=D):
        if c[a] == 0.0:
            continue
        term = c[a]
        for k in range(D):
            term = term * _dmono(a[k], deriv[k], pts[k])
        out = out + term
    return out


def _rand_unit(rng, n, D):
    v = rng.normal(size=(n, D))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


# 3D septic (512 unknowns, condition ~1e9) is left to the corner-condition test below: its
# numerical rank is not a reliable check in FP64, and it is the tensor product of the same
# 1D bases pinned here in 2D
@pytest.mark.parametrize("D,M", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2)])
def test_closed_form_equals_brute_force_solve(D, M):
    rng = np.random.default_rng(1000 + 10 * D + M)
    for _ in range(3):
        g = _rand_unit(rng, 2 ** D, D)
        c_brute, A, b = _brute_coeffs(D, M, g)
        c_orc = O.coeffs_2d(M, g) if D == 2 else O.coeffs_3d(M, g)
        # the system is square and non-singular, so a zero residual means the
        # oracle's coefficients are its unique solution
        assert np.linalg.matrix_rank(A) == A.shape[0]
        cv = c_orc.reshape(-1)
        scale = np.abs(A) @ np.abs(cv) + np.abs(b)
        assert np.all(np.abs(A @ cv - b) <= 1e-13 * scale + 1e-14)
        # and they match an independent LU solve to within its conditioning
        tol = 1e-13 * np.linalg.cond(A) * max(1.0, np.max(np.abs(c_brute)))
        np.testing.assert_allclose(c_orc, c_brute, atol=tol, rtol=0)
        # the Hermite evaluation equals the polynomial with those coefficients
        for _ in range(20):
            t = rng.random(D)
            h_poly = _poly_eval(c_orc, t)
            h_orc = O.cell_2d(M, g, *t) if D == 2 else O.cell_3d(M, g, *t)
            # rounding of the monomial sum (coefficients reach ~1e4 at M = 4)
            assert abs(h_orc - h_poly) < max(1e-11, 1e-15 * 20 * np.sum(np.abs(c_orc)))


def test_constraint_count_matches_paper():
    # eq. nconstraints: 2^D * sum_{i<=m} C(D+i-1, i) <= (n+1)^D
    def count(D, m):
        return 2 ** D * sum(math.comb(D + i - 1, i) for i in range(m + 1))
    assert count(2, 1) == 12  # the twelve D2M1N3 equations of Sec. 3.1
    assert count(2, 1) <= 4 ** 2
    assert count(3, 2) == 80 and count(3, 2) <= 5 ** 3
    # the tensor set {0..M}^D used here is square with degree n = 2M+1
    for D, M in [(2, 1), (2, 2), (3, 1), (3, 2)]:
        assert 2 ** D * (M + 1) ** D == (2 * M + 2) ** D


@pytest.mark.parametrize("M", [1, 2, 3])
def test_value_basis_is_smoothstep(M):
    """D1M1N3 with h(0)=0, h(1)=1 and zero end slopes is S3 (Sec. 3.4); the quintic
    analogue with zero end curvature is S5 (Sec. 5.1); with the third derivative zero too
    it is the degree-7 smoothstep 35t^4 - 84t^5 + 70t^6 - 20t^7."""
    n1 = 2 * M + 2
    rows, rhs = [], []
    for s, v in ((0, 0.0), (1, 1.0)):
        for d in range(M + 1):
            rows.append([_dmono(a, d, s) for a in range(n1)])
            rhs.append(v if d == 0 else 0.0)
    c = np.linalg.solve(np.array(rows), np.array(rhs))
    for t in np.linspace(0, 1, 37):
        b0, _ = O.basis(M, t)
        paper = (3 * t ** 2 - 2 * t ** 3 if M == 1 else 6 * t ** 5 - 15 * t ** 4 + 10 * t ** 3 if M == 2
                 else 35 * t ** 4 - 84 * t ** 5 + 70 * t ** 6 - 20 * t ** 7)
        assert abs(b0[1] - paper) < 1e-14
        assert abs(b0[1] - np.polyval(c[::-1], t)) < 1e-12
        assert abs(b0[0] + b0[1] - 1.0) < 1e-15  # partition of unity


@pytest.mark.parametrize("D,M", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3), (3, 4)])
def test_corner_values_and_gradients(D, M):
    rng = np.random.default_rng(7 + D + M)
    g = _rand_unit(rng, 2 ** D, D)
    c = O.coeffs_2d(M, g) if D == 2 else O.coeffs_3d(M, g)
    # rounding of a monomial sum with large cancelling coefficients (quintic 3D ~ 1e3,
    # septic ~ 1e4), grown by the falling factorials a derivative of order d multiplies in
    n = 2 * M + 1

    def tol(d):
        return (1e-14 * 25 * np.sum(np.abs(c)) + 1e-15) * np.prod([n ** k for k in d])

    for ci, corner in enumerate(itertools.product((0, 1), repeat=D)):
        corner = corner[::-1]
        assert abs(_poly_eval(c, corner)) < tol((0,) * D)
        for a in range(D):
            d = [0] * D
            d[a] = 1
            assert abs(_poly_eval(c, corner, tuple(d)) - g[ci][a]) < tol(d)
        # every other mixed derivative h^d with 0 <= d_k <= M vanishes
        for d in itertools.product(range(M + 1), repeat=D):
            if sum(d) > 1:
                assert abs(_poly_eval(c, corner, d)) < tol(d)


def test_edge_restriction_is_1d_hermite():
    """On the edge y = 0 the 2D C1 cell is the 1D cubic Hermite interpolant with zero
    end values and end slopes f00, f10 (eq. independance: the edge depends on its two
    corners only)."""
    rng = np.random.default_rng(3)
    g = _rand_unit(rng, 4, 2)
    for t in np.linspace(0, 1, 21):
        h = O.cell_2d(1, g, t, 0.0)
        # textbook cubic Hermite: p0 h00 + m0 h10 + p1 h01 + m1 h11 with p0 = p1 = 0
        herm = g[0][0] * (t ** 3 - 2 * t ** 2 + t) + g[1][0] * (t ** 3 - t ** 2)
        assert abs(h - herm) < 1e-14


@pytest.mark.parametrize("M", [1, 2, 3, 4])
def test_c1_c2_continuity_2d(M):
    """Two cells sharing a face, gradients on a shared 3x3 node grid: value and
    derivatives up to order M agree on the shared faces."""
    rng = np.random.default_rng(11 + M)
    G = _rand_unit(rng, 9, 2).reshape(3, 3, 2)  # [iy][ix]

    def corners(cx, cy):
        return np.array([G[cy + dy][cx + dx] for dy in (0, 1) for dx in (0, 1)])

    cA = O.coeffs_2d(M, corners(0, 0))
    cR = O.coeffs_2d(M, corners(1, 0))  # right neighbour, shared face x = 1 / x = 0
    cU = O.coeffs_2d(M, corners(0, 1))  # upper neighbour, shared face y = 1 / y = 0
    orders = [(i, j) for i in range(M + 1) for j in range(M + 1) if i + j <= M]
    mag = max(np.sum(np.abs(cA)), np.sum(np.abs(cR)), np.sum(np.abs(cU)))
    for s in np.linspace(0, 1, 9):
        for d in orders:
            # rounding grows with the derivative order and the coefficient magnitudes
            tol = max(1e-11 * (2 * M + 1) ** sum(d) / 3 ** sum(d), 1e-15 * mag * (2 * M + 1) ** sum(d))
            assert abs(_poly_eval(cA, (1.0, s), d) - _poly_eval(cR, (0.0, s), d)) < tol
            assert abs(_poly_eval(cA, (s, 1.0), d) - _poly_eval(cU, (s, 0.0), d)) < tol


@pytest.mark.parametrize("M", [1, 2, 3, 4])
def test_c1_c2_continuity_3d(M):
    rng = np.random.default_rng(21 + M)
    G = _rand_unit(rng, 27, 3).reshape(3, 3, 3, 3)  # [iz][iy][ix]

    def corners(cx, cy, cz):
        return np.array([G[cz + dz][cy + dy][cx + dx]
                         for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)])

    c0 = O.coeffs_3d(M, corners(0, 0, 0))
    nb = [O.coeffs_3d(M, corners(1, 0, 0)), O.coeffs_3d(M, corners(0, 1, 0)),
          O.coeffs_3d(M, corners(0, 0, 1))]
    orders = [d for d in itertools.product(range(M + 1), repeat=3) if sum(d) <= M]
    mag = max(np.sum(np.abs(c0)), *(np.sum(np.abs(c)) for c in nb))
    for axis in range(3):
        for _ in range(4):
            p = list(np.random.default_rng(axis).random(3))
            p0 = list(p)
            p1 = list(p)
            p0[axis] = 1.0
            p1[axis] = 0.0
            for d in orders:
                tol = max(1e-10, 1e-15 * mag * (2 * M + 1) ** sum(d))
                assert abs(_poly_eval(c0, p0, d) - _poly_eval(nb[axis], p1, d)) < tol


def _paper_d2m1n3(h, f, g):
    """Coefficients of the paper's D2M1N3 member (Sec. 3.1, eqs. c00..c11 with
    c22 = c23 = c32 = c33 = 0, and the x<->y symmetry rule for c_ji).
    h, f, g are 2x2 arrays indexed [i][j] for corner (i, j)."""
    c = np.zeros((4, 4))
    c[0, 0] = h[0][0]
    c[1, 0] = f[0][0]
    c[2, 0] = 3 * (h[1][0] - h[0][0]) - 2 * f[0][0] - f[1][0]
    c[3, 0] = f[1][0] + f[0][0] - 2 * (h[1][0] - h[0][0])
    c[2, 1] = 3 * (h[1][1] - h[0][1]) - 2 * f[0][1] - f[1][1] - c[2, 0]
    c[3, 1] = f[1][1] + f[0][1] - 2 * (h[1][1] - h[0][1]) - c[3, 0]
    c[1, 1] = h[0][1] + h[1][0] - h[0][0] - h[1][1] + f[0][1] + g[1][0] - g[0][0] - f[0][0]
    # symmetric counterparts: swap the index order and f <-> g
    c[0, 1] = g[0][0]
    c[0, 2] = 3 * (h[0][1] - h[0][0]) - 2 * g[0][0] - g[0][1]
    c[0, 3] = g[0][1] + g[0][0] - 2 * (h[0][1] - h[0][0])
    c[1, 2] = 3 * (h[1][1] - h[1][0]) - 2 * g[1][0] - g[1][1] - c[0, 2]
    c[1, 3] = g[1][1] + g[1][0] - 2 * (h[1][1] - h[1][0]) - c[0, 3]
    return c


def test_paper_member_meets_constraints_but_is_not_c1():
    """Negative control: the member printed in Sec. 3.1 meets its 12 corner
    constraints, yet its normal derivative on a shared edge depends on the far
    corners, so two stacked cells disagree there.  The zero-twist tensor member
    used by the oracle agrees (test_c1_c2_continuity_2d)."""
    rng = np.random.default_rng(5)
    H = rng.normal(size=(3, 2))  # node heights [i][j], nodes i in 0..2 (x), j in 0..1
    F = rng.normal(size=(3, 2))
    Gv = rng.normal(size=(3, 2))
    cA = _paper_d2m1n3(H[0:2], F[0:2], Gv[0:2])
    for i in (0, 1):
        for j in (0, 1):
            assert abs(_poly_eval(cA, (i, j)) - H[i][j]) < 1e-12
            assert abs(_poly_eval(cA, (i, j), (1, 0)) - F[i][j]) < 1e-12
            assert abs(_poly_eval(cA, (i, j), (0, 1)) - Gv[i][j]) < 1e-12
    # right neighbour shares the edge x = 1 (nodes i = 1)
    cB = _paper_d2m1n3(H[1:3], F[1:3], Gv[1:3])
    vals = [abs(_poly_eval(cA, (1.0, s)) - _poly_eval(cB, (0.0, s))) for s in np.linspace(0, 1, 7)]
    assert max(vals) < 1e-12  # C0 holds (edge boundary condition)
    dn = [abs(_poly_eval(cA, (1.0, s), (1, 0)) - _poly_eval(cB, (0.0, s), (1, 0)))
          for s in np.linspace(0, 1, 7)]
    assert max(dn) > 1e-3  # but the normal derivative jumps: not C1


def test_zero_gradient_form_sign():
    """eq. zg: with all corner gradients zero the paper's member reduces to
    h00 + S3(x) dx + S3(y) dy + A [S3(x) y + S3(y) x - x y]; the printed '+ x y'
    misses the corner h(1,1) = h11, the '- x y' reading matches it and the
    general coefficients everywhere."""
    rng = np.random.default_rng(9)
    h = rng.normal(size=(2, 2))
    z = np.zeros((2, 2))
    c = _paper_d2m1n3(h, z, z)
    dx, dy = h[1][0] - h[0][0], h[0][1] - h[0][0]
    A = h[1][1] + h[0][0] - h[1][0] - h[0][1]

    def s3(t):
        return 3 * t * t - 2 * t ** 3

    def zg(x, y, sign):
        return h[0][0] + s3(x) * dx + s3(y) * dy + A * (s3(x) * y + s3(y) * x + sign * x * y)

    assert abs(zg(1, 1, +1) - h[1][1]) > 1e-3
    assert abs(zg(1, 1, -1) - h[1][1]) < 1e-12
    for x, y in rng.random((10, 2)):
        assert abs(zg(x, y, -1) - _poly_eval(c, (x, y))) < 1e-12


@pytest.mark.parametrize("D,M,bound", [(2, 1, 0.5), (2, 2, 0.625), (2, 3, 0.6875), (3, 1, 0.75), (3, 2, 0.9375),
                                       (3, 3, 1.03125)])
def test_cell_bound(D, M, bound):
    """|h| <= D * max_t(|b1_0| + |b1_1|) for unit gradients: 1/4 per axis (cubic),
    5/16 per axis (quintic), 11/32 per axis (septic)."""
    rng = np.random.default_rng(31 * D + M)
    worst = 0.0
    for _ in range(400):
        g = _rand_unit(rng, 2 ** D, D)
        t = rng.random(D)
        h = O.cell_2d(M, g, *t) if D == 2 else O.cell_3d(M, g, *t)
        worst = max(worst, abs(h))
    assert worst <= bound


def test_perlin_cell_corner_data():
    """Perlin's polynomial (Sec. 3.2) is 0 at the nodes with gradient (f, g)."""
    rng = np.random.default_rng(17)
    g = _rand_unit(rng, 4, 2)
    eps = 1e-6
    for order in (3, 5):
        for ci, (cx, cy) in enumerate([(0, 0), (1, 0), (0, 1), (1, 1)]):
            assert abs(O.perlin_cell(order, g, cx, cy)) < 1e-15
            # one-sided difference pointing into the cell
            sx = 1 if cx == 0 else -1
            sy = 1 if cy == 0 else -1
            dfx = (O.perlin_cell(order, g, cx + sx * eps, cy) - O.perlin_cell(order, g, cx, cy)) / (sx * eps)
            dfy = (O.perlin_cell(order, g, cx, cy + sy * eps) - O.perlin_cell(order, g, cx, cy)) / (sy * eps)
            assert abs(dfx - g[ci][0]) < 1e-5
            assert abs(dfy - g[ci][1]) < 1e-5


def _solve_1d_bases(M):
    """The four 1D bases of order M from the 1D corner system (value and derivatives
    1..M prescribed at t = 0 and t = 1), solved here for their monomial coefficients."""
    n1 = 2 * M + 2
    rows = []
    conds = [(s, d) for s in (0, 1) for d in range(M + 1)]
    for s, d in conds:
        rows.append([_dmono(a, d, s) for a in range(n1)])
    A = np.array(rows)
    out = []
    for s, d in [(0, 0), (1, 0), (0, 1), (1, 1)]:  # b0[0], b0[1], b1[0], b1[1]
        rhs = np.array([1.0 if c == (s, d) else 0.0 for c in conds])
        out.append(np.linalg.solve(A, rhs))
    return out


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5, 6])
def test_closed_form_bases_solve_the_1d_corner_system(M):
    """The oracle's closed forms of the 1D bases (two-point Taylor interpolation, any order)
    against an independent solve of the 1D corner system; for M <= 3 also against the
    explicit polynomials the oracle evaluates (S3 / S5 / S7 and their slope bases)."""
    sols = _solve_1d_bases(M)
    tol = 1e-13 * (10 ** (M - 1))  # conditioning of the 1D system grows with M
    for t in np.linspace(0, 1, 33):
        c0, c1 = O.hermite_closed(M, t)
        got = [c0[0], c0[1], c1[0], c1[1]]
        for k in range(4):
            assert abs(got[k] - np.polyval(sols[k][::-1], t)) < tol, (M, k, t)
        e0, e1 = O.basis(M, t)
        assert np.allclose([e0[0], e0[1], e1[0], e1[1]], got, atol=1e-13, rtol=0)
        assert abs(c0[0] + c0[1] - 1.0) < 1e-13  # partition of unity
        # symmetry of the two slope bases: b1[1](t) = -b1[0](1 - t)
        r0, r1 = O.hermite_closed(M, 1.0 - t)
        assert abs(c1[1] + r1[0]) < 1e-13


def test_order_four_rejected_above_six():
    g = np.zeros((4, 2))
    with pytest.raises(ValueError):
        O.fbm_2d(7, 2, 0.5, 2.0, 0.1, 1, 0, 0, 4, 4)
    assert np.isfinite(O.cell_2d(6, g + 0.5, 0.3, 0.7))

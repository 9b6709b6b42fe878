"""Analytic gradient of the height field in the oracle (the gradient maps of Sec. 5.1),
pinned by central differences of the oracle's own value functions (the cells of the
three models, cubic to septic) and by the octave sum: dH/dX = sum_o a_o f_o dh_o/dt."""
import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("M", [1, 2, 3])
def test_basis_derivatives(M):
    e = 1e-6
    for t in np.linspace(0.05, 0.95, 11):
        db0, db1 = O.basis_deriv(M, t)
        p0, p1 = O.basis(M, t + e)
        m0, m1 = O.basis(M, t - e)
        assert np.allclose(db0, (p0 - m0) / (2 * e), atol=1e-8)
        assert np.allclose(db1, (p1 - m1) / (2 * e), atol=1e-8)


def _value(model, M, h, g, w, x, y):
    if model == "gradient":
        return O.cell_2d(M, g, x, y)
    if model == "zero_gradient":
        return O.zg_cell(h, x, y)
    return O.hg_cell(M, h, g, w, x, y)


@pytest.mark.parametrize("model,M", [("gradient", 1), ("gradient", 2), ("gradient", 3), ("zero_gradient", 1),
                                     ("height_gradient", 1), ("height_gradient", 2), ("height_gradient", 3)])
def test_cell_gradient_is_the_derivative_of_the_cell(model, M):
    rng = np.random.default_rng(40 + M)
    e = 1e-6
    for _ in range(10):
        h = rng.uniform(-1, 1, 4)
        ang = rng.uniform(0, 2 * np.pi, 4)
        g = np.stack([np.cos(ang), np.sin(ang)], axis=1)
        w = 0.37
        for x, y in rng.uniform(0.02, 0.98, (6, 2)):
            v = O.cell_2d_grad(model, M, h, g, w, x, y)
            assert v[0] == pytest.approx(_value(model, M, h, g, w, x, y), abs=1e-14)
            fx = (_value(model, M, h, g, w, x + e, y) - _value(model, M, h, g, w, x - e, y)) / (2 * e)
            fy = (_value(model, M, h, g, w, x, y + e) - _value(model, M, h, g, w, x, y - e)) / (2 * e)
            assert v[1] == pytest.approx(fx, abs=1e-7) and v[2] == pytest.approx(fy, abs=1e-7)


@pytest.mark.parametrize("model,M", [("gradient", 1), ("zero_gradient", 1), ("height_gradient", 2)])
def test_field_gradient_sums_octave_cells(model, M):
    f0, lac, pers, w, seed, n = 0.061, 2.0, 0.5, 0.2, 12, 3
    x0, y0 = -(1 << 35) + 1, (1 << 27) + 9
    H, HX, HY = O.fbm_2d_grad(model, M, n, pers, lac, f0, w, seed, x0, y0, 9, 6)
    # H as the value-only routines give it (the same terms, summed in another order)
    if model == "gradient":
        ref = O.fbm_2d(M, n, pers, lac, f0, seed, x0, y0, 9, 6)
    elif model == "zero_gradient":
        ref = O.zg_fbm_2d(n, pers, lac, f0, seed, x0, y0, 9, 6)
    else:
        ref = O.hg_fbm_2d(M, n, pers, lac, f0, w, seed, x0, y0, 9, 6)
    assert np.max(np.abs(H - ref)) < 1e-13
    for j in range(6):
        for i in range(9):
            wx = wy = 0.0
            f, a = f0, 1.0
            for o in range(n):
                cx, tx = O.coord(x0 + i, f)
                cy, ty = O.coord(y0 + j, f)
                keys = [O.key2(cx + dx, cy + dy, o, seed) for dy in (0, 1) for dx in (0, 1)]
                hh = [O.height2(k) if model == "zero_gradient" else O.height2_second(k) for k in keys]
                gg = np.array([O.grad2(k) for k in keys])
                v = O.cell_2d_grad(model, M, hh, gg, w, tx, ty)
                wx += a * f * v[1]
                wy += a * f * v[2]
                f *= lac
                a *= pers
            assert HX[j, i] == wx and HY[j, i] == wy


def _field(model, M, n, pers, lac, f0, w, seed, x0, y0, nx, ny):
    if model == "gradient":
        return O.fbm_2d(M, n, pers, lac, f0, seed, x0, y0, nx, ny)
    if model == "zero_gradient":
        return O.zg_fbm_2d(n, pers, lac, f0, seed, x0, y0, nx, ny)
    return O.hg_fbm_2d(M, n, pers, lac, f0, w, seed, x0, y0, nx, ny)


@pytest.mark.parametrize("model,M", [("gradient", 1), ("gradient", 2), ("gradient", 3), ("zero_gradient", 1),
                                     ("height_gradient", 1), ("height_gradient", 2)])
@pytest.mark.parametrize("n,f0,lac", [(1, 2.0 ** -14, 2.0), (4, 2.0 ** -14, 2.0), (3, 7.11e-5, 1.93)])
def test_world_gradient_is_the_finite_difference_of_the_field(model, M, n, f0, lac):
    """dH/dX and dH/dY in world units against a fourth-order central difference of the
    value-only field over world samples, (-H(X+2) + 8H(X+1) - 8H(X-1) + H(X-2)) / 12.
    The five samples of a stencil lie in one cell of every octave (periods >= 2048
    samples), where each octave is a polynomial of degree 2M+1 in X: the stencil is exact
    for degree <= 4 and its remainder (|X-step|^4 f^5 h^(5) / 30, f <= 2^-11) is below
    1e-15 for higher degrees, so the difference carries only the FP64 rounding of H.
    Power-of-two frequencies place samples exactly at any offset (here up to 2^40); the
    non-dyadic ladder stays within 2^20 samples of the origin, where the FP64 coordinate
    (X + 1/2) f carries below 2e-14 of a cell."""
    pers, w, seed = 0.5, 0.3, 77
    span = 1 << (40 if lac == 2.0 else 20)
    rng = np.random.default_rng(hash((model, M, n)) & 0xFFFF)
    freq, amp = O.octave_params(f0, lac, pers, n)
    scale = float(np.sum(amp * freq))
    checked = 0
    while checked < 25:
        X, Y = (int(v) for v in rng.integers(-span, span, size=2))
        inside = all(np.floor((X - 1.5) * f) == np.floor((X + 2.5) * f) and
                     np.floor((Y - 1.5) * f) == np.floor((Y + 2.5) * f) for f in freq)
        if not inside:
            continue
        _, HX, HY = O.fbm_2d_grad(model, M, n, pers, lac, f0, w, seed, X, Y, 1, 1)
        row = _field(model, M, n, pers, lac, f0, w, seed, X - 2, Y, 5, 1)[0]
        col = _field(model, M, n, pers, lac, f0, w, seed, X, Y - 2, 1, 5)[:, 0]
        st = np.array([1.0, -8.0, 0.0, 8.0, -1.0]) / 12.0
        assert abs(HX[0, 0] - float(st @ row)) <= 1e-9 * scale, (X, Y)
        assert abs(HY[0, 0] - float(st @ col)) <= 1e-9 * scale, (X, Y)
        checked += 1

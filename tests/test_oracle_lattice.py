"""Pins of the oracle's lattice, coordinate step and octave sum (CPU only).

* fmix32 is MurmurHash3's 32-bit finalizer: for an empty input, MurmurHash3_x86_32
  returns fmix32(seed), so its published test vectors pin the constants; the
  finalizer is also inverted here with the modular inverses of its multipliers.
* Gradients: unit norm, and the angle / height recovered by inverse trigonometry
  equals the key bits they are stated to come from; uniformity (chi^2).
* Coordinate step: for power-of-two frequencies it equals integer shift / mask
  arithmetic on 2X + 1 (exact), also at large and negative world offsets.
* Octave sum (Sec. 4): an N-octave field minus the (N-1)-octave field is exactly
  p^(N-1) times the last octave assembled sample by sample; crops of a larger
  field equal fields at the crop origin.
"""
import math

import numpy as np
import pytest

import oracle as O

M32 = 0xFFFFFFFF


def test_fmix32_published_vectors():
    # MurmurHash3_x86_32("", seed) = fmix32(seed ^ 0) for a zero-length input
    assert O.fmix32(0) == 0
    assert O.fmix32(1) == 0x514E28B7
    assert O.fmix32(0xFFFFFFFF) == 0x81F16F39


def _fmix32_inverse(h):
    inv1 = pow(0x85EBCA6B, -1, 1 << 32)
    inv2 = pow(0xC2B2AE35, -1, 1 << 32)

    def unxorshift(x, s):
        y = x
        for _ in range(32 // s + 1):
            y = x ^ (y >> s)
        return y & M32

    h = unxorshift(h, 16)
    h = (h * inv2) & M32
    h = unxorshift(h, 13)
    h = (h * inv1) & M32
    h = unxorshift(h, 16)
    return h


def test_fmix32_is_the_published_bijection():
    rng = np.random.default_rng(0)
    for x in list(rng.integers(0, 1 << 32, size=200, dtype=np.uint64)) + [0, 1, M32, 0x80000000]:
        x = int(x)
        assert _fmix32_inverse(O.fmix32(x)) == x


def test_key_avalanche_and_dependence():
    """Flipping any one bit of an index, the octave or the seed flips each key bit
    with probability close to 1/2."""
    rng = np.random.default_rng(1)
    n = 400
    flips = np.zeros(32)
    total = 0
    for _ in range(n):
        ix, iy = (int(v) for v in rng.integers(-(1 << 40), 1 << 40, size=2))
        o = int(rng.integers(0, 16))
        s = int(rng.integers(0, 1 << 32))
        k0 = O.key2(ix, iy, o, s)
        for var in range(4):
            b = int(rng.integers(0, 32))
            if var == 0:
                k1 = O.key2(ix ^ (1 << b), iy, o, s)
            elif var == 1:
                k1 = O.key2(ix, iy ^ (1 << b), o, s)
            elif var == 2:
                k1 = O.key2(ix, iy, o ^ (1 << (b % 5)), s)
            else:
                k1 = O.key2(ix, iy, o, s ^ (1 << b))
            d = k0 ^ k1
            flips += [(d >> i) & 1 for i in range(32)]
            total += 1
    p = flips / total
    assert np.all(np.abs(p - 0.5) < 0.08)


def test_key_high_words_matter():
    # int64 indices are folded as two 32-bit words: x and x + 2^32 differ
    for x in (0, 5, -7, 123456789):
        assert O.key2(x, 3, 0, 1) != O.key2(x + (1 << 32), 3, 0, 1)
        assert O.key2(3, x, 0, 1) != O.key2(3, x + (1 << 32), 0, 1)
        assert O.key3(3, 4, x, 0, 1) != O.key3(3, 4, x + (1 << 32), 0, 1)
    # x and y are not interchangeable
    assert O.key2(1, 2, 0, 1) != O.key2(2, 1, 0, 1)


def test_grad2_unit_and_angle_bits():
    rng = np.random.default_rng(2)
    for k in rng.integers(0, 1 << 32, size=500, dtype=np.uint64):
        k = int(k)
        g = O.grad2(k)
        assert abs(np.hypot(g[0], g[1]) - 1.0) < 1e-15
        turns = (math.atan2(g[1], g[0]) / (2 * math.pi)) % 1.0
        m = round(turns * (1 << 24)) % (1 << 24)
        assert m == (k >> 8)


def test_grad3_unit_and_height_bits():
    rng = np.random.default_rng(3)
    for k in rng.integers(0, 1 << 32, size=500, dtype=np.uint64):
        k = int(k)
        g = O.grad3(k)
        assert abs(np.linalg.norm(g) - 1.0) < 1e-12
        m1 = round(((1.0 - g[2]) * (1 << 24) - 1.0) / 2.0)
        assert m1 == (k >> 8)
        if abs(g[2]) < 0.999:
            turns = (math.atan2(g[1], g[0]) / (2 * math.pi)) % 1.0
            m2 = round(turns * (1 << 24)) % (1 << 24)
            assert m2 == (O.key3_second(k) >> 8)


def test_gradient_uniformity_chi2():
    """Angles of lattice gradients (2D) and z / azimuth of 3D gradients are uniform:
    chi^2 over 32 bins stays below the 0.999 quantile (~61.1 for 31 dof)."""
    n = 32 * 400
    ang = np.empty(n)
    z = np.empty(n)
    az = np.empty(n)
    i = 0
    for iy in range(80):
        for ix in range(160):
            g = O.grad2(O.key2(ix, iy, 0, 7))
            ang[i] = math.atan2(g[1], g[0])
            g3 = O.grad3(O.key3(ix, iy, 5, 2, 7))
            z[i] = g3[2]
            az[i] = math.atan2(g3[1], g3[0])
            i += 1

    def chi2(v, lo, hi):
        h, _ = np.histogram(v, bins=32, range=(lo, hi))
        e = n / 32
        return np.sum((h - e) ** 2 / e)

    assert chi2(ang, -math.pi, math.pi) < 61.1
    assert chi2(z, -1, 1) < 61.1
    assert chi2(az, -math.pi, math.pi) < 61.1


def test_octave_params_repeated_multiplication():
    f, a = O.octave_params(16 / 8192, 2.0, 0.5, 8)
    assert list(f) == [16 / 8192 * 2 ** o for o in range(8)]
    assert list(a) == [0.5 ** o for o in range(8)]
    f, a = O.octave_params(0.013, 1.9, 0.55, 5)
    ff, aa = 0.013, 1.0
    for o in range(5):
        assert f[o] == ff and a[o] == aa
        ff *= 1.9
        aa *= 0.55


@pytest.mark.parametrize("k", [0, 1, 2, 5, 9, 12])
def test_dyadic_coordinate_step_is_integer_arithmetic(k):
    """With f = 2^-k: (X + 1/2) f = (2X+1) / 2^(k+1), so the cell is an arithmetic
    shift of 2X+1 (floor, also for negatives) and the fraction its low bits."""
    f = 2.0 ** -k
    rng = np.random.default_rng(k)
    xs = [0, -1, 1, -3 * 2 ** 20 - 7, 2 ** 33 + 5, -(2 ** 46), 2 ** 46 - 1]
    xs += [int(v) for v in rng.integers(-(1 << 48), 1 << 48, size=200)]
    for X in xs:
        c, t = O.coord(X, f)
        num = 2 * X + 1
        assert c == num >> (k + 1)
        assert t == (num & ((1 << (k + 1)) - 1)) / 2 ** (k + 1)


def test_fp32_coordinates_fail_at_large_offsets():
    """Why the coordinate step is FP64: at X ~ 2^33 FP32 spacing is 1024 samples, so
    FP32 sample positions collapse and cells are wrong."""
    f = 1.0 / 512
    bad = 0
    for X in range(2 ** 33 + 5, 2 ** 33 + 5 + 600):
        c64, _ = O.coord(X, f)
        u32 = (np.float32(X) + np.float32(0.5)) * np.float32(f)
        if int(np.floor(u32)) != c64:
            bad += 1
    assert bad > 0


def _octave_alone_2d(smooth, o, f, seed, x0, y0, nx, ny):
    out = np.empty((ny, nx))
    for j in range(ny):
        for i in range(nx):
            cx, tx = O.coord(x0 + i, f)
            cy, ty = O.coord(y0 + j, f)
            g = np.array([O.grad2(O.key2(cx + dx, cy + dy, o, seed)) for dy in (0, 1) for dx in (0, 1)])
            out[j, i] = O.cell_2d(smooth, g, tx, ty)
    return out


@pytest.mark.parametrize("smooth", [1, 2])
def test_octave_sum_structure_2d(smooth):
    f0, L, p, seed = 1 / 8, 2.0, 0.5, 3
    x0, y0, nx, ny = -37, 1 << 33, 24, 20
    freq, amp = O.octave_params(f0, L, p, 4)
    prev = O.fbm_2d(smooth, 3, p, L, f0, seed, x0, y0, nx, ny)
    full = O.fbm_2d(smooth, 4, p, L, f0, seed, x0, y0, nx, ny)
    last = _octave_alone_2d(smooth, 3, freq[3], seed, x0, y0, nx, ny)
    np.testing.assert_allclose(full - prev, amp[3] * last, atol=1e-14, rtol=0)
    one = O.fbm_2d(smooth, 1, p, L, f0, seed, x0, y0, nx, ny)
    np.testing.assert_allclose(one, _octave_alone_2d(smooth, 0, f0, seed, x0, y0, nx, ny), atol=0, rtol=0)


def test_octave_sum_structure_3d():
    f0, L, p, seed = 1 / 4, 2.0, 0.5, 9
    a = O.fbm_3d(2, 2, p, L, f0, seed, 5, -6, 7, 6, 5, 4)
    b = O.fbm_3d(2, 1, p, L, f0, seed, 5, -6, 7, 6, 5, 4)
    diff = a - b
    for k in range(4):
        for j in range(5):
            for i in range(6):
                X, Y, Z = 5 + i, -6 + j, 7 + k
                cs = [O.coord(v, f0 * 2) for v in (X, Y, Z)]
                g = np.array([O.grad3(O.key3(cs[0][0] + dx, cs[1][0] + dy, cs[2][0] + dz, 1, seed))
                              for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)])
                h = O.cell_3d(2, g, cs[0][1], cs[1][1], cs[2][1])
                assert abs(diff[k, j, i] - 0.5 * h) < 1e-14


def test_crop_invariance_and_points():
    args = (1, 4, 0.5, 2.0, 8 / 256, 0xDEADBEEF)
    big = O.fbm_2d(*args, -3 * 2 ** 20 - 7 - 5, 2 ** 33 + 5 - 9, 40, 30)
    small = O.fbm_2d(*args, -3 * 2 ** 20 - 7, 2 ** 33 + 5, 20, 12)
    np.testing.assert_array_equal(big[9:21, 5:25], small)
    X = np.array([-3 * 2 ** 20 - 7 + 3, -3 * 2 ** 20 - 7 + 19])
    Y = np.array([2 ** 33 + 5 + 0, 2 ** 33 + 5 + 11])
    pts = O.fbm_points_2d(*args, X, Y)
    assert pts[0] == small[0, 3] and pts[1] == small[11, 19]
    v = O.fbm_3d(2, 3, 0.5, 2.0, 1 / 8, 1, 10, 20, 30, 8, 7, 6)
    w = O.fbm_3d(2, 3, 0.5, 2.0, 1 / 8, 1, 12, 21, 33, 4, 5, 2)
    np.testing.assert_array_equal(v[3:5, 1:6, 2:6], w)
    q = O.fbm_points_3d(2, 3, 0.5, 2.0, 1 / 8, 1, np.array([13]), np.array([22]), np.array([34]))
    assert q[0] == w[1, 1, 1]


def test_field_bounded_by_total_amplitude():
    # |H| <= sum_o p^o |h_o| <= 0.5 A for 2D C1
    h = O.fbm_2d(1, 4, 0.5, 2.0, 8 / 256, 1, 0, 0, 256, 256)
    A = sum(0.5 ** o for o in range(4))
    assert np.max(np.abs(h)) <= 0.5 * A
    assert np.std(h) > 0.02  # not degenerate


def test_rejects_bad_parameters():
    with pytest.raises(ValueError):
        O.fbm_2d(7, 4, 0.5, 2.0, 0.1, 1, 0, 0, 4, 4)  # smoothness 1..6
    with pytest.raises(ValueError):
        O.fbm_2d(1, 0, 0.5, 2.0, 0.1, 1, 0, 0, 4, 4)
    with pytest.raises(ValueError):
        O.fbm_2d(1, 4, 0.5, 2.0, -0.1, 1, 0, 0, 4, 4)

"""The oracle's lattice keys and gradient maps against an independent restatement (CPU only).

The lattice is a stated hash (the paper's Sec. 3.2 only says that a grid of gradients is
generated; the hash, its words and salts are this library's reading, written out in the
public header).  The restatement below is typed from that statement in plain Python
integer arithmetic -- it shares nothing with the oracle's C code -- so a swapped word
order, a swapped salt or a mis-folded negative index in the oracle fails here:

    fmix32(h): h ^= h >> 16; h *= 0x85EBCA6B; h ^= h >> 13; h *= 0xC2B2AE35; h ^= h >> 16
    prefix    = fmix32(fmix32(seed ^ 0x9E3779B9) ^ octave)
    line(k,i) = fmix32(fmix32(k ^ lo32(i)) ^ hi32(i))            (i as 64-bit two's complement)
    key2      = fmix32(line(prefix, iy) ^ line(0x27D4EB2F, ix))
    key3      = fmix32(line(line(prefix, iz), iy) ^ line(0x27D4EB2F, ix))
    second3   = fmix32(key3 ^ 0x165667B1)
    2D gradient: angle 2 pi (key >> 8) / 2^24
    3D gradient: z = 1 - (2 (key >> 8) + 1) / 2^24, azimuth 2 pi (second3 >> 8) / 2^24,
                 radius sqrt(1 - z^2)
"""
import math

import numpy as np
import pytest

import oracle as O

MASK = 0xFFFFFFFF


def r_fmix32(h):
    h &= MASK
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & MASK
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & MASK
    h ^= h >> 16
    return h


def r_line(k, i):
    u = i & 0xFFFFFFFFFFFFFFFF  # two's complement of the int64 index
    k = r_fmix32(k ^ (u & MASK))
    return r_fmix32(k ^ (u >> 32))


def r_prefix(seed, octave):
    return r_fmix32(r_fmix32(seed ^ 0x9E3779B9) ^ octave)


def r_key2(ix, iy, octave, seed):
    return r_fmix32(r_line(r_prefix(seed, octave), iy) ^ r_line(0x27D4EB2F, ix))


def r_key3(ix, iy, iz, octave, seed):
    return r_fmix32(r_line(r_line(r_prefix(seed, octave), iz), iy) ^ r_line(0x27D4EB2F, ix))


def r_second(key):
    return r_fmix32(key ^ 0x165667B1)


def _indices(rng, n):
    """int64 indices: small, negative, around +-2^32 and up to +-2^62."""
    out = []
    for _ in range(n):
        c = int(rng.integers(0, 5))
        if c == 0:
            v = int(rng.integers(-300, 300))
        elif c == 1:
            v = int(rng.integers(-(1 << 31), 1 << 31))
        elif c == 2:
            v = (1 << 32) * int(rng.choice([-1, 1])) + int(rng.integers(-5, 5))
        elif c == 3:
            v = int(rng.integers(-(1 << 46), 1 << 46))
        else:
            v = int(rng.integers(-(1 << 62), 1 << 62))
        out.append(v)
    return out


def test_restated_fmix32_matches_published_vectors():
    # MurmurHash3_x86_32 of the empty input with seed s is fmix32(s)
    assert r_fmix32(1) == 0x514E28B7 and r_fmix32(0xFFFFFFFF) == 0x81F16F39


def test_key2_matches_restatement():
    rng = np.random.default_rng(20250)
    ix = _indices(rng, 2500)
    iy = _indices(rng, 2500)
    for q in range(2500):
        o = q % 16
        seed = int(rng.integers(0, 1 << 32))
        assert O.key2(ix[q], iy[q], o, seed) == r_key2(ix[q], iy[q], o, seed), (ix[q], iy[q], o, seed)


def test_key3_and_second_word_match_restatement():
    rng = np.random.default_rng(20251)
    ix, iy, iz = (_indices(rng, 1500) for _ in range(3))
    for q in range(1500):
        o = (7 * q) % 16
        seed = int(rng.integers(0, 1 << 32))
        k = O.key3(ix[q], iy[q], iz[q], o, seed)
        assert k == r_key3(ix[q], iy[q], iz[q], o, seed), (ix[q], iy[q], iz[q], o, seed)
        assert O.key3_second(k) == r_second(k)


def test_axes_are_not_interchangeable():
    """The word order is part of the statement: swapping x and y (or y and z) changes the key,
    and so does absorbing hi before lo (checked through the restatement's own variants)."""
    rng = np.random.default_rng(20252)
    for _ in range(200):
        a, b = (int(v) for v in rng.integers(-(1 << 40), 1 << 40, size=2))
        if a == b:
            continue
        seed, o = int(rng.integers(0, 1 << 32)), int(rng.integers(0, 16))
        assert O.key2(a, b, o, seed) != O.key2(b, a, o, seed)
        swapped = r_fmix32(r_fmix32(r_prefix(seed, o) ^ ((b & 0xFFFFFFFFFFFFFFFF) >> 32)) ^ (b & MASK))
        wrong = r_fmix32(swapped ^ r_line(0x27D4EB2F, a))
        if (b & MASK) != ((b & 0xFFFFFFFFFFFFFFFF) >> 32):
            assert O.key2(a, b, o, seed) != wrong


def test_gradient_maps_match_restatement():
    rng = np.random.default_rng(20253)
    for k in [0, 1, 255, 256, MASK, 0x80000000] + [int(v) for v in rng.integers(0, 1 << 32, size=3000)]:
        th = 2.0 * math.pi * ((k >> 8) / 16777216.0)
        g2 = O.grad2(k)
        assert abs(g2[0] - math.cos(th)) < 1e-15 and abs(g2[1] - math.sin(th)) < 1e-15
        z = 1.0 - (2.0 * (k >> 8) + 1.0) / 16777216.0
        phi = 2.0 * math.pi * ((r_second(k) >> 8) / 16777216.0)
        r = math.sqrt(max(0.0, 1.0 - z * z))
        g3 = O.grad3(k)
        assert abs(g3[0] - r * math.cos(phi)) < 1e-15
        assert abs(g3[1] - r * math.sin(phi)) < 1e-15
        assert g3[2] == z


def test_fields_use_the_restated_keys():
    """One oracle sample assembled from restated keys and the oracle's cell: the field's
    corner lookup (cell index, corner order, octave number) is the stated one."""
    f0, seed = 1.0 / 64.0, 0xC0FFEE
    X, Y = -(1 << 33) - 17, (1 << 40) + 3
    H = 0.0
    f, a = f0, 1.0
    for o in range(3):
        cx = math.floor((X + 0.5) * f)
        cy = math.floor((Y + 0.5) * f)
        tx, ty = (X + 0.5) * f - cx, (Y + 0.5) * f - cy
        g = []
        for dy in (0, 1):
            for dx in (0, 1):
                k = r_key2(cx + dx, cy + dy, o, seed)
                th = 2.0 * math.pi * ((k >> 8) / 16777216.0)
                g.append([math.cos(th), math.sin(th)])
        H += a * O.cell_2d(1, np.array(g), tx, ty)
        f *= 2.0
        a *= 0.5
    ref = O.fbm_points_2d(1, 3, 0.5, 2.0, f0, seed, [X], [Y])[0]
    assert ref == pytest.approx(H, abs=1e-15)

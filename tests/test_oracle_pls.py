"""Pins of the point-light-source oracle (Sec. 2.4, Eqs. pls_fre and pls_fre_cgh).

* Points on the hologram's pixel grid at one depth: the field is the convolution-form
  Fresnel oracle (itself pinned by brute force and the Gaussian closed form) applied to a
  field holding A_j at those pixels, divided by its quadrature factor dx dy: two
  independent routes (FFT convolution vs direct sum) to the same numbers.
* Several depths: the sum of per-depth convolution-form propagations, each rescaled from
  its own prefactor to the common one.
* The hologram is the real part of the field without its prefactor, checked on the grid
  case against the convolution form directly.
* A point on the axis gives a pattern symmetric under m -> -m, n -> -n (and x <-> y for
  equal pitches); moving the object by s pixels moves the hologram by s pixels.
"""
import math

import numpy as np
import pytest

from oracle import diffraction as D, pls as PL

RNG = np.random.default_rng(777)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def grid_points(n, p, count, z_choices, rng):
    """count distinct pixels of an n x n grid, as (X, Y, Z, A) records (float32-exact)."""
    idx = rng.choice(n * n, size=count, replace=False)
    iy, ix = np.divmod(idx, n)
    pts = np.zeros((count, 4), dtype=np.float32)
    pts[:, 0] = (ix - n // 2) * p
    pts[:, 1] = (iy - n // 2) * p
    pts[:, 2] = rng.choice(z_choices, size=count)
    pts[:, 3] = rng.uniform(0.2, 1.0, count)
    return pts, ix, iy


def test_grid_points_one_depth_match_the_convolution_form():
    n, p, lam, z = 32, 1.0 / 131072, 633e-9, 0.02     # p = 2^-17 m: grid positions FP32-exact
    pts, ix, iy = grid_points(n, p, 40, [0.0], RNG)
    assert np.all(pts[:, 0].astype(np.float64) == (ix - n // 2) * p)
    u1 = np.zeros((n, n), complex)
    u1[iy, ix] = pts[:, 3].astype(np.float64)
    conv = D.fresnel(u1, p, p, lam, z) / (p * p)
    got = PL.field(pts, n, n, p, p, lam, 0.0, 0.0, z)
    tol = 1e-12 + 8 * np.finfo(float).eps * (2 * math.pi / lam) * abs(z)
    assert rel(got, conv) < tol


def test_grid_points_several_depths():
    n, p, lam, oz = 32, 1.0 / 131072, 532e-9, 0.015     # p = 2^-17 m: FP32 exact
    dz = [0.0, 0.0025, -0.004]
    pts, ix, iy = grid_points(n, p, 60, dz, RNG)
    want = np.zeros((n, n), complex)
    for d in dz:
        sel = pts[:, 2] == np.float32(d)
        zd = oz + float(np.float32(d))
        u1 = np.zeros((n, n), complex)
        u1[iy[sel], ix[sel]] = pts[sel, 3].astype(np.float64)
        want += D.fresnel(u1, p, p, lam, zd) / (p * p) * (PL.prefactor(lam, oz) / PL.prefactor(lam, zd))
    got = PL.field(pts, n, n, p, p, lam, 0.0, 0.0, oz)
    tol = 1e-12 + 16 * np.finfo(float).eps * (2 * math.pi / lam) * abs(oz)
    assert rel(got, want) < tol


def test_hologram_is_the_real_part_of_the_wavelet_sum():
    n, p, lam, z = 32, 1.0 / 131072, 633e-9, 0.01
    pts, ix, iy = grid_points(n, p, 30, [0.0], RNG)
    u1 = np.zeros((n, n), complex)
    u1[iy, ix] = pts[:, 3].astype(np.float64)
    conv = D.fresnel(u1, p, p, lam, z) / (p * p * PL.prefactor(lam, z))
    got = PL.cgh(pts, n, n, p, p, lam, 0.0, 0.0, z)
    assert rel(got, conv.real) < 1e-10
    f = PL.field(pts, n, n, p, p, lam, 0.0, 0.0, z) / PL.prefactor(lam, z)
    assert rel(got, f.real) < 1e-13


def test_axis_point_symmetry_and_translation():
    n, p, lam, z = 64, 4e-6, 633e-9, 0.05
    pts = np.array([[0.0, 0.0, 0.0, 1.0]], dtype=np.float32)
    h = PL.cgh(pts, n, n, p, p, lam, 0.0, 0.0, z)
    c = n // 2
    core = h[1:, 1:]                      # indices 1..n-1 are symmetric about c
    assert np.allclose(core, core[::-1, ::-1], rtol=0, atol=1e-12)
    assert np.allclose(h, h.T, rtol=0, atol=1e-12)
    assert h[c, c] == pytest.approx(1.0, abs=1e-15)
    # the object moved by s pixels in x and t in y moves the hologram by (s, t) pixels
    s, t = 5, -3
    moved = PL.cgh(pts, n, n, p, p, lam, s * p, t * p, z)
    assert np.allclose(moved[max(t, 0):n + min(t, 0), max(s, 0):n + min(s, 0)],
                       h[max(-t, 0):n + min(-t, 0), max(-s, 0):n + min(-s, 0)], rtol=0, atol=1e-9)


def test_zone_plate_radii():
    # one point on the axis: I = cos(pi r^2/(lambda z)) changes sign at
    # r^2 = lambda z (k + 1/2) (Fresnel zone plate), found along the centre row
    n, p, lam, z = 1024, 2e-6, 500e-9, 0.1
    pts = np.array([[0.0, 0.0, 0.0, 1.0]], dtype=np.float32)
    row = PL.cgh(pts, n, n, p, p, lam, 0.0, 0.0, z, rows=[n // 2])[0]
    x = (np.arange(n) - n // 2) * p
    right = row[n // 2:]
    flips = np.nonzero(np.sign(right[1:]) != np.sign(right[:-1]))[0]
    xs = x[n // 2:]
    assert len(flips) >= 6
    for k, i in enumerate(flips[:6]):
        rk = math.sqrt(lam * z * (k + 0.5))
        assert xs[i] <= rk <= xs[i + 1]


def test_rows_and_invalid():
    pts = RNG.uniform(-1e-4, 1e-4, (20, 4)).astype(np.float32)
    pts[:, 3] = 1.0
    full = PL.cgh(pts, 32, 16, 5e-6, 6e-6, 633e-9, 1e-4, -2e-4, 0.1)
    part = PL.cgh(pts, 32, 16, 5e-6, 6e-6, 633e-9, 1e-4, -2e-4, 0.1, rows=[2, 11])
    assert np.array_equal(part, full[[2, 11]])
    with pytest.raises(ValueError):
        PL.cgh(pts, 32, 16, 5e-6, 6e-6, 633e-9, 0, 0, 0.0)
    with pytest.raises(ValueError):
        PL.cgh(pts[:, :3], 32, 16, 5e-6, 6e-6, 633e-9, 0, 0, 0.1)
    with pytest.raises(ValueError):
        PL.field(pts, 32, 16, -5e-6, 6e-6, 633e-9, 0, 0, 0.1)

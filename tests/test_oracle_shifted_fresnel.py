"""Pins of the shifted Fresnel oracle (Sec. 2.1.3, Eqs. shift_fre1 - shift_fre3).

* equal pitches and zero offsets reduce it to the convolution-form oracle, which has
  its own brute-force and closed-form pins;
* an off-axis Gaussian beam between windows of different pitches and offsets against
  the closed form of the Fresnel integral (translation invariance of free space);
* a naive quadruple loop over the unseparated 2-D kernel on a small grid.
"""
import math

import numpy as np
import pytest

from oracle import diffraction as D, shifted_fresnel as SF

RNG = np.random.default_rng(4242)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def test_equal_pitch_no_offset_is_the_convolution_form():
    u = RNG.standard_normal((32, 64)) + 1j * RNG.standard_normal((32, 64))
    dx, dy, lam, z = 8e-6, 10e-6, 532e-9, 0.04
    got = SF.propagate(u, dx, dy, dx, dy, lam, z)
    # FP64 phases of size k z carry ~eps * k |z| of representation error on both sides
    tol = 1e-12 + 8 * np.finfo(float).eps * (2 * math.pi / lam) * abs(z)
    assert rel(got, D.fresnel(u, dx, dy, lam, z)) < tol


def test_off_axis_gaussian_between_different_grids():
    n, lam, w0, z = 128, 633e-9, 100e-6, 0.05
    p0, p1 = 10e-6, 6e-6
    ox0, oy0, ox1, oy1 = 3e-4, -2e-4, 3e-4, -1e-4
    a, b = 3.2e-4, -1.8e-4   # beam centre, > 5.8 w0 from the source window's edges
    x0 = (np.arange(n) - n // 2) * p0
    u0 = np.exp(-(((x0 + oy0 - b) ** 2)[:, None] + ((x0 + ox0 - a) ** 2)[None, :]) / w0 ** 2)
    x1 = (np.arange(n) - n // 2) * p1
    r2 = ((x1 + oy1 - b) ** 2)[:, None] + ((x1 + ox1 - a) ** 2)[None, :]
    q = 1 + 1j * z / (math.pi * w0 ** 2 / lam)
    expect = np.exp(1j * 2 * math.pi / lam * z) / q * np.exp(-r2 / (w0 ** 2 * q))
    got = SF.propagate(u0, p0, p0, p1, p1, lam, z, ox0, oy0, ox1, oy1)
    assert rel(got, expect) < 1e-10


def test_naive_quadruple_loop():
    ny, nx = 16, 16
    u = RNG.standard_normal((ny, nx)) + 1j * RNG.standard_normal((ny, nx))
    dx0, dy0, dx1, dy1 = 9e-6, 7e-6, 5e-6, 11e-6
    lam, z = 473e-9, -0.02
    ox0, oy0, ox1, oy1 = 1e-5, -3e-5, 4e-5, 2e-5
    x0 = (np.arange(nx) - nx // 2) * dx0 + ox0
    y0 = (np.arange(ny) - ny // 2) * dy0 + oy0
    x1 = (np.arange(nx) - nx // 2) * dx1 + ox1
    y1 = (np.arange(ny) - ny // 2) * dy1 + oy1
    c = np.exp(1j * 2 * math.pi / lam * z) / (1j * lam * z) * dx0 * dy0
    want = np.zeros((ny, nx), complex)
    for a in range(ny):
        for b in range(nx):
            ph = math.pi * ((x1[b] - x0[None, :]) ** 2 + (y1[a] - y0[:, None]) ** 2) / (lam * z)
            want[a, b] = c * np.sum(u * np.exp(1j * ph))
    tol = 1e-12 + 8 * np.finfo(float).eps * (2 * math.pi / lam) * abs(z)
    assert rel(SF.propagate(u, dx0, dy0, dx1, dy1, lam, z, ox0, oy0, ox1, oy1), want) < tol


def test_row_subset_and_invalid():
    u = RNG.standard_normal((32, 32)) + 0j
    full = SF.propagate(u, 8e-6, 8e-6, 5e-6, 5e-6, 633e-9, 0.1, 1e-4, 0, -2e-4, 3e-5)
    part = SF.propagate(u, 8e-6, 8e-6, 5e-6, 5e-6, 633e-9, 0.1, 1e-4, 0, -2e-4, 3e-5, rows=[3, 17])
    assert np.array_equal(part, full[[3, 17]])
    with pytest.raises(ValueError):
        SF.propagate(u, 8e-6, 8e-6, 5e-6, 5e-6, 633e-9, 0.0)
    with pytest.raises(ValueError):
        SF.propagate(u, 8e-6, 8e-6, 0.0, 5e-6, 633e-9, 0.1)
    with pytest.raises(ValueError):
        SF.propagate(u, 8e-6, 8e-6, 5e-6, 5e-6, 633e-9, 0.1, math.inf)

"""Pins of the shifted angular spectrum oracle (Sec. 2.1.5, Eqs. shift_ang1, shift_ang2).

Each pin checks the oracle against something other than itself: a brute-force
circular convolution of the plain transfer function read at translated output
positions (the linear phase), closed-form plane waves (the band-limit masks and
their boundary), and a numerical derivative of the transfer function's phase
(the on-axis band-limit width).
"""
import math

import numpy as np
import pytest

from oracle import dft, diffraction as D, shifted_asm as S

RNG = np.random.default_rng(1107)


def crandn(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _full_circular(u1, dx, dy, lam, z):
    """The whole 2N x 2N circular convolution u1 (*) g, g = IDFT_M(H_A), by direct sums."""
    ny, nx = u1.shape
    my, mx = 2 * ny, 2 * nx
    g = dft.dft2_direct(D.asm_transfer(my, mx, dy, dx, lam, z), inverse=True) / (mx * my)
    full = np.zeros((my, mx), complex)
    jy = np.arange(ny)[:, None]
    jx = np.arange(nx)[None, :]
    for ym in range(my):
        for xm in range(mx):
            full[ym, xm] = np.sum(u1 * g[(ym - jy) % my, (xm - jx) % mx])
    return full


@pytest.mark.parametrize("a,b", [(5, -3), (-7, 11), (20, 1), (0, 0)])
def test_whole_pixel_shift_translates_the_window(a, b):
    # with Ox = a*dx, Oy = b*dy the output is the circular result read at (m + a, n + b)
    ny, nx = 16, 16
    dx, dy, lam, z = 6e-6, 9e-6, 633e-9, 0.015
    u1 = crandn(ny, nx)
    full = _full_circular(u1, dx, dy, lam, z)
    want = full[(np.arange(ny)[:, None] + b) % (2 * ny), (np.arange(nx)[None, :] + a) % (2 * nx)]
    got = S.propagate(u1, dx, dy, lam, z, ox=a * dx, oy=b * dy)
    assert rel(got, want) < 1e-12


def _plane_wave(n, p0, q0):
    j = np.arange(n)
    return np.exp(2j * math.pi * (q0 * j[:, None] + p0 * j[None, :]) / n)


def _shifted_plane_wave_out(n, p0, q0, d, lam, z, ox, oy):
    # closed form: u * exp(i z sqrt(k^2 - 4 pi^2 f^2)) * exp(i 2 pi (ox fx + oy fy))
    fx, fy = p0 / (n * d), q0 / (n * d)
    k = 2.0 * math.pi / lam
    kappa = math.sqrt(k * k - 4.0 * math.pi ** 2 * (fx * fx + fy * fy))
    return _plane_wave(n, p0, q0) * np.exp(1j * (z * kappa + 2.0 * math.pi * (ox * fx + oy * fy)))


def _phase_tol(lam, z):
    # an FP64 phase of size k*|z| carries a representation error of a few ulps of it
    return 1e-12 + 8.0 * np.finfo(float).eps * (2.0 * math.pi / lam) * abs(z)


def test_band_limit_passes_and_stops_plane_waves():
    n, d, lam, z = 32, 8e-6, 532e-9, 0.03
    ox, oy = 3.3e-5, -1.7e-5
    df = 1.0 / (n * d)
    u_in = _plane_wave(n, 5, -3)
    u_out = _plane_wave(n, -9, 4)
    u = u_in + u_out
    # x band centred at +2 bins, 16 bins wide: keeps fx = 5 df, drops fx = -9 df
    got = S.propagate(u, d, d, lam, z, ox=ox, oy=oy, cx=2 * df, wx=16 * df, nopad=True)
    want = _shifted_plane_wave_out(n, 5, -3, d, lam, z, ox, oy)
    assert rel(got, want) < _phase_tol(lam, z)
    # a y band that excludes q = -3 as well leaves nothing at all
    got0 = S.propagate(u, d, d, lam, z, ox=ox, oy=oy, cx=2 * df, wx=16 * df, cy=8 * df,
                       wy=4 * df, nopad=True)
    assert np.max(np.abs(got0)) < 1e-13


def test_band_limit_boundary_is_inside():
    # (f - c)/w == 1/2 exactly counts as inside the band
    n, d, lam, z = 32, 8e-6, 532e-9, 0.03
    df = 1.0 / (n * d)
    u = _plane_wave(n, 6, 0)
    got = S.propagate(u, d, d, lam, z, cx=0.0, wx=12 * df, nopad=True)
    assert rel(got, _shifted_plane_wave_out(n, 6, 0, d, lam, z, 0.0, 0.0)) < _phase_tol(lam, z)
    got = S.propagate(u, d, d, lam, z, cx=0.0, wx=11.999 * df, nopad=True)
    assert np.max(np.abs(got)) < 1e-13


def test_on_axis_band_limit_is_the_phase_nyquist_frequency():
    # at f = w/2 the transfer function's phase advances by pi per frequency step:
    # phi(f) = 2 pi z sqrt(1/lambda^2 - f^2), checked with the analytic derivative and
    # with a central difference
    for n, d, lam, z in [(1024, 8e-6, 532e-9, 0.5), (256, 10e-6, 633e-9, 2.0),
                         (2048, 4e-6, 473e-9, 0.05)]:
        f = S.band_limit(n, d, lam, z) / 2.0
        df = 1.0 / (2 * n * d)
        slope = 2.0 * math.pi * z * f / math.sqrt(1.0 / lam ** 2 - f * f)
        assert abs(slope * df - math.pi) < 1e-12 * math.pi

        def phase(fx):
            return 2.0 * math.pi * z * math.sqrt(1.0 / lam ** 2 - fx * fx)

        h = f * 1e-4
        num = abs(phase(f + h) - phase(f - h)) / (2.0 * h)
        assert abs(num * df - math.pi) < 1e-5 * math.pi


def test_no_shift_no_limit_is_the_plain_method():
    u = crandn(16, 32)
    assert rel(S.propagate(u, 6e-6, 9e-6, 633e-9, 0.02), D.asm(u, 6e-6, 9e-6, 633e-9, 0.02)) < 1e-15


def test_invalid_shift_parameters():
    u = crandn(16, 16)
    with pytest.raises(ValueError):
        S.propagate(u, 6e-6, 6e-6, 633e-9, 0.02, ox=math.nan)
    with pytest.raises(ValueError):
        S.propagate(u, 6e-6, 6e-6, 633e-9, 0.02, wy=math.inf)

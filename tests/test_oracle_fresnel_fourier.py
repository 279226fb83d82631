"""Pins of the Fresnel Fourier-form oracle (Sec. 2.1.2, Eqs. fre_fourier1 - fre_fourier3).

* a brute-force double sum of Eq. fre_fourier1 over explicit coordinates (no DFT, no
  index arithmetic) on small rectangular grids;
* the Gaussian-beam closed form of the Fresnel integral, evaluated on the Fourier
  form's destination grid (fixes the destination pitch, the chirps, the constant and
  the quadrature factor);
* the direct and FFT routes of the centred DFT agree.
"""
import math

import numpy as np
import pytest

from oracle import fresnel_fourier as F

RNG = np.random.default_rng(2112)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _brute(u1, dx, dy, lam, z):
    ny, nx = u1.shape
    x1 = (np.arange(nx) - nx // 2) * dx
    y1 = (np.arange(ny) - ny // 2) * dy
    dx2, dy2 = lam * z / (nx * dx), lam * z / (ny * dy)
    x2 = (np.arange(nx) - nx // 2) * dx2
    y2 = (np.arange(ny) - ny // 2) * dy2
    k = 2 * math.pi / lam
    pre = u1 * np.exp(1j * math.pi * (y1[:, None] ** 2 + x1[None, :] ** 2) / (lam * z))
    out = np.zeros((ny, nx), complex)
    for a in range(ny):
        for b in range(nx):
            ker = np.exp(-2j * math.pi * (x2[b] * x1[None, :] + y2[a] * y1[:, None]) / (lam * z))
            out[a, b] = np.sum(pre * ker) * dx * dy
    post = np.exp(1j * math.pi * (y2[:, None] ** 2 + x2[None, :] ** 2) / (lam * z))
    return np.exp(1j * k * z) / (1j * lam * z) * post * out


@pytest.mark.parametrize("shape,dx,dy,z", [((16, 16), 10e-6, 10e-6, 0.05),
                                          ((16, 32), 8e-6, 12e-6, 0.02),
                                          ((32, 16), 6e-6, 6e-6, -0.03)])
def test_brute_force_double_sum(shape, dx, dy, z):
    lam = 633e-9
    u1 = RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)
    want = _brute(u1, dx, dy, lam, z)
    # the brute force carries k z and x^2/(lambda z) unreduced: FP64 phase error ~ eps * k|z|
    tol = 1e-12 + 8 * np.finfo(float).eps * (2 * math.pi / lam) * abs(z)
    assert rel(F.propagate(u1, dx, dy, lam, z), want) < tol


def test_gaussian_closed_form_on_the_destination_grid():
    # u1 = exp(-r^2/w0^2) -> e^{ikz}/q exp(-r2^2/(w0^2 q)), q = 1 + i z/zR, zR = pi w0^2/lam
    n, d, lam, w0, z = 256, 10e-6, 633e-9, 200e-6, 0.1
    c1 = (np.arange(n) - n // 2) * d
    u1 = np.exp(-(c1[:, None] ** 2 + c1[None, :] ** 2) / w0 ** 2)
    d2 = F.destination_pitch(n, d, lam, z)
    c2 = (np.arange(n) - n // 2) * d2
    r2 = c2[:, None] ** 2 + c2[None, :] ** 2
    q = 1 + 1j * z / (math.pi * w0 ** 2 / lam)
    expect = np.exp(1j * 2 * math.pi / lam * z) / q * np.exp(-r2 / (w0 ** 2 * q))
    assert rel(F.propagate(u1, d, d, lam, z), expect) < 1e-10


def test_direct_and_fft_routes_agree():
    a = RNG.standard_normal((64, 128)) + 1j * RNG.standard_normal((64, 128))
    assert rel(F.centred_dft2(a, "fft"), F.centred_dft2(a, "direct")) < 1e-13


def test_destination_pitch_and_invalid():
    assert F.destination_pitch(512, 10e-6, 633e-9, 0.2) == pytest.approx(633e-9 * 0.2 / (512 * 10e-6))
    with pytest.raises(ValueError):
        F.propagate(np.ones((16, 16)), 10e-6, 10e-6, 633e-9, 0.0)
    with pytest.raises(ValueError):
        F.propagate(np.ones((16, 16)), -1e-6, 10e-6, 633e-9, 0.1)

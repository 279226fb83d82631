"""Oracle: Fresnel diffraction, Fourier form, FP64 (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this module; it shares nothing with the product library.

Sec. 2.1.2 (Eqs. fre_fourier1 - fre_fourier3): expanding the quadratic term of the
Fresnel integral gives one Fourier transform of the field times a chirp,

    u'(x1, y1) = u(x1, y1) exp(i pi (x1^2 + y1^2) / (lambda z))
    u(x2, y2)  = exp(i k z)/(i lambda z) exp(i pi (x2^2 + y2^2)/(lambda z))
                 * sum u'(x1, y1) exp(-i 2 pi (x2 x1 + y2 y1)/(lambda z)) dx1 dy1

on N x N samples without padding (one FFT, Table of diffraction classes).

Readings of points the paper leaves open:

* Sample positions are centred: array index j is coordinate (j - N/2) * pitch on
  both planes (the paper's index range -N/2 <= m < N/2).
* The destination pitch is printed as dx1/(lambda z), which is not a length; the
  kernel exp(-i 2 pi x2 x1/(lambda z)) becomes the DFT kernel exp(-i 2 pi m1 m2/N)
  only for dx2 = lambda z/(N dx1), which is taken (dy2 likewise with Ny, dy1). For
  z < 0 the pitch is negative: the destination axes are mirrored.
* The second product in the exponent of Eq. fre_fourier1 is read as y2*y1.
* The sum carries the quadrature factor dx1*dy1 of the integral, as the convolution
  form does.
* z must be non-zero (the form is singular at z = 0).
"""
from __future__ import annotations

import math

import numpy as np

from . import _native

_DIRECT_MAX = 256


def destination_pitch(n: int, d: float, wavelength: float, z: float) -> float:
    """dx2 = lambda z / (N dx1)."""
    return wavelength * z / (n * d)


def centred(n: int) -> np.ndarray:
    """Centred sample index m = j - N/2 of array index j."""
    return np.arange(n, dtype=np.float64) - n // 2


def chirp(x: np.ndarray, wavelength: float, z: float) -> np.ndarray:
    """exp(i pi x^2/(lambda z)), the phase reduced modulo one revolution in FP64."""
    t = (x * x) / (2.0 * wavelength * z)
    r = t - np.rint(t)
    return np.cos(2.0 * math.pi * r) + 1j * np.sin(2.0 * math.pi * r)


def constant(dx: float, dy: float, wavelength: float, z: float) -> complex:
    """dx1 dy1 exp(i k z)/(i lambda z), k z reduced modulo 2 pi in FP64."""
    t = z / wavelength
    r = t - round(t)
    ang = 2.0 * math.pi * r
    return dx * dy * complex(math.cos(ang), math.sin(ang)) / (1j * wavelength * z)


def centred_dft2(a: np.ndarray, method: str = "auto") -> np.ndarray:
    """A[k2, k1] = sum a[j2, j1] exp(-i 2 pi ((j1 - N1/2)(k1 - N1/2)/N1 + (j2 - N2/2)(k2 - N2/2)/N2)).

    Small sizes: the definition as a matrix product with exact integer angles. Larger:
    the textbook FFT between the usual index shifts (the centred DFT is the plain DFT
    of the half-rotated array, half-rotated back)."""
    ny, nx = a.shape
    if method == "direct" or (method == "auto" and max(a.shape) <= _DIRECT_MAX):
        def mat(n):
            m = centred(n).astype(np.int64)
            e = np.mod(np.outer(m, m), n).astype(np.float64) / n
            return np.cos(2 * math.pi * e) - 1j * np.sin(2 * math.pi * e)
        return mat(ny) @ a @ mat(nx).T
    shifted = np.roll(a, (-(ny // 2), -(nx // 2)), axis=(0, 1))
    return np.roll(_native.fft2(shifted, False), (ny // 2, nx // 2), axis=(0, 1))


def propagate(u1: np.ndarray, dx: float, dy: float | None = None, wavelength: float = 633e-9,
              z: float = 0.1, method: str = "auto") -> np.ndarray:
    """u2 on the destination grid (pitches lambda z/(N dx1), lambda z/(N dy1))."""
    dy = dx if dy is None else dy
    u1 = np.asarray(u1)
    if u1.ndim != 2:
        raise ValueError("field must be 2-D [ny][nx]")
    for v, name in ((dx, "dx"), (dy, "dy"), (wavelength, "wavelength")):
        if not (math.isfinite(v) and v > 0):
            raise ValueError("%s must be finite and > 0" % name)
    if not math.isfinite(z) or z == 0.0:
        raise ValueError("z must be finite and non-zero")
    ny, nx = u1.shape
    x1 = centred(nx) * dx
    y1 = centred(ny) * dy
    up = u1.astype(np.complex128) * chirp(y1, wavelength, z)[:, None] * chirp(x1, wavelength, z)[None, :]
    spec = centred_dft2(up, method)
    x2 = centred(nx) * destination_pitch(nx, dx, wavelength, z)
    y2 = centred(ny) * destination_pitch(ny, dy, wavelength, z)
    post = chirp(y2, wavelength, z)[:, None] * chirp(x2, wavelength, z)[None, :]
    return constant(dx, dy, wavelength, z) * post * spec

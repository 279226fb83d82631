"""Oracle: point-light-source (PLS) field and hologram, FP64 direct sums (test
infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this module; it shares nothing with the product library.

Sec. 2.4 (Eqs. pls_fre and pls_fre_cgh) treats a 3-D object as N point sources
(x_j, y_j, z_j) with amplitudes A_j and sums their Fresnel wavelets on the hologram
plane:

    u(x, y) = exp(i k z)/(i lambda z) * sum_j A_j exp(i pi ((x - x_j)^2 + (y - y_j)^2)/(lambda z_j))
    I(x, y) = sum_j A_j cos(pi ((x - x_j)^2 + (y - y_j)^2)/(lambda z_j))

(k = 2 pi/lambda; pi r^2/(lambda z_j) is the paper's (2 pi/lambda) r^2/(2 z_j)). Both are
O(N Nx Ny) sums with no transform; the oracle evaluates them term by term.

Readings of points the paper leaves open:

* The printed exponent of the field lacks the imaginary unit; the Fresnel wavelet
  exp(+i pi r^2/(lambda z_j)) is meant (the sign of the convolution form's impulse
  response, so a point on the grid reproduces that form).
* The prefactor exp(i k z)/(i lambda z) sits outside the sum with one distance z: the
  object's reference distance, the third offset of the listing of Sec. 2.4.
* Hologram pixel (m, n) is at x = (m - Nx/2) px, y = (n - Ny/2) py (centred, as the
  other readings); point j is at (ox + X_j, oy + Y_j, oz + Z_j) with (X_j, Y_j, Z_j) the
  object's own coordinates and (ox, oy, oz) its offset.
* A_j (called a light intensity) enters linearly, as printed.
* Points are passed as FP32 (X, Y, Z, A) records, as the library takes them; the oracle
  upcasts those exact values. Phases are reduced modulo one revolution in FP64 before the
  cosine and sine.
"""
from __future__ import annotations

import math

import numpy as np


def centred(n: int, pitch: float) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) - n // 2) * pitch


def _check(points, nx, ny, px, py, wavelength, oz):
    pts = np.asarray(points)
    if pts.ndim != 2 or pts.shape[1] != 4:
        raise ValueError("points must be [N][4] (X, Y, Z, A)")
    if nx <= 0 or ny <= 0:
        raise ValueError("hologram sizes must be positive")
    for v, name in ((px, "px"), (py, "py"), (wavelength, "wavelength")):
        if not (math.isfinite(v) and v > 0):
            raise ValueError("%s must be finite and > 0" % name)
    if not math.isfinite(oz) or oz == 0.0:
        raise ValueError("the reference distance must be finite and non-zero")
    return pts.astype(np.float32).astype(np.float64)


def _phase_sums(points, nx, ny, px, py, wavelength, ox, oy, oz, rows, want_sin):
    pts = _check(points, nx, ny, px, py, wavelength, oz)
    x = centred(nx, px)
    y = centred(ny, py)
    if rows is not None:
        y = y[np.asarray(rows)]
    xj = ox + pts[:, 0]
    yj = oy + pts[:, 1]
    zj = oz + pts[:, 2]
    aj = pts[:, 3]
    re = np.zeros((len(y), nx))
    im = np.zeros((len(y), nx)) if want_sin else None
    for j in range(len(pts)):
        # phase in revolutions: r^2 / (2 lambda z_j), reduced modulo one
        t = (((x - xj[j]) ** 2)[None, :] + ((y - yj[j]) ** 2)[:, None]) / (2.0 * wavelength * zj[j])
        r = t - np.rint(t)
        re += aj[j] * np.cos(2.0 * math.pi * r)
        if want_sin:
            im += aj[j] * np.sin(2.0 * math.pi * r)
    return re, im


def cgh(points, nx: int, ny: int, px: float, py: float, wavelength: float,
        ox: float, oy: float, oz: float, rows=None) -> np.ndarray:
    """The hologram I(x, y) [ny][nx] (or only the rows in `rows`), FP64."""
    re, _ = _phase_sums(points, nx, ny, px, py, wavelength, ox, oy, oz, rows, False)
    return re


def prefactor(wavelength: float, z: float) -> complex:
    """exp(i k z)/(i lambda z), k z reduced modulo one revolution in FP64."""
    t = z / wavelength
    ang = 2.0 * math.pi * (t - round(t))
    return complex(math.cos(ang), math.sin(ang)) / (1j * wavelength * z)


def field(points, nx: int, ny: int, px: float, py: float, wavelength: float,
          ox: float, oy: float, oz: float, rows=None) -> np.ndarray:
    """The complex field u(x, y) [ny][nx] (or only the rows in `rows`), FP64."""
    re, im = _phase_sums(points, nx, ny, px, py, wavelength, ox, oy, oz, rows, True)
    return prefactor(wavelength, oz) * (re + 1j * im)

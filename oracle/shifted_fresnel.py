"""Oracle: shifted Fresnel diffraction, FP64 (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this module; it shares nothing with the product library.

Sec. 2.1.3 (Eqs. shift_fre1 - shift_fre3) computes, with arbitrary pitches on both
planes and windows shifted off the axis, the discretised Fresnel integral

    u1[m1, n1] = exp(i k z)/(i lambda z) dx0 dy0
                 * sum_{m0, n0} u0[m0, n0] exp(i pi ((x1 - x0)^2 + (y1 - y0)^2)/(lambda z))
    x0 = m0 px0 + Ox0, y0 = n0 py0 + Oy0   (source plane)
    x1 = m1 px1 + Ox1, y1 = n1 py1 + Oy1   (destination plane)

by a chirp convolution (two chirp multiplications around a 2N x 2N convolution with
h[m, n] = exp(i pi (Sx m^2 + Sy n^2)), Sx = px0 px1/(lambda z)). That route reaches
this sum exactly up to rounding, so the oracle is the sum itself: the kernel separates
into x and y factors and the sum is two matrix products.

Readings of points the paper leaves open:

* Indices are centred, m = j - N/2 for array index j, on both planes (the paper's
  range -N/2 <= m < N/2); so (Ox0, Oy0) and (Ox1, Oy1) are the window centres.
* In the paper's C_S and u', the offset products are garbled (a length times a length
  over lambda z where a pure number is needed); the sum above fixes them.
* The sum carries the quadrature factor dx0 dy0, as the convolution form does.
* z must be non-zero.
"""
from __future__ import annotations

import math

import numpy as np


def centred(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) - n // 2


def kernel_1d(n1: int, p1: float, o1: float, n0: int, p0: float, o0: float,
              wavelength: float, z: float, rows: np.ndarray | None = None) -> np.ndarray:
    """K[m1, m0] = exp(i pi (x1 - x0)^2/(lambda z)), phase reduced modulo one revolution
    in FP64 (only the destination indices in `rows` when given)."""
    m1 = centred(n1) if rows is None else np.asarray(rows, dtype=np.float64) - n1 // 2
    x1 = m1 * p1 + o1
    x0 = centred(n0) * p0 + o0
    d = x1[:, None] - x0[None, :]
    t = (d * d) / (2.0 * wavelength * z)
    r = t - np.rint(t)
    return np.cos(2.0 * math.pi * r) + 1j * np.sin(2.0 * math.pi * r)


def constant(dx0: float, dy0: float, wavelength: float, z: float) -> complex:
    """dx0 dy0 exp(i k z)/(i lambda z), k z reduced modulo 2 pi in FP64."""
    t = z / wavelength
    r = t - round(t)
    ang = 2.0 * math.pi * r
    return dx0 * dy0 * complex(math.cos(ang), math.sin(ang)) / (1j * wavelength * z)


def _check(u0, dx0, dy0, dx1, dy1, wavelength, z, offs):
    u0 = np.asarray(u0)
    if u0.ndim != 2:
        raise ValueError("field must be 2-D [ny][nx]")
    for v, name in ((dx0, "dx0"), (dy0, "dy0"), (dx1, "dx1"), (dy1, "dy1"),
                    (wavelength, "wavelength")):
        if not (math.isfinite(v) and v > 0):
            raise ValueError("%s must be finite and > 0" % name)
    if not math.isfinite(z) or z == 0.0:
        raise ValueError("z must be finite and non-zero")
    if not all(math.isfinite(v) for v in offs):
        raise ValueError("offsets must be finite")
    return u0


def propagate(u0: np.ndarray, dx0: float, dy0: float, dx1: float, dy1: float,
              wavelength: float, z: float, ox0: float = 0.0, oy0: float = 0.0,
              ox1: float = 0.0, oy1: float = 0.0, rows=None) -> np.ndarray:
    """The destination field [Ny][Nx] (or only the destination rows `rows`)."""
    u0 = _check(u0, dx0, dy0, dx1, dy1, wavelength, z, (ox0, oy0, ox1, oy1))
    ny, nx = u0.shape
    kx = kernel_1d(nx, dx1, ox1, nx, dx0, ox0, wavelength, z)
    ky = kernel_1d(ny, dy1, oy1, ny, dy0, oy0, wavelength, z, rows)
    return constant(dx0, dy0, wavelength, z) * (ky @ u0.astype(np.complex128) @ kx.T)

"""Oracle: shifted angular spectrum method, FP64 (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this module; it shares nothing with the product library.

Sec. 2.1.5 (Eqs. shift_ang1, shift_ang2): the angular-spectrum pipeline of
Eq. ang3 with the transfer function replaced by

    H_SA(fx, fy) = H_A(fx, fy) * exp(i*2*pi*(Ox*fx + Oy*fy))

and the product masked by the band-limit functions Rect((fx - cx)/wx) and
Rect((fy - cy)/wy). The padding, frequency grid, normalisation and crop are those
of the plain method (``oracle.diffraction``).

Readings of points the paper leaves open:

* Eq. shift_ang2 prints the exponent without the imaginary unit; a linear phase
  exp(+i*2*pi*(Ox*fx + Oy*fy)) is taken. It moves the destination window: output
  sample (m, n) lies at (m*dx + Ox, n*dy + Oy) of the unshifted geometry.
* The Rect arguments are taken in frequency units (cx, wx in cycles per metre);
  the paper's index form is the same with c and w divided by the frequency pitch.
* Rect(t) = 1 for |t| <= 1/2 and 0 otherwise; a width w <= 0 means no limit on
  that axis.
* The band-limit parameters are inputs: the paper defers their choice to its
  reference. For the on-axis case (O = 0) ``band_limit`` returns the limit of the
  band-limited angular spectrum method (Matsushima and Shimobaba, Opt. Express 17,
  19662 (2009)): the transfer function's phase is sampled finely enough where
  |fx| <= 1 / (lambda * sqrt((2*dfx*z)^2 + 1)), dfx = 1/(Mx*dx).
"""
from __future__ import annotations

import math

import numpy as np

from . import diffraction as D


def rect(t: np.ndarray) -> np.ndarray:
    """1 where |t| <= 1/2, else 0."""
    return (np.abs(t) <= 0.5).astype(np.float64)


def axis_mask(f: np.ndarray, c: float, w: float) -> np.ndarray:
    """Rect((f - c)/w) along one axis; w <= 0 leaves the axis unlimited."""
    if not (w > 0.0):
        return np.ones_like(f)
    return rect((f - c) / w)


def linear_phase(f: np.ndarray, offset: float) -> np.ndarray:
    """exp(i*2*pi*offset*f), the phase in revolutions reduced in FP64 before the
    sine and cosine."""
    t = offset * f
    r = t - np.rint(t)
    return np.cos(2.0 * math.pi * r) + 1j * np.sin(2.0 * math.pi * r)


def transfer(my: int, mx: int, dy: float, dx: float, lam: float, z: float,
             ox: float = 0.0, oy: float = 0.0, cx: float = 0.0, wx: float = 0.0,
             cy: float = 0.0, wy: float = 0.0) -> np.ndarray:
    """H_SA times the two band-limit functions on the [My][Mx] padded grid."""
    fx = D.frequencies(mx, dx)
    fy = D.frequencies(my, dy)
    h = D.asm_transfer(my, mx, dy, dx, lam, z)
    shift = linear_phase(fy, oy)[:, None] * linear_phase(fx, ox)[None, :]
    mask = axis_mask(fy, cy, wy)[:, None] * axis_mask(fx, cx, wx)[None, :]
    return h * shift * mask


def propagate(u1: np.ndarray, dx: float, dy: float | None = None, wavelength: float = 633e-9,
              z: float = 0.1, ox: float = 0.0, oy: float = 0.0, cx: float = 0.0,
              wx: float = 0.0, cy: float = 0.0, wy: float = 0.0, nopad: bool = False,
              method: str = "auto") -> np.ndarray:
    """u2 = crop(IDFT(DFT(pad(u1)) * H_SA * Rect * Rect)) (Eq. shift_ang1)."""
    dy = dx if dy is None else dy
    u1 = np.asarray(u1)
    D.validate(u1, dx, dy, wavelength, z, D.ASM)
    for v, name in ((ox, "ox"), (oy, "oy"), (cx, "cx"), (cy, "cy"), (wx, "wx"), (wy, "wy")):
        if not math.isfinite(v):
            raise ValueError("%s must be finite" % name)
    ny, nx = u1.shape
    my, mx = D.padded_size(ny, nopad), D.padded_size(nx, nopad)
    a = D.pad(u1.astype(np.complex128), my, mx)
    spectrum = D.dft2(a, False, method)
    h = transfer(my, mx, dy, dx, wavelength, z, ox, oy, cx, wx, cy, wy)
    b = D.dft2(spectrum * h, True, method) / float(mx * my)
    return b[:ny, :nx].copy()


def band_limit(n: int, d: float, wavelength: float, z: float, nopad: bool = False) -> float:
    """Full width 2*f_limit of the on-axis band limit along an axis of N samples."""
    m = D.padded_size(n, nopad)
    df = 1.0 / (m * d)
    return 2.0 / (wavelength * math.sqrt((2.0 * df * z) ** 2 + 1.0))

"""Oracle: field epilogues of the paper's examples (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this module; it shares nothing with the product library.

* Intensity (Sec. 3.1, Eq. of the intensity field): I = |u|^2.
* Scale (Sec. 3.1, Eq. norm): I_top = (I - min I)/(max I - min I) * top, the paper's
  256-step image for top = 255.
* Phase (Sec. 7.1, kinoform): the argument of u, atan2(Im u, Re u).
* Complex (Sec. 7.1): a phase field back to a complex field, A exp(i phi) (A = 1 for a
  kinoform).

Readings:

* The epilogues run on complex64 fields in FP32: I = re*re + im*im, and Eq. norm
  evaluated in the order it is written, (I - min), then / (max - min), then * top, each
  operation rounded to nearest in FP32; the 8-bit image is that value rounded to the
  nearest integer (ties to even) and clamped to [0, 255]. These FP32 definitions decide
  the 8-bit codes, so the GPU is compared with them bit for bit.
* A constant field (max == min) scales to 0.
* The phase lies in [-pi, pi]; the sign of a zero imaginary part picks the end.
"""
from __future__ import annotations

import numpy as np


def intensity(u: np.ndarray) -> np.ndarray:
    """|u|^2 of a complex64 field in FP32 (two products, one sum, each rounded)."""
    u = np.asarray(u, dtype=np.complex64)
    re = u.real.astype(np.float32)
    im = u.imag.astype(np.float32)
    return (re * re + im * im).astype(np.float32)


def scale(i: np.ndarray, top: float = 255.0) -> np.ndarray:
    """Eq. norm, (I - min)/(max - min) * top, in FP32 in the printed order: the
    difference, the quotient by the range, the product with top, each rounded to
    nearest (0 where max == min)."""
    i = np.asarray(i, dtype=np.float32)
    mn = np.float32(i.min())
    mx = np.float32(i.max())
    if mx == mn:
        return np.zeros_like(i)
    rng = np.float32(mx - mn)
    return (((i - mn) / rng) * np.float32(top)).astype(np.float32)


def scale_u8(i: np.ndarray, top: float = 255.0) -> np.ndarray:
    """The 8-bit image: the FP32 scale rounded to nearest (ties to even), clamped."""
    return np.clip(np.rint(scale(i, top)), 0, 255).astype(np.uint8)


def phase(u: np.ndarray) -> np.ndarray:
    """atan2(Im u, Re u) in FP64 of the complex64 components."""
    u = np.asarray(u, dtype=np.complex64)
    return np.arctan2(u.imag.astype(np.float64), u.real.astype(np.float64))


def polar(phi: np.ndarray, amp: np.ndarray | None = None) -> np.ndarray:
    """A exp(i phi) in FP64 (A = 1 when amp is None)."""
    phi = np.asarray(phi, dtype=np.float64)
    a = 1.0 if amp is None else np.asarray(amp, dtype=np.float64)
    return a * (np.cos(phi) + 1j * np.sin(phi))

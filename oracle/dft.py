"""Oracle: direct discrete Fourier transform in FP64 (test infrastructure only).

The DFT written out as a matrix product, for small sizes and for pinning the
textbook FFT in ``fft64.c``:

    X[k] = sum_j x[j] * exp(-2*pi*i * j*k / M)          (forward)
    x[j] = sum_k X[k] * exp(+2*pi*i * j*k / M)          (inverse, unnormalised)

Each entry of the DFT matrix is evaluated from the integer product reduced
first, ``(j*k mod M) / M``; for power-of-two M that quotient is exact in FP64,
so every twiddle is one correctly rounded ``exp`` of an exact argument times
``2*pi``. The 2-D DFT is ``F_y @ a @ F_x`` (both DFT matrices are symmetric).
"""
from __future__ import annotations

import numpy as np

_TWO_PI = 2.0 * np.pi


def dft_matrix(m: int, inverse: bool = False) -> np.ndarray:
    """The m x m DFT matrix with entries exp(-+2*pi*i*((j*k) mod m)/m)."""
    j = np.arange(m, dtype=np.int64)
    jk = np.outer(j, j) % m
    ang = _TWO_PI * (jk.astype(np.float64) / float(m))
    sign = 1.0 if inverse else -1.0
    return np.cos(ang) + 1j * (sign * np.sin(ang))


def dft1_direct(x: np.ndarray, inverse: bool = False) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128).reshape(-1)
    return dft_matrix(x.size, inverse) @ x


def dft2_direct(a: np.ndarray, inverse: bool = False) -> np.ndarray:
    """Unnormalised 2-D DFT of a [ny][nx] array by two DFT-matrix products."""
    a = np.asarray(a, dtype=np.complex128)
    fy = dft_matrix(a.shape[0], inverse)
    fx = dft_matrix(a.shape[1], inverse)
    return fy @ a @ fx

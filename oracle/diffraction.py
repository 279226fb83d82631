"""Oracle: scalar diffraction by FFT convolution, FP64 (test infrastructure only).

This module is the reference the HIP path is checked against. Only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
it. It shares no code with the product library (no kernels, headers, tables or
constants), and it never imports the product package.

It follows the paper's definitions, in the paper's order and notation:

* Fresnel diffraction, convolution form (Sec. 2.1.1, Eqs. fre_conv, fresnel_conv,
  fre_conv_fft, fre_conv_prop_d): the field is convolved with the sampled
  impulse response h_F(m, n) = exp(i*pi/(lambda*z) * ((m*dx)^2 + (n*dy)^2)),
  evaluated as IFFT[FFT[u] * FFT[h_F]] and scaled by exp(i*k*z)/(i*lambda*z).
  Three transforms (Table of diffraction classes: 3 FFTs, 2N x 2N).
* Angular spectrum method (Sec. 2.1.4, Eqs. ang1-ang3): u2 = IFFT[FFT[u1] * H_A],
  H_A(fx, fy) = exp(i*z*sqrt(k^2 - 4*pi^2*(fx^2 + fy^2))), k = 2*pi/lambda.
  Two transforms.
* Both convolution forms expand the N x N planes to 2N x 2N with zeros and
  extract the N x N result afterwards (Sec. 2.1.6), so the circular
  convolution does not alias.

Readings of points the paper leaves open:

* The field sits at the top-left of the padded grid and the result is cropped
  from the top-left (a circular shift commutes with the circular convolution,
  so any consistent placement gives the same crop).
* The frequency pitch is df = 1/(M*d) of the padded grid; bin p maps to p*df for
  p < M/2 and to (p - M)*df otherwise.
* The inverse transform carries the 1/(Mx*My) normalisation.
* The ASM radicand is written k^2 * (1 - lambda^2*(fx^2 + fy^2)); the bin is
  propagating when s = (lambda*fx)^2 + (lambda*fy)^2 <= 1 (s == 1 counts as
  propagating, H = 1) and evanescent bins get H = 0.
* The Fresnel sum includes the quadrature factor dx*dy of the continuous
  integral (Eq. fre_conv), which the discrete Eq. fre_conv_fft leaves out.
* The impulse response is sampled on the padded grid at signed offsets
  s(d) = d for d < N and d - M for d >= N.
* z = 0 is the identity for ASM and invalid for Fresnel; z < 0 propagates back.
"""
from __future__ import annotations

import math

import numpy as np

from . import _native
from .dft import dft2_direct

ASM = "asm"
FRESNEL = "fresnel"

# sizes at or below this use the direct DFT; larger ones the textbook FFT
_DIRECT_MAX = 256


def dft2(a: np.ndarray, inverse: bool = False, method: str = "auto") -> np.ndarray:
    """Unnormalised 2-D DFT: direct matrix form for small arrays, else the FP64 FFT."""
    if method == "direct" or (method == "auto" and max(a.shape) <= _DIRECT_MAX):
        return dft2_direct(a, inverse)
    return _native.fft2(a, inverse)


# ---- step 1: pad (Sec. 2.1.6) -------------------------------------------------

def pad(u1: np.ndarray, my: int, mx: int) -> np.ndarray:
    """Place the Ny x Nx field at the top-left of an My x Mx array of zeros."""
    ny, nx = u1.shape
    a = np.zeros((my, mx), dtype=np.complex128)
    a[:ny, :nx] = u1
    return a


# ---- step 3: frequencies of the padded grid ----------------------------------

def frequencies(m: int, d: float) -> np.ndarray:
    """Spatial frequency of each DFT bin as index times pitch (Sec. 2.1.4: f = m1 * df):
    df = 1/(M*d) and the signed index is p for p < M/2, else p - M."""
    p = np.arange(m, dtype=np.float64)
    signed = np.where(p < m / 2, p, p - m)
    df = 1.0 / (m * d)
    return signed * df


# ---- step 4a: angular-spectrum transfer function (Eq. ang2) -------------------

def asm_radicand_fraction(my: int, mx: int, dy: float, dx: float, lam: float) -> np.ndarray:
    """s = (lambda*fx)^2 + (lambda*fy)^2 on the [My][Mx] grid, evaluated in FP64 as
    ax = lam*fx, s = ax*ax + ay*ay (the propagating test is s <= 1)."""
    ax = lam * frequencies(mx, dx)
    ay = lam * frequencies(my, dy)
    return (ay * ay)[:, None] + (ax * ax)[None, :]


def asm_transfer(my: int, mx: int, dy: float, dx: float, lam: float, z: float) -> np.ndarray:
    """H_A = exp(i*z*sqrt(k^2 - 4 pi^2 (fx^2+fy^2))) = exp(i*z*k*sqrt(1 - s)); 0 if s > 1."""
    k = 2.0 * math.pi / lam
    s = asm_radicand_fraction(my, mx, dy, dx, lam)
    prop = s <= 1.0
    phase = z * k * np.sqrt(np.where(prop, 1.0 - s, 0.0))
    h = np.cos(phase) + 1j * np.sin(phase)
    return np.where(prop, h, 0.0 + 0.0j)


# ---- step 4b: Fresnel impulse response and its transform (Eqs. fre_conv_prop_d) --

def signed_offsets(m: int, n: int) -> np.ndarray:
    """Offset of each padded-grid index: d for d < N, d - M for d >= N."""
    d = np.arange(m, dtype=np.float64)
    return np.where(d < n, d, d - m)


def fresnel_impulse(my: int, mx: int, ny: int, nx: int, dy: float, dx: float,
                    lam: float, z: float) -> np.ndarray:
    """h_F(m, n) = exp(i*pi/(lambda*z) * ((m*dx)^2 + (n*dy)^2)) on the padded grid."""
    x = signed_offsets(mx, nx) * dx
    y = signed_offsets(my, ny) * dy
    arg = (math.pi / (lam * z)) * ((y * y)[:, None] + (x * x)[None, :])
    return np.cos(arg) + 1j * np.sin(arg)


def fresnel_constant(dy: float, dx: float, lam: float, z: float) -> complex:
    """dx*dy * exp(i*k*z) / (i*lambda*z)  (Eq. fre_conv with its quadrature factor)."""
    k = 2.0 * math.pi / lam
    kz = k * z
    return dx * dy * complex(math.cos(kz), math.sin(kz)) / (1j * lam * z)


def fresnel_transfer_analytic(my: int, mx: int, dy: float, dx: float, lam: float,
                              z: float) -> np.ndarray:
    """Fourier transform of Eq. fre_conv's kernel: exp(i*k*z) * exp(-i*pi*lambda*z*(fx^2+fy^2))."""
    k = 2.0 * math.pi / lam
    fx = frequencies(mx, dx)
    fy = frequencies(my, dy)
    arg = -math.pi * lam * z * ((fy * fy)[:, None] + (fx * fx)[None, :])
    return complex(math.cos(k * z), math.sin(k * z)) * (np.cos(arg) + 1j * np.sin(arg))


# ---- the whole pipeline -------------------------------------------------------

def padded_size(n: int, nopad: bool) -> int:
    return n if nopad else 2 * n


def validate(u1: np.ndarray, dx: float, dy: float, lam: float, z: float, kind: str) -> None:
    if u1.ndim != 2:
        raise ValueError("field must be 2-D [ny][nx]")
    for v, name in ((dx, "dx"), (dy, "dy"), (lam, "wavelength")):
        if not (math.isfinite(v) and v > 0):
            raise ValueError("%s must be finite and > 0" % name)
    if not math.isfinite(z):
        raise ValueError("z must be finite")
    if kind == FRESNEL and z == 0.0:
        raise ValueError("Fresnel diffraction is singular at z = 0")


def transfer_function(kind: str, my: int, mx: int, ny: int, nx: int, dy: float, dx: float,
                      lam: float, z: float, fresnel_tf: str = "sampled",
                      method: str = "auto") -> np.ndarray:
    """The array the spectrum is multiplied with (step 4 of the pipeline)."""
    if kind == ASM:
        return asm_transfer(my, mx, dy, dx, lam, z)
    if kind == FRESNEL:
        if fresnel_tf == "analytic":
            return fresnel_transfer_analytic(my, mx, dy, dx, lam, z)
        h = fresnel_impulse(my, mx, ny, nx, dy, dx, lam, z)
        return fresnel_constant(dy, dx, lam, z) * dft2(h, False, method)   # FFT[h_F], 3rd transform
    raise ValueError("unknown kind %r" % (kind,))


def propagate(u1: np.ndarray, kind: str, dx: float, dy: float | None = None,
              wavelength: float = 633e-9, z: float = 0.1, nopad: bool = False,
              fresnel_tf: str = "sampled", method: str = "auto") -> np.ndarray:
    """u2 = crop(IDFT(DFT(pad(u1)) * H)) with the 1/(Mx*My) inverse normalisation.

    ``u1`` is upcast to complex128 exactly; the result is complex128 [Ny][Nx].
    ``nopad`` keeps M = N (circular convolution; used only for exactness pins).
    """
    dy = dx if dy is None else dy
    u1 = np.asarray(u1)
    validate(u1, dx, dy, wavelength, z, kind)
    ny, nx = u1.shape
    my, mx = padded_size(ny, nopad), padded_size(nx, nopad)
    a = pad(u1.astype(np.complex128), my, mx)                          # step 1
    spectrum = dft2(a, False, method)                                  # step 2
    h = transfer_function(kind, my, mx, ny, nx, dy, dx, wavelength, z, fresnel_tf, method)  # 3-4
    b = dft2(spectrum * h, True, method) / float(mx * my)              # steps 5-6
    return b[:ny, :nx].copy()                                          # step 7


def asm(u1, dx, dy=None, wavelength=633e-9, z=0.1, **kw):
    return propagate(u1, ASM, dx, dy, wavelength, z, **kw)


def fresnel(u1, dx, dy=None, wavelength=633e-9, z=0.1, **kw):
    return propagate(u1, FRESNEL, dx, dy, wavelength, z, **kw)


def rel_l2(y: np.ndarray, ref: np.ndarray) -> float:
    """||y - ref||_2 / ||ref||_2 (0 when both are zero)."""
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    den = float(np.linalg.norm(ref.ravel()))
    num = float(np.linalg.norm((y - ref).ravel()))
    if den == 0.0:
        return 0.0 if num == 0.0 else math.inf
    return num / den

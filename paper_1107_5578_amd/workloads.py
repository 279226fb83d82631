"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no diffraction arithmetic: it only draws fields and
parameters. The same arrays feed the HIP path and the FP64 oracle, so both see
identical complex64 bytes.

The paper's inputs (an N x N photograph padded to 2N x 2N for N = 512...2048,
a recorded hologram, a GS target image) are not available; timing does not
depend on content, so these fields take the paper's shapes and sizes:

* ``uniform_random_field``  amplitude U[0,1), phase U[0, 2*pi)   (plain ASM, 256^2)
* ``rectangles_field``      0/1 image of 64 axis-aligned rectangles with sides
                            U{32..512} px placed uniformly, per-pixel phase U[0, 2*pi)
* ``speckle_field``         circular Gaussian speckle (g1 + i*g2)/sqrt(2)
* ``zstack_distances``      64 distances uniform on [0.05, 0.2] m
* ``serving_requests``      a Poisson-arrival request mix of sizes, kinds,
                            distances and wavelengths

Random numbers come from numpy's PCG64 ``default_rng(seed)``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

LAMBDA_DEFAULT = 633e-9   # default wavelength of the paper's library
PITCH_DEFAULT = 10e-6     # default sampling pitch of the paper's library


def _complex64(amp: np.ndarray, phase: np.ndarray) -> np.ndarray:
    u = amp.astype(np.float64) * np.exp(1j * phase.astype(np.float64))
    return u.astype(np.complex64)


def uniform_random_field(n: int, seed: int, ny: int | None = None) -> np.ndarray:
    """Amplitude U[0,1), phase U[0, 2*pi), complex64 [ny][n]."""
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    amp = rng.random((ny, n))
    phase = 2.0 * math.pi * rng.random((ny, n))
    return _complex64(amp, phase)


def rectangles_amplitude(n: int, seed: int, count: int = 64, side_lo: int = 32,
                         side_hi: int = 512) -> np.ndarray:
    """0/1 float32 image: union of ``count`` axis-aligned rectangles, integer sides
    uniform in [side_lo, side_hi] (clipped to n), placed uniformly inside n x n."""
    rng = np.random.default_rng(seed)
    img = np.zeros((n, n), dtype=np.float32)
    lo = min(side_lo, n)
    hi = min(side_hi, n)
    for _ in range(count):
        w = int(rng.integers(lo, hi + 1))
        h = int(rng.integers(lo, hi + 1))
        x0 = int(rng.integers(0, n - w + 1))
        y0 = int(rng.integers(0, n - h + 1))
        img[y0:y0 + h, x0:x0 + w] = 1.0
    return img


def rectangles_field(n: int, seed: int) -> np.ndarray:
    """Rectangles amplitude with a per-pixel random phase U[0, 2*pi), complex64."""
    amp = rectangles_amplitude(n, seed)
    rng = np.random.default_rng(seed + 1_000_003)
    phase = 2.0 * math.pi * rng.random((n, n))
    return _complex64(amp, phase)


def speckle_field(n: int, seed: int) -> np.ndarray:
    """(g1 + i*g2)/sqrt(2), g i.i.d. N(0,1), complex64 [n][n]."""
    rng = np.random.default_rng(seed)
    g1 = rng.standard_normal((n, n))
    g2 = rng.standard_normal((n, n))
    return ((g1 + 1j * g2) / math.sqrt(2.0)).astype(np.complex64)


def random_phase(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return 2.0 * math.pi * rng.random((n, n))


def zstack_distances(count: int = 64, z0: float = 0.05, z1: float = 0.2) -> np.ndarray:
    """count distances uniform on [z0, z1]: z_j = z0 + j*(z1 - z0)/(count - 1)."""
    if count == 1:
        return np.array([z0])
    j = np.arange(count, dtype=np.float64)
    return z0 + j * ((z1 - z0) / (count - 1))


# ---- the named configurations ----------------------------------------------

@dataclasses.dataclass(frozen=True)
class PlaneConfig:
    name: str
    n: int
    pitch: float
    wavelength: float
    z: float
    seed: int


PLAIN_ASM_256 = PlaneConfig("asm-256", 256, 10e-6, 633e-9, 0.1, 1)
PLANE_2048 = PlaneConfig("plane-2048", 2048, 8e-6, 532e-9, 0.5, 2)
ZSTACK_1024 = PlaneConfig("zstack-1024x64", 1024, 4e-6, 633e-9, 0.05, 3)
GS_2048 = PlaneConfig("gs-2048", 2048, 8e-6, 532e-9, 0.1, 41)


def field_for(cfg: PlaneConfig, n: int | None = None) -> np.ndarray:
    """The synthetic field of a named configuration (optionally at another size)."""
    n = cfg.n if n is None else n
    if cfg.name.startswith("asm-256"):
        return uniform_random_field(n, cfg.seed)
    if cfg.name.startswith("plane-2048"):
        return rectangles_field(n, cfg.seed)
    if cfg.name.startswith("zstack"):
        return speckle_field(n, cfg.seed)
    raise ValueError(cfg.name)


def gs_problem(n: int = 2048, seeds=(41, 42, 43)):
    """Two rectangle amplitude targets and the start field A1*exp(i*phi0)."""
    a1 = rectangles_amplitude(n, seeds[0])
    a2 = rectangles_amplitude(n, seeds[1])
    phi0 = random_phase(n, seeds[2])
    u0 = _complex64(a1, phi0)
    return a1, a2, u0


# ---- point-light-source object ----------------------------------------------

@dataclasses.dataclass(frozen=True)
class PlsConfig:
    """A hologram of n x n pixels of pitch `pitch` from a point object offset by
    (ox, oy, oz); point counts as in the paper's hologram timings."""
    n: int = 2048
    pitch: float = 4e-6
    wavelength: float = 633e-9
    ox: float = 2500 * 4e-6
    oy: float = -512 * 4e-6
    oz: float = 0.2
    counts: tuple = (248, 4596, 11646)


PLS_2048 = PlsConfig()


def pls_points(count: int, seed: int, half_extent: float = 4e-3) -> np.ndarray:
    """Synthetic stand-in for a scanned 3-D object: `count` points uniform in a cube of
    half-width `half_extent` (the object's coordinates normalised to +-4 mm, as the paper
    scales its model), amplitudes uniform on [0.5, 1]; float32 [count][4] (X, Y, Z, A)."""
    rng = np.random.default_rng(seed)
    pts = np.empty((count, 4), dtype=np.float32)
    pts[:, :3] = rng.uniform(-half_extent, half_extent, (count, 3))
    pts[:, 3] = rng.uniform(0.5, 1.0, count)
    return pts


# ---- serving request stream --------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Request:
    index: int
    arrival_s: float
    n: int
    kind: str           # "asm" or "fresnel"
    z: float
    wavelength: float
    pitch: float
    seed: int


def serving_requests(count: int, rate_per_s: float, seed: int = 5,
                     sizes=(512, 1024, 2048, 4096), pitch: float = 8e-6):
    """Poisson arrivals at ``rate_per_s``; size uniform over ``sizes``; kind ASM/Fresnel
    50/50; z ~ U[0.01, 1] m; wavelength uniform over {473, 532, 633} nm. Request i's
    field content is ``uniform_random_field(n, 5000 + i)``."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    lams = (473e-9, 532e-9, 633e-9)
    for i in range(count):
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        kind = "asm" if rng.random() < 0.5 else "fresnel"
        z = float(rng.uniform(0.01, 1.0))
        lam = float(lams[int(rng.integers(0, 3))])
        out.append(Request(i, float(t[i]), n, kind, z, lam, pitch, 5000 + i))
    return out

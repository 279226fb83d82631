"""Oracle: amplitude-constrained ping-pong iteration (test infrastructure only).

The Gerchberg-Saxton style loop of the paper's GS application (Sec. 7.2,
"GS algorithm"): the field is propagated by the angular spectrum method to a
plane at distance z, an amplitude constraint is imposed there, the field is
propagated back by -z, and a constraint is imposed at the start plane.

Reading used here (the Fresnel ping-pong variant with two amplitude targets;
the paper's kinoform loop is the special case A1 == 1):

    v_k     = ASM_{+z}(u_k)
    E_k     = || |v_k| - A2 ||_2 / || A2 ||_2          (error before the constraint)
    v_k'    = A2 * v_k / |v_k|        (A2 where |v_k| == 0: phase 0)
    w_k     = ASM_{-z}(v_k')
    u_{k+1} = A1 * w_k / |w_k|        (A1 where |w_k| == 0)

The phase of a field is its argument (atan2 of imaginary and real part), so
A*u/|u| keeps the phase and replaces the amplitude.
"""
from __future__ import annotations

import numpy as np

from .diffraction import asm


def amplitude_constraint(u: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Replace |u| by a, keeping the phase; where u == 0 the result is a (phase 0)."""
    u = np.asarray(u, dtype=np.complex128)
    a = np.asarray(a, dtype=np.float64)
    mag = np.abs(u)
    safe = np.where(mag > 0, mag, 1.0)
    return np.where(mag > 0, a * (u / safe), a + 0j)


def error(v: np.ndarray, a: np.ndarray) -> float:
    a = np.asarray(a, dtype=np.float64)
    return float(np.linalg.norm((np.abs(v) - a).ravel()) / np.linalg.norm(a.ravel()))


def iteration(u: np.ndarray, a1: np.ndarray, a2: np.ndarray, dx: float, wavelength: float,
              z: float, dy: float | None = None):
    """One ping-pong step from u_k; returns (u_{k+1}, E_k)."""
    v = asm(u, dx, dy, wavelength, z)
    e = error(v, a2)
    w = asm(amplitude_constraint(v, a2), dx, dy, wavelength, -z)
    return amplitude_constraint(w, a1), e

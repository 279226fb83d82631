"""Pins of the epilogue oracle (Sec. 3.1 Intensity/Scale, Sec. 7.1 Phase/Complex):
hand-computed values, the paper's 0..255 range, rounding ties, degenerate fields,
quadrants and signed zeros of the phase, and the phase/complex round trip."""
import math

import numpy as np

from oracle import epilogues as P


def test_intensity_values():
    u = np.array([3 + 4j, -1j, 0, 0.1 + 0j, 2.5 - 1.5j], dtype=np.complex64)
    got = P.intensity(u)
    assert got.dtype == np.float32
    assert list(got[:3]) == [25.0, 1.0, 0.0]
    assert got[3] == np.float32(np.float32(0.1) * np.float32(0.1))  # one FP32 rounding
    assert got[4] == np.float32(8.5)


def test_scale_maps_min_to_0_and_max_to_top():
    i = np.array([2.0, 4.0, 6.0, 3.0], dtype=np.float32)
    s = P.scale(i)
    assert s[0] == 0.0 and s[2] == 255.0
    assert s[1] == np.float32(127.5)
    assert s[3] == np.float32(63.75)
    assert list(P.scale_u8(i)) == [0, 128, 255, 64]  # 127.5 ties to even 128, 63.75 -> 64


def test_scale_degenerate_and_top():
    c = np.full(7, 3.25, dtype=np.float32)
    assert not P.scale(c).any()
    assert not P.scale_u8(c).any()
    i = np.array([0, 1, 2], dtype=np.float32)
    assert list(P.scale(i, 1.0)) == [0.0, 0.5, 1.0]


def test_phase_quadrants_and_signed_zero():
    u = np.array([1 + 0j, 1j, -1 + 0j, -1j, 1 + 1j, complex(-1, -0.0)], dtype=np.complex64)
    ph = P.phase(u)
    assert np.allclose(ph[:5], [0, math.pi / 2, math.pi, -math.pi / 2, math.pi / 4], atol=0, rtol=1e-15)
    assert ph[5] == -math.pi


def test_polar_round_trip():
    rng = np.random.default_rng(5)
    phi = rng.uniform(-math.pi, math.pi, 1000)
    a = rng.uniform(0.1, 3, 1000)
    u = P.polar(phi, a)
    assert np.allclose(np.abs(u), a, rtol=1e-14)
    assert np.allclose(np.angle(u), phi, atol=1e-14)
    assert np.allclose(P.polar(phi), np.exp(1j * phi), atol=1e-15)

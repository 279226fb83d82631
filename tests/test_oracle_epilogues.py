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


def _round32(q):
    """Nearest float32 to the exact rational q, ties to even (independent of numpy's
    float32 arithmetic: neighbours compared in exact rational arithmetic)."""
    from fractions import Fraction

    c = np.float32(float(q))
    best = None
    for cand in (np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))):
        d = abs(Fraction(float(cand)) - q)
        if best is None or d < best[0] or (d == best[0] and (cand.view(np.uint32) & 1) == 0):
            best = (d, cand)
    return best[1]


def _scale_exact_order(i, mn, mx, top):
    """Eq. norm with each operation of its printed order rounded once to FP32."""
    from fractions import Fraction

    F = Fraction
    d = _round32(F(float(i)) - F(float(mn)))
    r = _round32(F(float(mx)) - F(float(mn)))
    q = _round32(F(float(d)) / F(float(r)))
    return _round32(F(float(q)) * F(float(top)))


def test_scale_follows_the_printed_order_where_orders_round_apart():
    # (I - min)/(max - min) * 255 lands just above 226.5 in the printed order and exactly
    # on 226.5 with the factor 255/(max - min) formed first: the two orders give 8-bit
    # codes 227 and 226, so this case tells them apart.
    mn, i, mx = np.float32(0.7443469762802124), np.float32(1.8845739364624023), np.float32(2.028046131134033)
    arr = np.array([mn, i, mx], dtype=np.float32)
    want = _scale_exact_order(i, mn, mx, np.float32(255))
    got = P.scale(arr)
    assert got[1] == want
    other = np.float32(np.float32(i - mn) * np.float32(np.float32(255) / np.float32(mx - mn)))
    assert other != want and np.rint(other) != np.rint(want)
    assert P.scale_u8(arr)[1] == 227
    assert got[0] == 0.0 and got[2] == 255.0


def test_scale_matches_per_operation_rounding_on_random_values():
    rng = np.random.default_rng(11)
    arr = rng.uniform(0.3, 7.0, 200).astype(np.float32)
    mn, mx = arr.min(), arr.max()
    got = P.scale(arr, 200.0)
    for k in range(0, 200, 7):
        assert got[k] == _scale_exact_order(arr[k], mn, mx, np.float32(200.0))

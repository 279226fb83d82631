"""Pins of the FP64 oracle against what the mathematics and the physics fix.

Nothing here compares the oracle with itself: each test checks it against a
closed form, an invariant, a brute-force sum written independently below, or an
independent library routine (numpy's pocketfft). A plausible slip in the oracle
(a dropped factor, a wrong sign, a transposed axis, a wrong frequency pitch, a
missing normalisation, the wrong crop) fails at least one of them.
"""
import math

import numpy as np
import pytest

from oracle import _native, diffraction as D, dft, gs

RNG = np.random.default_rng(12345)


def crandn(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


# ---- the DFT itself ----------------------------------------------------------

def test_direct_dft_closed_forms():
    # a delta at j0 transforms to exp(-2 pi i j0 k / M); a constant to M*delta;
    # forward then inverse is M times the identity
    m = 64
    for j0 in (0, 1, 7, 33):
        x = np.zeros(m, complex)
        x[j0] = 1.0
        k = np.arange(m)
        expect = np.exp(-2j * np.pi * ((j0 * k) % m) / m)
        assert np.max(np.abs(dft.dft1_direct(x) - expect)) < 1e-15
    ones = np.ones(m, complex)
    d = dft.dft1_direct(ones)
    assert abs(d[0] - m) < 1e-12 and np.max(np.abs(d[1:])) < 1e-12
    x = crandn(m)
    back = dft.dft1_direct(dft.dft1_direct(x), inverse=True) / m
    assert rel(back, x) < 1e-14


def test_direct_dft_matches_pocketfft():
    for m in (8, 16, 32, 128):
        x = crandn(m)
        assert rel(dft.dft1_direct(x), np.fft.fft(x)) < 1e-13
    a = crandn(16, 32)
    assert rel(dft.dft2_direct(a), np.fft.fft2(a)) < 1e-13
    assert rel(dft.dft2_direct(a, True), np.fft.ifft2(a) * a.size) < 1e-13


@pytest.mark.parametrize("m", [8, 16, 32, 64, 128, 256, 512])
def test_textbook_fft_vs_direct_dft(m):
    x = crandn(m)
    assert rel(_native.fft1(x), dft.dft1_direct(x)) < 1e-13
    assert rel(_native.fft1(x, True), dft.dft1_direct(x, True)) < 1e-13


def test_textbook_fft2_vs_direct_and_pocketfft():
    a = crandn(32, 64)
    assert rel(_native.fft2(a), dft.dft2_direct(a)) < 1e-13
    assert rel(_native.fft2(a, True), dft.dft2_direct(a, True)) < 1e-13
    b = crandn(256, 128)
    assert rel(_native.fft2(b), np.fft.fft2(b)) < 1e-13
    assert rel(_native.fft2(b, True), np.fft.ifft2(b) * b.size) < 1e-13


def test_textbook_fft_parseval_and_thread_independence():
    a = crandn(128, 64)
    A = _native.fft2(a)
    assert abs(np.sum(np.abs(a) ** 2) - np.sum(np.abs(A) ** 2) / a.size) / np.sum(np.abs(a) ** 2) < 1e-13
    assert np.array_equal(_native.fft2(a, threads=1), _native.fft2(a, threads=4))


def test_twiddle_table_exact_angles():
    m = 1024
    assert _native.twiddle(0, m) == complex(1.0, -0.0) or _native.twiddle(0, m) == 1.0
    w = _native.twiddle(m // 4, m)
    assert abs(w.real) < 1e-17 and w.imag == -1.0
    w = _native.twiddle(m // 2, m)
    assert w.real == -1.0 and abs(w.imag) < 1e-17
    w = _native.twiddle(m // 8, m)
    h = math.sqrt(0.5)
    assert abs(w.real - h) < 2e-16 and abs(w.imag + h) < 2e-16
    # every entry is within one FP64 ulp of exp(-2 pi i k/m) evaluated in x87 extended precision
    pi_ld = np.longdouble("3.14159265358979323846264338327950288")
    for k in range(m):
        ang = np.longdouble(2) * pi_ld * np.longdouble(k) / np.longdouble(m)
        w = _native.twiddle(k, m)
        assert abs(np.longdouble(w.real) - np.cos(ang)) < 1.2e-16
        assert abs(np.longdouble(w.imag) + np.sin(ang)) < 1.2e-16


# ---- frequencies, padding -------------------------------------------------

def test_frequency_grid():
    f = D.frequencies(8, 0.5)
    assert np.array_equal(f, np.array([0, 1, 2, 3, -4, -3, -2, -1]) / 4.0)


# ---- angular spectrum method --------------------------------------------------

@pytest.mark.parametrize("p0,q0", [(0, 0), (3, 0), (0, 5), (7, -4), (-12, 9)])
def test_asm_plane_wave_nopad(p0, q0):
    # a plane wave on the periodic grid is an eigenfunction: it picks up exactly
    # exp(i z sqrt(k^2 - 4 pi^2 (fx^2 + fy^2))) with fx = p0/(N dx), fy = q0/(N dy)
    n, dx, dy, lam, z = 32, 10e-6, 8e-6, 633e-9, 0.137
    jy, jx = np.mgrid[0:n, 0:n]
    u = np.exp(2j * np.pi * (p0 * jx / n + q0 * jy / n))
    out = D.asm(u, dx, dy, lam, z, nopad=True)
    k = 2 * np.pi / lam
    fx, fy = p0 / (n * dx), q0 / (n * dy)
    kappa = math.sqrt(k * k - 4 * np.pi ** 2 * (fx * fx + fy * fy))
    expect = u * np.exp(1j * z * kappa)
    # the phase z*kappa is ~1.4e6 rad: FP64 represents it to ~|phase|*2^-52, so the
    # bound is a few ulps of the phase on top of the transform's own rounding
    tol = 1e-12 + 8 * np.finfo(float).eps * k * abs(z)
    assert rel(out, expect) < tol
    if p0 == 0 and q0 == 0:
        assert rel(out, u * np.exp(1j * k * z)) < tol


def test_asm_z0_is_identity_padded():
    u = crandn(24 * 2, 40 * 2)[:32, :64]
    out = D.asm(u, 10e-6, 10e-6, 633e-9, 0.0)
    assert rel(out, u) < 1e-14


def test_asm_round_trip_nopad():
    u = crandn(64, 32)
    fwd = D.asm(u, 10e-6, 12e-6, 633e-9, 0.21, nopad=True)
    back = D.asm(fwd, 10e-6, 12e-6, 633e-9, -0.21, nopad=True)
    assert rel(back, u) < 1e-12


def test_asm_parseval():
    u = crandn(64, 64)
    out = D.asm(u, 10e-6, 10e-6, 633e-9, 0.3, nopad=True)
    assert abs(np.linalg.norm(out) / np.linalg.norm(u) - 1.0) < 1e-12
    out = D.asm(u, 10e-6, 10e-6, 633e-9, 0.3)
    assert np.linalg.norm(out) <= np.linalg.norm(u) * (1 + 1e-12)


def test_asm_evanescent_cutoff_exact_boundary():
    # dx = 2^-20 m, M = 16, lambda = 2^-18 m: bin p has lambda*fx = p/4 exactly,
    # so p = 4 sits on the boundary (s == 1, propagating, H = 1) and |p| > 4 is evanescent
    dx = 2.0 ** -20
    lam = 2.0 ** -18
    h = D.asm_transfer(16, 16, dx, dx, lam, 0.37)
    row = h[0]
    assert row[4] == 1.0 and row[12] == 1.0            # s == 1 exactly, both signs
    for p in (5, 6, 7, 8, 9, 10, 11):
        assert row[p] == 0.0
    assert np.all(np.abs(np.abs(row[[0, 1, 2, 3, 13, 14, 15]]) - 1.0) < 1e-15)
    # realistic case: 0.3 um pitch, 633 nm: exactly the bins with f > 1/lambda are zero
    m, d, lam = 64, 0.3e-6, 633e-9
    h = D.asm_transfer(m, m, d, d, lam, 1e-5)
    f = D.frequencies(m, d)
    f2 = f[:, None] ** 2 + f[None, :] ** 2
    assert np.all(h[f2 > 1.0 / lam ** 2] == 0)
    assert np.all(np.abs(np.abs(h[f2 < 0.999 / lam ** 2]) - 1.0) < 1e-14)


def _gaussian_grid(n, d, w0):
    c = (np.arange(n) - n / 2) * d
    y, x = np.meshgrid(c, c, indexing="ij")
    return np.exp(-(x * x + y * y) / w0 ** 2), x * x + y * y


def _gaussian_fresnel_closed_form(r2, w0, lam, z):
    zr = np.pi * w0 ** 2 / lam
    q = 1 + 1j * z / zr
    k = 2 * np.pi / lam
    return np.exp(1j * k * z) / q * np.exp(-r2 / (w0 ** 2 * q))


def test_fresnel_gaussian_closed_form():
    # u1 = exp(-r^2/w0^2) -> e^{ikz}/(1 + iz/zR) exp(-r^2/(w0^2 (1 + iz/zR))), zR = pi w0^2/lam;
    # z >= 2 N dx^2 / lam keeps the chirp sampled; the beam stays far from the edges
    n, d, lam, w0, z = 256, 10e-6, 633e-9, 200e-6, 0.1
    u1, r2 = _gaussian_grid(n, d, w0)
    expect = _gaussian_fresnel_closed_form(r2, w0, lam, z)
    out = D.fresnel(u1, d, d, lam, z)
    assert rel(out, expect) < 1e-12
    out_tf = D.fresnel(u1, d, d, lam, z, fresnel_tf="analytic")
    assert rel(out_tf, expect) < 1e-9


def test_asm_gaussian_paraxial():
    n, d, lam, w0, z = 256, 10e-6, 633e-9, 200e-6, 0.1
    u1, r2 = _gaussian_grid(n, d, w0)
    expect = _gaussian_fresnel_closed_form(r2, w0, lam, z)
    out = D.asm(u1, d, d, lam, z)
    assert rel(out, expect) < 1e-5


def _fresnel_brute(u1, dx, dy, lam, z):
    ny, nx = u1.shape
    k = 2 * np.pi / lam
    c = dx * dy * np.exp(1j * k * z) / (1j * lam * z)
    out = np.zeros((ny, nx), complex)
    jy, jx = np.mgrid[0:ny, 0:nx]
    for my in range(ny):
        for mx in range(nx):
            ox = (mx - jx) * dx
            oy = (my - jy) * dy
            out[my, mx] = c * np.sum(u1 * np.exp(1j * np.pi * (ox * ox + oy * oy) / (lam * z)))
    return out


@pytest.mark.parametrize("shape", [(32, 32), (16, 32)])
def test_fresnel_brute_force_sum(shape):
    u1 = crandn(*shape)
    dx, dy, lam, z = 10e-6, 7e-6, 532e-9, 0.05
    out = D.fresnel(u1, dx, dy, lam, z)
    assert rel(out, _fresnel_brute(u1, dx, dy, lam, z)) < 1e-12


def test_fresnel_negative_z_brute_force():
    u1 = crandn(16, 16)
    out = D.fresnel(u1, 9e-6, 9e-6, 473e-9, -0.08)
    assert rel(out, _fresnel_brute(u1, 9e-6, 9e-6, 473e-9, -0.08)) < 1e-12


@pytest.mark.parametrize("shape", [(32, 32), (16, 32)])
def test_asm_brute_force_circular_sum(shape):
    # u2[m] = sum_j u1[j] g[(m - j) mod M], g = IDFT_M(H), on the 2N x 2N circle
    ny, nx = shape
    u1 = crandn(ny, nx)
    dx, dy, lam, z = 6e-6, 9e-6, 633e-9, 0.02
    my, mx = 2 * ny, 2 * nx
    h = D.asm_transfer(my, mx, dy, dx, lam, z)
    g = dft.dft2_direct(h, inverse=True) / (mx * my)
    out = np.zeros((ny, nx), complex)
    for ym in range(ny):
        for xm in range(nx):
            iy = (ym - np.arange(ny))[:, None] % my
            ix = (xm - np.arange(nx))[None, :] % mx
            out[ym, xm] = np.sum(u1 * g[iy, ix])
    assert rel(D.asm(u1, dx, dy, lam, z), out) < 1e-12


def test_fresnel_impulse_transform_is_separable():
    # DFT2 of h(y) h(x) equals the outer product of the two 1-D DFTs
    my, mx, ny, nx = 32, 64, 16, 32
    dy, dx, lam, z = 8e-6, 10e-6, 633e-9, 0.07
    h = D.fresnel_impulse(my, mx, ny, nx, dy, dx, lam, z)
    hx = h[0, :] / h[0, 0]
    hy = h[:, 0]
    full = dft.dft2_direct(h)
    sep = np.outer(dft.dft1_direct(hy), dft.dft1_direct(hx))
    assert rel(full, sep) < 1e-13


def test_placement_invariance():
    # any consistent placement of the field in the padded grid gives the same crop
    ny, nx = 16, 16
    u1 = crandn(ny, nx)
    dx, lam, z = 10e-6, 633e-9, 0.03
    ref = D.asm(u1, dx, dx, lam, z)
    my, mx = 2 * ny, 2 * nx
    a = np.zeros((my, mx), complex)
    oy, ox = 7, 11
    a[oy:oy + ny, ox:ox + nx] = u1
    spec = dft.dft2_direct(a) * D.asm_transfer(my, mx, dx, dx, lam, z)
    b = dft.dft2_direct(spec, True) / (mx * my)
    assert rel(b[oy:oy + ny, ox:ox + nx], ref) < 1e-13


def test_linearity():
    u, v = crandn(32, 32), crandn(32, 32)
    al, be = 0.3 - 1.2j, -2.0 + 0.5j
    for kind in (D.ASM, D.FRESNEL):
        lhs = D.propagate(al * u + be * v, kind, 8e-6, 8e-6, 532e-9, 0.05)
        rhs = al * D.propagate(u, kind, 8e-6, 8e-6, 532e-9, 0.05) + \
            be * D.propagate(v, kind, 8e-6, 8e-6, 532e-9, 0.05)
        assert rel(lhs, rhs) < 1e-13


def test_direct_and_fft_backends_agree():
    u = crandn(128, 128)
    for kind in (D.ASM, D.FRESNEL):
        a = D.propagate(u, kind, 8e-6, 8e-6, 532e-9, 0.05, method="direct")
        b = D.propagate(u, kind, 8e-6, 8e-6, 532e-9, 0.05, method="fft")
        assert rel(a, b) < 1e-13


def test_invalid_parameters():
    u = crandn(16, 16)
    with pytest.raises(ValueError):
        D.fresnel(u, 10e-6, 10e-6, 633e-9, 0.0)
    with pytest.raises(ValueError):
        D.asm(u, -1e-6, 10e-6, 633e-9, 0.1)
    with pytest.raises(ValueError):
        D.asm(u, 1e-6, 10e-6, float("nan"), 0.1)


# ---- GS ping-pong step ---------------------------------------------------------

def test_amplitude_constraint():
    u = crandn(16, 16)
    u[3, 4] = 0
    a = np.abs(crandn(16, 16))
    c = gs.amplitude_constraint(u, a)
    assert np.allclose(np.abs(c), a, rtol=1e-15, atol=0)
    mask = np.abs(u) > 0
    assert np.allclose(np.angle(c[mask]), np.angle(u[mask]), atol=1e-14)
    assert c[3, 4] == a[3, 4]


def test_gs_iteration_composition():
    n = 32
    a1 = np.abs(crandn(n, n))
    a2 = np.abs(crandn(n, n))
    u0 = a1 * np.exp(1j * RNG.uniform(0, 2 * np.pi, (n, n)))
    u1, e0 = gs.iteration(u0, a1, a2, 8e-6, 532e-9, 0.02)
    assert np.allclose(np.abs(u1), a1, rtol=1e-14, atol=0)
    v = D.asm(u0, 8e-6, 8e-6, 532e-9, 0.02)
    assert abs(e0 - np.linalg.norm(np.abs(v) - a2) / np.linalg.norm(a2)) < 1e-15


def test_gs_error_hand_values():
    # |v| = (5, 0, 1) against a = (5, 2, 1): the difference is (0, -2, 0), so
    # E = 2 / sqrt(25 + 4 + 1)
    v = np.array([3 + 4j, 0, 1j])
    a = np.array([5.0, 2.0, 1.0])
    assert gs.error(v, a) == pytest.approx(2 / math.sqrt(30), rel=1e-15)
    # the amplitude alone counts: any phase on the target amplitude gives 0
    ph = np.exp(1j * np.array([0.3, -2.0, 3.1]))
    assert gs.error(a * ph, a) < 1e-15  # |a e^{i phi}| rounds to within an ulp of a
    # a zero field and a field of twice the amplitude are both at distance ||a||
    assert gs.error(np.zeros(3), a) == 1.0
    assert gs.error(2 * a * ph, a) == pytest.approx(1.0, rel=1e-15)
    # 2-D arrays: the norm runs over every element
    assert gs.error(np.array([[1j, 0], [0, 0]]), np.array([[1.0, 1.0], [1.0, 1.0]])) == \
        pytest.approx(math.sqrt(3) / 2, rel=1e-15)


def test_gs_iteration_at_zero_distance_is_a_fixed_point():
    # ASM at z = 0 is the identity, so from u0 = A1 exp(i phi) the step returns u0 and
    # E_0 = ||A1 - A2|| / ||A2||, here from hand values on a 16x16 grid with two levels
    n = 16
    a1 = np.full((n, n), 2.0)
    a2 = np.full((n, n), 1.0)
    a2[: n // 2] = 3.0
    phi = np.linspace(-3.0, 3.0, n * n).reshape(n, n)
    u0 = a1 * np.exp(1j * phi)
    u1, e0 = gs.iteration(u0, a1, a2, 8e-6, 532e-9, 0.0)
    assert np.allclose(u1, u0, rtol=0, atol=1e-13)
    # half the pixels differ by 1, half by 1; ||A2||^2 = n^2/2 * (9 + 1)
    assert e0 == pytest.approx(math.sqrt(n * n) / math.sqrt(n * n / 2 * 10), rel=1e-13)

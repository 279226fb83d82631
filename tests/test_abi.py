"""CPU-side checks of the C ABI: the library loads, exports every symbol the header
declares, and validates parameters on the host (no compute call needs a GPU here)."""
import ctypes
import math
import os
import re

import pytest

from paper_1107_5578_amd import cwo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "cwo.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cwo_\w+)\s*\(", txt)))


def test_header_declarations_are_exported():
    lib = cwo.load()
    names = declared_functions()
    assert "cwo_asm" in names and "cwo_fresnel" in names
    for name in names:
        assert hasattr(lib, name), name
    # the binding knows every declared symbol and nothing else
    assert sorted(cwo.SIGNATURES) == names


def test_params_struct_layout_matches_header():
    # int32 nx, ny; double dx, dy, wavelength, z; int32 kind, precision; uint32 flags
    assert ctypes.sizeof(cwo.Params) == 4 + 4 + 8 * 4 + 4 + 4 + 4 + 4  # trailing pad to 8
    assert cwo.Params.dx.offset == 8 and cwo.Params.kind.offset == 40


def test_strerror_and_version():
    assert cwo.strerror(0) == "ok"
    assert "unsupported" in cwo.strerror(cwo.CWO_ERR_UNSUPPORTED)
    assert cwo.strerror(12345) == "unknown status"
    assert cwo.load().cwo_version() >= 100


@pytest.mark.parametrize("kind", [cwo.ANGULAR, cwo.FRESNEL_CONV])
def test_valid_params(kind):
    for n in (16, 32, 256, 1024, 4096):
        p = cwo.make_params(n, n, 10e-6, z=0.1)
        assert cwo.check_params(p, kind) == cwo.CWO_OK
    p = cwo.make_params(64, 16, 8e-6, 4e-6, 532e-9, -0.3)
    assert cwo.check_params(p, kind) == cwo.CWO_OK


@pytest.mark.parametrize("nx,ny", [(15, 16), (300, 256), (8, 8), (8192, 16), (16, 0), (-16, 16)])
def test_unsupported_sizes(nx, ny):
    p = cwo.make_params(nx, ny, 10e-6, z=0.1)
    assert cwo.check_params(p, cwo.ANGULAR) == cwo.CWO_ERR_UNSUPPORTED


@pytest.mark.parametrize("field,value", [("dx", 0.0), ("dx", -1e-6), ("dy", math.nan),
                                          ("wavelength", 0.0), ("wavelength", math.inf),
                                          ("z", math.nan), ("z", -math.inf)])
def test_invalid_physical_params(field, value):
    p = cwo.make_params(64, 64, 10e-6, z=0.1)
    setattr(p, field, value)
    assert cwo.check_params(p, cwo.ANGULAR) == cwo.CWO_ERR_INVALID


def test_fresnel_z0_invalid_asm_z0_valid():
    p = cwo.make_params(64, 64, 10e-6, z=0.0)
    assert cwo.check_params(p, cwo.FRESNEL_CONV) == cwo.CWO_ERR_INVALID
    assert cwo.check_params(p, cwo.ANGULAR) == cwo.CWO_OK


def test_kind_flags_precision_checks():
    p = cwo.make_params(64, 64, 10e-6, z=0.1, kind=cwo.FRESNEL_CONV)
    assert cwo.check_params(p, cwo.ANGULAR) == cwo.CWO_ERR_INVALID   # kind mismatch
    assert cwo.check_params(p, 7) == cwo.CWO_ERR_INVALID             # unknown kind
    p = cwo.make_params(64, 64, 10e-6, z=0.1)
    p.flags = 0x80
    assert cwo.check_params(p, cwo.ANGULAR) == cwo.CWO_ERR_INVALID
    p = cwo.make_params(64, 64, 10e-6, z=0.1)
    p.precision = 9
    assert cwo.check_params(p, cwo.ANGULAR) == cwo.CWO_ERR_INVALID
    assert cwo.load().cwo_check_params(None, cwo.ANGULAR) == cwo.CWO_ERR_INVALID


def test_fresnel_tf_flag_only_for_the_convolution_form():
    for nopad in (False, True):
        p = cwo.make_params(64, 32, 10e-6, 8e-6, 633e-9, -0.1, cwo.FRESNEL_CONV, "f32", nopad, True)
        assert p.flags == (cwo.FLAG_FRESNEL_TF | (cwo.FLAG_NOPAD if nopad else 0))
        assert cwo.check_params(p, cwo.FRESNEL_CONV) == cwo.CWO_OK
    p = cwo.make_params(64, 64, 10e-6, None, 633e-9, 0.1, cwo.FRESNEL_CONV, "f16", False, True)
    assert cwo.check_params(p, cwo.FRESNEL_CONV) == cwo.CWO_OK
    for kind in (cwo.ANGULAR, cwo.FRESNEL_FOURIER, cwo.FRESNEL_SHIFTED):
        p = cwo.make_params(64, 64, 10e-6, None, 633e-9, 0.1, kind, "f32", False, True)
        assert cwo.check_params(p, kind) == cwo.CWO_ERR_INVALID


def test_scratch_bytes():
    lib = cwo.load()
    p = cwo.make_params(2048, 2048, 8e-6, z=0.5)
    assert lib.cwo_scratch_bytes(ctypes.byref(p)) == 8 * 2048 * 4096
    p = cwo.make_params(64, 32, 8e-6, z=0.5, nopad=True)
    assert lib.cwo_scratch_bytes(ctypes.byref(p)) == 8 * 32 * 64
    p = cwo.make_params(63, 32, 8e-6, z=0.5)
    assert lib.cwo_scratch_bytes(ctypes.byref(p)) == 0


def test_null_context_and_pointers_are_invalid():
    lib = cwo.load()
    p = cwo.make_params(64, 64, 10e-6, z=0.1)
    assert lib.cwo_asm(None, ctypes.byref(p), None, None, None) == cwo.CWO_ERR_INVALID
    assert lib.cwo_destroy(None) == cwo.CWO_ERR_INVALID
    assert lib.cwo_create(None, 0, 0) == cwo.CWO_ERR_INVALID


def test_low_precision_storage_params():
    for prec in (cwo.PREC_F16, cwo.PREC_BF16):
        p = cwo.make_params(256, 256, 10e-6, z=0.1, precision=prec)
        assert cwo.check_params(p, cwo.ANGULAR) == cwo.CWO_OK
        assert cwo.check_params(p, cwo.FRESNEL_CONV) == cwo.CWO_OK
        assert cwo.load().cwo_scratch_bytes(ctypes.byref(p)) == 4 * 256 * 512
        p = cwo.make_params(256, 256, 10e-6, z=0.1, precision=prec, nopad=True)
        assert cwo.check_params(p, cwo.ANGULAR) == cwo.CWO_ERR_UNSUPPORTED


def test_band_limit_host_function():
    from oracle import shifted_asm as S
    lib = cwo.load()
    for n, d, lam, z, nopad in [(2048, 8e-6, 532e-9, 0.5, False), (256, 10e-6, 633e-9, 2.0, True),
                                (64, 4e-6, 473e-9, -0.05, False)]:
        wx, wy = cwo.band_limit(n, n // 2, d, 2 * d, lam, z, nopad)
        assert math.isclose(wx, S.band_limit(n, d, lam, z, nopad), rel_tol=1e-14)
        assert math.isclose(wy, S.band_limit(n // 2, 2 * d, lam, z, nopad), rel_tol=1e-14)
    sh = cwo.Shift()
    p = cwo.make_params(64, 64, 10e-6, z=0.1)
    assert lib.cwo_band_limit(None, ctypes.byref(sh)) == cwo.CWO_ERR_INVALID
    assert lib.cwo_band_limit(ctypes.byref(p), None) == cwo.CWO_ERR_INVALID
    p.dx = 0.0
    assert lib.cwo_band_limit(ctypes.byref(p), ctypes.byref(sh)) == cwo.CWO_ERR_INVALID
    assert lib.cwo_asm_shifted(None, ctypes.byref(p), ctypes.byref(sh), None, None,
                               None) == cwo.CWO_ERR_INVALID


def test_fresnel_fourier_params_and_pitch():
    from oracle import fresnel_fourier as F
    lib = cwo.load()
    K = cwo.FRESNEL_FOURIER
    p = cwo.make_params(512, 256, 10e-6, 8e-6, 633e-9, 0.2, kind=K)
    assert cwo.check_params(p, K) == cwo.CWO_OK
    dx2, dy2 = cwo.fresnel_fourier_pitch(512, 256, 10e-6, 8e-6, 633e-9, 0.2)
    assert math.isclose(dx2, F.destination_pitch(512, 10e-6, 633e-9, 0.2), rel_tol=1e-15)
    assert math.isclose(dy2, F.destination_pitch(256, 8e-6, 633e-9, 0.2), rel_tol=1e-15)
    dx2, _ = cwo.fresnel_fourier_pitch(64, 64, 10e-6, 10e-6, 633e-9, -0.1)
    assert dx2 < 0
    bad = [dict(z=0.0), dict(z=math.nan), dict(dx=0.0), dict(flags=1), dict(kind=1)]
    for b in bad:
        q = cwo.make_params(64, 64, 10e-6, z=0.1, kind=K)
        for k, v in b.items():
            setattr(q, k, v)
        assert cwo.check_params(q, K) == cwo.CWO_ERR_INVALID, b
    q = cwo.make_params(64, 64, 10e-6, z=0.1, kind=K, precision="f16")
    assert cwo.check_params(q, K) == cwo.CWO_ERR_UNSUPPORTED
    q = cwo.make_params(8192, 64, 10e-6, z=0.1, kind=K)
    assert cwo.check_params(q, K) == cwo.CWO_ERR_UNSUPPORTED
    assert lib.cwo_fresnel_fourier(None, ctypes.byref(p), None, None, None) == cwo.CWO_ERR_INVALID


def test_fresnel_shifted_params():
    lib = cwo.load()
    K = cwo.FRESNEL_SHIFTED
    p = cwo.make_params(256, 128, 10e-6, 8e-6, 633e-9, 0.2, kind=K)
    assert cwo.check_params(p, K) == cwo.CWO_OK
    for b in [dict(z=0.0), dict(flags=1), dict(kind=2), dict(wavelength=-1.0)]:
        q = cwo.make_params(64, 64, 10e-6, z=0.1, kind=K)
        for k, v in b.items():
            setattr(q, k, v)
        assert cwo.check_params(q, K) == cwo.CWO_ERR_INVALID, b
    q = cwo.make_params(64, 64, 10e-6, z=0.1, kind=K, precision="bf16")
    assert cwo.check_params(q, K) == cwo.CWO_ERR_UNSUPPORTED
    w = cwo.SFresnel(5e-6, 5e-6, 0.0, 0.0, 1e-3, 0.0)
    assert lib.cwo_fresnel_shifted(None, ctypes.byref(p), ctypes.byref(w), None, None,
                                   None) == cwo.CWO_ERR_INVALID


def test_autotune_null_context():
    p = cwo.make_params(64, 64, 10e-6, z=0.1, kind=cwo.ANGULAR)
    t = cwo.Tuning()
    assert cwo.load().cwo_autotune(None, ctypes.byref(p), 1, None, None, None,
                                   ctypes.byref(t)) == cwo.CWO_ERR_INVALID


def test_point_light_source_and_fused_intensity_null_context():
    lib = cwo.load()
    pp = cwo.PlsParams(64, 32, 4e-6, 4e-6, 633e-9, 0.0, 0.0, 0.2)
    assert ctypes.sizeof(cwo.PlsParams) == 56
    for fn in (lib.cwo_pls_cgh, lib.cwo_pls_field):
        assert fn(None, ctypes.byref(pp), None, 0, None, None) == cwo.CWO_ERR_INVALID
        assert fn(None, None, None, 0, None, None) == cwo.CWO_ERR_INVALID
    p = cwo.make_params(64, 64, 10e-6, z=0.1)
    for fn in (lib.cwo_asm_intensity, lib.cwo_fresnel_intensity):
        assert fn(None, ctypes.byref(p), None, None, None) == cwo.CWO_ERR_INVALID

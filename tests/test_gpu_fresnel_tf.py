"""GPU parity of the Fresnel propagation with the analytic transfer function
(CWO_FLAG_FRESNEL_TF: H = exp(ikz) exp(-i pi lambda z (fx^2 + fy^2)), the Fourier transform
of the continuous Fresnel kernel of Sec. 2.1.1) against the oracle's analytic form.

The oracle's analytic form is pinned in the CPU suite by the Gaussian-beam closed form.
Gates as for the other FP32 parity tests: relative L2 <= 1e-5 and every element within
1e-5 of the plane's peak; FP16 storage relative L2 <= 3e-3. Z-stack planes and batched
jobs with the flag are bit-identical to single calls with it, and the flag is shown to
change the result where the sampled chirp is aliased (so the two forms differ).
"""
import sys

import numpy as np
import pytest

from oracle import diffraction as D
from paper_1107_5578_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_1107_5578_amd import cwo
    c = cwo.Context(0)
    yield c
    c.close()


def note(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def run(ctx, u, dx, dy, lam, z, nopad=False, precision="f32"):
    import torch
    note("fresnel-tf n=%s dx=%g dy=%g lam=%g z=%g nopad=%s %s" % (u.shape, dx, dy, lam, z, nopad,
                                                                  precision))
    t = torch.from_numpy(np.ascontiguousarray(u.astype(np.complex64))).cuda()
    out = ctx.fresnel(t, dx, dy, lam, z, nopad=nopad, precision=precision, fresnel_tf=True)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(y, ref, label, rel_tol=1e-5, elem_tol=1e-5):
    rl = D.rel_l2(y, ref)
    peak = float(np.max(np.abs(ref)))
    emax = float(np.max(np.abs(y.astype(np.complex128) - ref)))
    note("%s rel_l2=%.3e max_abs_err/peak=%.3e" % (label, rl, emax / peak))
    assert np.all(np.isfinite(y))
    assert rl <= rel_tol
    if elem_tol is not None:
        assert emax <= elem_tol * peak


@pytest.mark.parametrize("nx,ny,dx,dy,lam,z", [
    (256, 256, 10e-6, 10e-6, 633e-9, 0.1),
    (128, 256, 8e-6, 12e-6, 532e-9, 0.03),
    (64, 32, 6e-6, 6e-6, 473e-9, -0.02),
    (16, 16, 10e-6, 10e-6, 633e-9, 0.5),
])
def test_parity_small(ctx, nx, ny, dx, dy, lam, z):
    u = W.uniform_random_field(nx, 71, ny=ny)
    ref = D.fresnel(u, dx, dy, lam, z, fresnel_tf="analytic")
    check(run(ctx, u, dx, dy, lam, z), ref, "tf-%dx%d" % (ny, nx))


def test_parity_nopad(ctx):
    u = W.uniform_random_field(128, 72)
    ref = D.fresnel(u, 8e-6, 8e-6, 633e-9, 0.05, nopad=True, fresnel_tf="analytic")
    check(run(ctx, u, 8e-6, 8e-6, 633e-9, 0.05, nopad=True), ref, "tf-nopad-128")


def test_parity_2048(ctx):
    cfg = W.PLANE_2048
    u = W.field_for(cfg)
    ref = D.fresnel(u, cfg.pitch, cfg.pitch, cfg.wavelength, cfg.z, fresnel_tf="analytic")
    check(run(ctx, u, cfg.pitch, cfg.pitch, cfg.wavelength, cfg.z), ref, "tf-2048")


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_low_precision(ctx, prec):
    u = W.rectangles_field(512, 73)
    ref = D.fresnel(u, 8e-6, 8e-6, 532e-9, 0.2, fresnel_tf="analytic")
    check(run(ctx, u, 8e-6, 8e-6, 532e-9, 0.2, precision=prec), ref, "tf-512-" + prec,
          rel_tol=3e-3, elem_tol=None)


def test_differs_from_sampled_kernel(ctx):
    # z well below 2 N dx^2 / lambda: the sampled chirp aliases, the two forms differ
    import torch
    u = W.uniform_random_field(128, 74)
    t = torch.from_numpy(u).cuda()
    a = ctx.fresnel(t, 10e-6, 10e-6, 633e-9, 0.005, fresnel_tf=True).cpu().numpy()
    b = ctx.fresnel(t, 10e-6, 10e-6, 633e-9, 0.005).cpu().numpy()
    ra = D.fresnel(u, 10e-6, 10e-6, 633e-9, 0.005, fresnel_tf="analytic")
    rb = D.fresnel(u, 10e-6, 10e-6, 633e-9, 0.005)
    assert D.rel_l2(ra, rb) > 1e-2
    check(a, ra, "tf-aliased")
    check(b, rb, "sampled-aliased")


def test_zstack_and_batch_match_single_calls(ctx):
    import torch
    u = W.speckle_field(256, 75)
    t = torch.from_numpy(u).cuda()
    zs = [0.02, -0.05, 0.11, 0.3]
    stack = ctx.zstack(t, zs, 8e-6, 8e-6, 532e-9, kind="fresnel", fresnel_tf=True)
    singles = [ctx.fresnel(t, 8e-6, 8e-6, 532e-9, z, fresnel_tf=True) for z in zs]
    # a batch mixing the two forms on one field: not grouped into one stack
    o1 = torch.empty_like(t)
    o2 = torch.empty_like(t)
    ctx.batch([("fresnel", t, o1, dict(dx=8e-6, wavelength=532e-9, z=0.11, fresnel_tf=True)),
               ("fresnel", t, o2, dict(dx=8e-6, wavelength=532e-9, z=0.11))])
    plain = ctx.fresnel(t, 8e-6, 8e-6, 532e-9, 0.11)
    torch.cuda.synchronize()
    for k, z in enumerate(zs):
        assert torch.equal(stack[k], singles[k]), z
    assert torch.equal(o1, singles[2])
    assert torch.equal(o2, plain)
    ref = D.fresnel(u, 8e-6, 8e-6, 532e-9, 0.11, fresnel_tf="analytic")
    check(o1.cpu().numpy(), ref, "tf-batch")


def test_flag_rejected_elsewhere(ctx):
    import torch
    from paper_1107_5578_amd import cwo
    for kind in (cwo.ANGULAR, cwo.FRESNEL_FOURIER):
        p = cwo.make_params(64, 64, 10e-6, 10e-6, 633e-9, 0.1, kind, "f32", False, True)
        assert cwo.check_params(p, kind) == cwo.CWO_ERR_INVALID
    p = cwo.make_params(64, 64, 10e-6, 10e-6, 633e-9, 0.1, cwo.FRESNEL_CONV, "f32", False, True)
    assert cwo.check_params(p, cwo.FRESNEL_CONV) == cwo.CWO_OK
    u = torch.zeros((64, 64), dtype=torch.complex64, device="cuda")
    with pytest.raises(cwo.CwoError) as e:
        ctx.fresnel(u, 10e-6, z=0.0, fresnel_tf=True)
    assert e.value.status == cwo.CWO_ERR_INVALID

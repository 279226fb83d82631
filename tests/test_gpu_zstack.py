"""GPU parity of the z-stack (one field, many distances) and the batch entry point.

Every plane of a stack is compared with the single-plane call of the same distance
(same kernels for the shared forward part; the inverse part differs only in
instruction scheduling, so agreement is expected to rounding level) and with the
FP64 oracle (relative L2 <= 1e-5 per plane, element-wise <= 1e-5 of the plane's peak).
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


def check(y, ref, label, rel_tol=1e-5, elem_tol=1e-5):
    rl = D.rel_l2(y, ref)
    peak = float(np.max(np.abs(ref)))
    emax = float(np.max(np.abs(y.astype(np.complex128) - ref)))
    note("%s rel_l2=%.3e max_abs_err/peak=%.3e" % (label, rl, emax / peak))
    assert rl <= rel_tol, (label, rl)
    assert emax <= elem_tol * peak, (label, emax / peak)


def single(ctx, kind, t, dx, lam, z):
    fn = ctx.asm if kind == "asm" else ctx.fresnel
    return fn(t, dx, dx, lam, z)


def test_zstack_1024_64_planes(ctx):
    import torch
    cfg = W.ZSTACK_1024
    u = W.field_for(cfg)
    zs = W.zstack_distances(64, 0.05, 0.2)
    note("zstack asm n=1024 nz=64 pitch=%g lam=%g" % (cfg.pitch, cfg.wavelength))
    t = torch.from_numpy(u).cuda()
    stack = ctx.zstack(t, zs, cfg.pitch, cfg.pitch, cfg.wavelength, kind="asm")
    torch.cuda.synchronize()
    worst = 0.0
    for k, z in enumerate(zs):
        one = single(ctx, "asm", t, cfg.pitch, cfg.wavelength, z)
        torch.cuda.synchronize()
        worst = max(worst, D.rel_l2(stack[k].cpu().numpy(), one.cpu().numpy().astype(np.complex128)))
    note("zstack vs single calls: worst rel_l2 = %.3e" % worst)
    assert worst <= 1e-6
    for k in (0, 21, 42, 63):
        ref = D.asm(u, cfg.pitch, cfg.pitch, cfg.wavelength, zs[k])
        check(stack[k].cpu().numpy(), ref, "zstack-1024 plane %d" % k)


@pytest.mark.parametrize("kind", ["asm", "fresnel"])
@pytest.mark.parametrize("n,ny", [(256, 256), (64, 128), (2048, 2048)])
def test_zstack_sizes(ctx, kind, n, ny):
    import torch
    u = W.uniform_random_field(n, n + ny, ny=ny)
    zs = [0.02, -0.05, 0.11, 0.3, 0.5] if kind == "asm" else [0.02, -0.05, 0.11, 0.3]
    note("zstack %s %dx%d nz=%d" % (kind, n, ny, len(zs)))
    t = torch.from_numpy(u).cuda()
    stack = ctx.zstack(t, zs, 8e-6, 8e-6, 532e-9, kind=kind)
    torch.cuda.synchronize()
    for k, z in enumerate(zs):
        one = single(ctx, kind, t, 8e-6, 532e-9, z).cpu().numpy()
        assert D.rel_l2(stack[k].cpu().numpy(), one.astype(np.complex128)) <= 1e-6
    for k in (0, len(zs) - 1):
        ref = D.propagate(u, kind, 8e-6, 8e-6, 532e-9, zs[k])
        check(stack[k].cpu().numpy(), ref, "zstack-%s-%dx%d plane %d" % (kind, n, ny, k))


@pytest.mark.parametrize("kind", ["asm", "fresnel"])
def test_zstack_4096(ctx, kind):
    # padded length 8192: the longest transforms (32 values per thread), the largest
    # z-stack LDS footprint and the largest FP64 chirp transforms
    import torch
    n = 4096
    u = W.uniform_random_field(n, 4096 + (kind == "fresnel"))
    zs = [0.35, -0.6]
    note("zstack %s %dx%d nz=%d" % (kind, n, n, len(zs)))
    t = torch.from_numpy(u).cuda()
    stack = ctx.zstack(t, zs, 8e-6, 8e-6, 532e-9, kind=kind)
    torch.cuda.synchronize()
    for k, z in enumerate(zs):
        one = single(ctx, kind, t, 8e-6, 532e-9, z).cpu().numpy()
        assert D.rel_l2(stack[k].cpu().numpy(), one.astype(np.complex128)) <= 1e-6
    ref = D.propagate(u, kind, 8e-6, 8e-6, 532e-9, zs[1])
    check(stack[1].cpu().numpy(), ref, "zstack-%s-4096 plane 1" % kind)


def test_zstack_exact_phase_path(ctx):
    # 0.6 um pitch at 633 nm: s reaches 2*(lambda/2dx)^2 = 0.56 > 0.05, so the stack takes
    # the exact per-bin FP64 form (and evanescent bins appear at the corners)
    import torch
    u = W.uniform_random_field(128, 77)
    zs = [1e-5, 3e-5, -2e-5]
    t = torch.from_numpy(u).cuda()
    stack = ctx.zstack(t, zs, 0.6e-6, 0.6e-6, 633e-9, kind="asm")
    torch.cuda.synchronize()
    for k, z in enumerate(zs):
        check(stack[k].cpu().numpy(), D.asm(u, 0.6e-6, 0.6e-6, 633e-9, z), "exact-z plane %d" % k)


def test_zstack_chunked_by_budget(ctx):
    # a budget that holds the spectrum and two planes forces chunks of two
    import torch
    from paper_1107_5578_amd import cwo
    n = 128
    plane = 8 * n * 2 * n
    small = cwo.Context(0, hbm_budget_bytes=3 * plane)
    try:
        u = torch.from_numpy(W.uniform_random_field(n, 5)).cuda()
        zs = [0.01 * (k + 1) for k in range(7)]
        a = small.zstack(u, zs, 10e-6, 10e-6, 633e-9, kind="asm")
        b = ctx.zstack(u, zs, 10e-6, 10e-6, 633e-9, kind="asm")
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        tiny = cwo.Context(0, hbm_budget_bytes=plane)
        with pytest.raises(cwo.CwoError) as e:
            tiny.zstack(u, zs, 10e-6, 10e-6, 633e-9, kind="asm")
        assert e.value.status == cwo.CWO_ERR_NOMEM
        tiny.close()
    finally:
        small.close()


def test_batch_mixed(ctx):
    import torch
    u1 = torch.from_numpy(W.uniform_random_field(256, 1)).cuda()
    u2 = torch.from_numpy(W.uniform_random_field(512, 2)).cuda()
    u3 = torch.from_numpy(W.uniform_random_field(64, 3, ny=32)).cuda()
    jobs = []
    outs = []
    spec = [("asm", u1, dict(dx=10e-6, wavelength=633e-9, z=0.1)),
            ("asm", u1, dict(dx=10e-6, wavelength=633e-9, z=0.2)),
            ("asm", u1, dict(dx=10e-6, wavelength=633e-9, z=-0.05)),
            ("fresnel", u2, dict(dx=8e-6, wavelength=532e-9, z=0.3)),
            ("fresnel", u2, dict(dx=8e-6, wavelength=532e-9, z=0.4)),
            ("asm", u3, dict(dx=4e-6, wavelength=473e-9, z=0.01)),
            ("fresnel", u1, dict(dx=10e-6, wavelength=633e-9, z=0.1))]
    for kind, u, kw in spec:
        o = torch.empty_like(u)
        outs.append(o)
        jobs.append((kind, u, o, kw))
    ctx.batch(jobs)
    torch.cuda.synchronize()
    for (kind, u, kw), o in zip(spec, outs):
        one = (ctx.asm if kind == "asm" else ctx.fresnel)(u, kw["dx"], kw["dx"], kw["wavelength"],
                                                          kw["z"])
        torch.cuda.synchronize()
        assert D.rel_l2(o.cpu().numpy(), one.cpu().numpy().astype(np.complex128)) <= 1e-6
    ref = D.fresnel(u2.cpu().numpy(), 8e-6, 8e-6, 532e-9, 0.4)
    check(outs[4].cpu().numpy(), ref, "batch fresnel 512")


def test_batch_validation_before_launch(ctx):
    import torch
    from paper_1107_5578_amd import cwo
    u = torch.from_numpy(W.uniform_random_field(64, 1)).cuda()
    o = torch.zeros_like(u)
    with pytest.raises(cwo.CwoError) as e:
        ctx.batch([("asm", u, o, dict(z=0.1)), ("fresnel", u, torch.zeros_like(u), dict(z=0.0))])
    assert e.value.status == cwo.CWO_ERR_INVALID
    torch.cuda.synchronize()
    assert torch.count_nonzero(o).item() == 0   # nothing ran


@pytest.mark.parametrize("n,kind", [(256, "asm"), (512, "fresnel"), (64, "asm")])
def test_batch_independent_fields(ctx, n, kind):
    # identical parameters on different fields run as one batch per pass: every output
    # equals the single call bit for bit (same kernels, one more grid dimension)
    import torch
    note("batch of independent %s fields %d^2" % (kind, n))
    fields = [torch.from_numpy(W.uniform_random_field(n, 700 + k)).cuda() for k in range(11)]
    outs = [torch.empty_like(f) for f in fields]
    kw = dict(dx=8e-6, dy=8e-6, wavelength=532e-9, z=0.07)
    ctx.batch([(kind, f, o, kw) for f, o in zip(fields, outs)])
    torch.cuda.synchronize()
    single = ctx.asm if kind == "asm" else ctx.fresnel
    for f, o in zip(fields, outs):
        ref = single(f, 8e-6, 8e-6, 532e-9, 0.07)
        torch.cuda.synchronize()
        assert torch.equal(o, ref)
    check(outs[3].cpu().numpy(), D.propagate(fields[3].cpu().numpy(), kind, 8e-6, 8e-6, 532e-9,
                                             0.07), "batched field 3")


@pytest.mark.parametrize("n", [256, 2048])
def test_batch_mixed_parameters_one_launch_per_pass(ctx, n):
    """Jobs of one geometry on different fields with different distances, wavelengths and
    kinds run as one batch: one launch for each row pass and one column launch per
    transfer-function form present (the library's own launch counts), every plane equal to
    its single call bit for bit, and planes of each kind against the FP64 oracle (ASM and
    Fresnel, near and far, negative z)."""
    import torch
    from paper_1107_5578_amd import cwo
    note("mixed-parameter batch %d^2" % n)
    rng = np.random.default_rng(91)
    specs = []
    for k in range(9):
        kind = "asm" if k % 3 != 1 else "fresnel"
        z = float(rng.uniform(0.02, 0.9)) * (-1.0 if k == 5 else 1.0)
        lam = float((473e-9, 532e-9, 633e-9)[k % 3])
        specs.append((kind, dict(dx=8e-6, dy=8e-6, wavelength=lam, z=z)))
    fields = [torch.from_numpy(W.uniform_random_field(n, 900 + k)).cuda() for k in range(len(specs))]
    outs = [torch.empty_like(f) for f in fields]
    ctx.batch([(kind, f, o, kw) for (kind, kw), f, o in zip(specs, fields, outs)])
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.batch([(kind, f, o, kw) for (kind, kw), f, o in zip(specs, fields, outs)])
    counts = {st: ctx.profile_read(st)[1] for st in (cwo.STAGE_ROW_FWD, cwo.STAGE_COL,
                                                      cwo.STAGE_ROW_INV)}
    ctx.profile(False)
    # ASM planes of one series length plus Fresnel planes: two column launches (at most three)
    assert counts[cwo.STAGE_ROW_FWD] == 1 and counts[cwo.STAGE_ROW_INV] == 1, counts
    assert 2 <= counts[cwo.STAGE_COL] <= 3, counts
    for (kind, kw), f, o in zip(specs, fields, outs):
        one = (ctx.asm if kind == "asm" else ctx.fresnel)(f, kw["dx"], kw["dy"], kw["wavelength"],
                                                          kw["z"])
        torch.cuda.synchronize()
        assert torch.equal(o, one), (kind, kw)
    for k in (0, 1, 5):
        kind, kw = specs[k]
        ref = D.propagate(fields[k].cpu().numpy(), kind, kw["dx"], kw["dy"], kw["wavelength"],
                          kw["z"])
        check(outs[k].cpu().numpy(), ref, "mixed batch plane %d (%s)" % (k, kind))


def test_batch_mixed_parameters_4096(ctx):
    """A mixed batch at 4096^2 (tiled plane, split transforms): one launch per row pass,
    every plane equal to its single call bit for bit, the Fresnel plane against the oracle."""
    import torch
    from paper_1107_5578_amd import cwo
    note("mixed-parameter batch 4096^2")
    specs = [("asm", dict(dx=8e-6, dy=8e-6, wavelength=473e-9, z=0.6)),
             ("fresnel", dict(dx=8e-6, dy=8e-6, wavelength=532e-9, z=0.35)),
             ("asm", dict(dx=8e-6, dy=8e-6, wavelength=633e-9, z=-0.2))]
    fields = [torch.from_numpy(W.uniform_random_field(4096, 940 + k)).cuda()
              for k in range(len(specs))]
    outs = [torch.empty_like(f) for f in fields]
    ctx.profile(True)
    ctx.batch([(kind, f, o, kw) for (kind, kw), f, o in zip(specs, fields, outs)])
    counts = {st: ctx.profile_read(st)[1] for st in (cwo.STAGE_ROW_FWD, cwo.STAGE_ROW_INV)}
    ctx.profile(False)
    assert counts[cwo.STAGE_ROW_FWD] == 1 and counts[cwo.STAGE_ROW_INV] == 1, counts
    for (kind, kw), f, o in zip(specs, fields, outs):
        one = (ctx.asm if kind == "asm" else ctx.fresnel)(f, kw["dx"], kw["dy"], kw["wavelength"],
                                                          kw["z"])
        torch.cuda.synchronize()
        assert torch.equal(o, one), (kind, kw)
    kind, kw = specs[1]
    ref = D.propagate(fields[1].cpu().numpy(), kind, kw["dx"], kw["dy"], kw["wavelength"], kw["z"])
    check(outs[1].cpu().numpy(), ref, "mixed batch 4096 plane 1 (fresnel)")


def test_batch_chained_jobs_keep_their_order(ctx):
    # a job that reads another job's output is not batched with it
    import torch
    u = torch.from_numpy(W.uniform_random_field(128, 5)).cuda()
    a = torch.empty_like(u)
    b = torch.empty_like(u)
    kw = dict(dx=8e-6, dy=8e-6, wavelength=532e-9, z=0.05)
    ctx.batch([("asm", u, a, kw), ("asm", a, b, kw)])
    torch.cuda.synchronize()
    ref = ctx.asm(ctx.asm(u, 8e-6, 8e-6, 532e-9, 0.05), 8e-6, 8e-6, 532e-9, 0.05)
    torch.cuda.synchronize()
    assert torch.equal(b, ref)

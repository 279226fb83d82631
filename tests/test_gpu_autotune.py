"""cwo_autotune: the picked schedule is a valid candidate, is kept for the parameter set,
and does not change any result (the candidates differ in scheduling only)."""
import sys

import pytest

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


@pytest.mark.parametrize("n,kind", [(2048, "asm"), (1024, "fresnel"), (256, "asm")])
def test_autotune_single_plane(ctx, n, kind):
    import torch
    u = torch.from_numpy(W.uniform_random_field(n, 60 + n)).cuda()
    fn = ctx.asm if kind == "asm" else ctx.fresnel
    before = fn(u, 8e-6, 8e-6, 532e-9, 0.3)
    torch.cuda.synchronize()
    form, zchunk, us = ctx.autotune(u, 1, 8e-6, 8e-6, 532e-9, 0.3, kind=kind)
    note("autotune %s %d: row_form=%d zchunk=%d %.1f us/plane" % (kind, n, form, zchunk, us))
    assert zchunk == 0 and us > 0
    assert form in ((1, 2) if n >= 512 else (0,))
    after = fn(u, 8e-6, 8e-6, 532e-9, 0.3)
    torch.cuda.synchronize()
    assert torch.equal(before, after)


def test_autotune_zstack(ctx):
    import torch
    cfg = W.ZSTACK_1024
    u = torch.from_numpy(W.field_for(cfg)).cuda()
    zs = list(W.zstack_distances(64, 0.05, 0.2))
    before = ctx.zstack(u, zs, cfg.pitch, cfg.pitch, cfg.wavelength)
    torch.cuda.synchronize()
    form, zchunk, us = ctx.autotune(u, 64, cfg.pitch, cfg.pitch, cfg.wavelength, 0.1)
    note("autotune zstack 1024x64: row_form=%d zchunk=%d %.1f us/plane" % (form, zchunk, us))
    assert zchunk in (2, 4, 8, 16, 32, 64) and form in (1, 2)
    after = ctx.zstack(u, zs, cfg.pitch, cfg.pitch, cfg.wavelength)
    torch.cuda.synchronize()
    assert torch.equal(before, after)


def test_autotune_errors(ctx):
    import torch
    from paper_1107_5578_amd import cwo
    u = torch.from_numpy(W.uniform_random_field(64, 1)).cuda()
    with pytest.raises(cwo.CwoError) as e:
        ctx.autotune(u, 0, 8e-6, 8e-6, 532e-9, 0.3)
    assert e.value.status == cwo.CWO_ERR_INVALID
    with pytest.raises(cwo.CwoError) as e:
        ctx.autotune(u, 4, 8e-6, 8e-6, 532e-9, 0.0, kind="fresnel")
    assert e.value.status == cwo.CWO_ERR_INVALID

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
    form, zchunk, us, layout, col_form = ctx.autotune(u, 1, 8e-6, 8e-6, 532e-9, 0.3, kind=kind)
    note("autotune %s %d: row_form=%d zchunk=%d layout=%d col_form=%d %.1f us/plane"
         % (kind, n, form, zchunk, layout, col_form, us))
    assert zchunk == 0 and us > 0
    if n >= 1024:   # padded rows of 2048 or more: row-major (two row forms) or tiled
        assert (layout, form) in ((1, 1), (1, 2), (2, 0))
        # the tiled plane's column forms exist for padded columns of 4096 and 8192
        assert col_form == 0 if layout == 1 or n < 2048 else col_form in (1, 2)
    else:
        assert layout == 0 and form in ((1, 2) if n >= 512 else (0,)) and col_form == 0
    after = fn(u, 8e-6, 8e-6, 532e-9, 0.3)
    torch.cuda.synchronize()
    # the tuned schedule runs other kernels over the same arithmetic: the default result to
    # the schedules' bar (1e-6 relative), usually bit for bit
    import numpy as np
    from oracle import diffraction as D
    err = D.rel_l2(after.cpu().numpy(), before.cpu().numpy().astype(np.complex128))
    note("autotune %s %d: rel_l2 vs default %.2e, equal %s"
         % (kind, n, err, torch.equal(before, after)))
    assert err <= 1e-6


@pytest.mark.parametrize("n,kind", [(2048, "asm"), (1024, "fresnel"), (2048, "fresnel"),
                                    (4096, "asm")])
def test_every_schedule_gives_the_default_result(ctx, n, kind):
    """Every candidate schedule of a single plane (row-major with each row-pass form, tiled
    with each column form), installed with cwo_set_tuning, gives the default schedule's
    result: the schedules move the same arithmetic through different layouts and launch
    shapes; the split column form (two half-length transforms per column) is a different
    factorisation of the same transform, so the bar is 1e-6 relative, not bit equality."""
    import numpy as np
    import torch
    from oracle import diffraction as D
    u = torch.from_numpy(W.uniform_random_field(n, 160 + n)).cuda()
    fn = ctx.asm if kind == "asm" else ctx.fresnel
    ctx.set_tuning(n, n, kind=kind, clear=True)
    ref = fn(u, 8e-6, 8e-6, 532e-9, 0.4)
    torch.cuda.synchronize()
    ref_np = ref.cpu().numpy().astype(np.complex128)
    scheds = [(1, 1, 0), (1, 2, 0)]
    scheds += [(2, 0, 1), (2, 0, 2)] if n >= 2048 else [(2, 0, 0)]
    try:
        for layout, form, col_form in scheds:
            ctx.set_tuning(n, n, kind=kind, row_form=form, layout=layout, col_form=col_form)
            y = fn(u, 8e-6, 8e-6, 532e-9, 0.4)
            torch.cuda.synchronize()
            err = D.rel_l2(y.cpu().numpy(), ref_np)
            note("%s %d layout=%d row_form=%d col_form=%d: rel_l2 vs default %.2e, equal %s"
                 % (kind, n, layout, form, col_form, err, torch.equal(y, ref)))
            assert err <= 1e-6
    finally:
        ctx.set_tuning(n, n, kind=kind, clear=True)


def test_column_form_validation(ctx):
    """A column form other than the default needs the tiled plane with padded columns of 4096
    or 8192; elsewhere cwo_set_tuning refuses it."""
    from paper_1107_5578_amd import cwo
    with pytest.raises(cwo.CwoError) as e:
        ctx.set_tuning(512, 512, col_form=2)              # row-major plane
    assert e.value.status == cwo.CWO_ERR_UNSUPPORTED
    with pytest.raises(cwo.CwoError) as e:
        ctx.set_tuning(2048, 2048, layout=1, col_form=1)  # row-major forced
    assert e.value.status == cwo.CWO_ERR_UNSUPPORTED
    with pytest.raises(cwo.CwoError) as e:
        ctx.set_tuning(2048, 2048, col_form=3)
    assert e.value.status == cwo.CWO_ERR_INVALID
    ctx.set_tuning(2048, 2048, col_form=2)                # default (tiled) plane: accepted
    ctx.set_tuning(2048, 2048, clear=True)


def test_tune_cache_round_trip(tmp_path, monkeypatch):
    """CWO_TUNE_CACHE: an autotuned schedule is written to the file and a new context loads
    it (installed schedules are what later calls use)."""
    import json
    import torch
    from paper_1107_5578_amd import cwo
    path = tmp_path / "tune.json"
    monkeypatch.setenv("CWO_TUNE_CACHE", str(path))
    u = torch.from_numpy(W.uniform_random_field(1024, 7)).cuda()
    c1 = cwo.Context(0)
    try:
        form, zchunk, us, layout, col_form = c1.autotune(u, 1, 8e-6, 8e-6, 532e-9, 0.2)
    finally:
        c1.close()
    entries = json.loads(path.read_text())
    mine = [e for e in entries if e["nx"] == 1024 and e["nz"] == 1 and e["kind"] == cwo.ANGULAR]
    assert len(mine) == 1
    assert (mine[0]["row_form"], mine[0]["zchunk"], mine[0]["layout"],
            mine[0]["col_form"]) == (form, zchunk, layout, col_form)
    # a second context reads the file: a forced schedule written there is used and kept
    mine[0]["layout"], mine[0]["row_form"] = 1, 2
    path.write_text("[\n" + ",\n".join(" " + json.dumps(e) for e in entries) + "\n]\n")
    c2 = cwo.Context(0)
    try:
        # autotuning another parameter set rewrites the file with both schedules
        c2.autotune(torch.from_numpy(W.uniform_random_field(256, 8)).cuda(), 1, 8e-6, 8e-6,
                    532e-9, 0.2)
    finally:
        c2.close()
    entries = json.loads(path.read_text())
    kept = [e for e in entries if e["nx"] == 1024 and e["nz"] == 1 and e["kind"] == cwo.ANGULAR]
    assert (kept[0]["layout"], kept[0]["row_form"]) == (1, 2)
    assert any(e["nx"] == 256 for e in entries)


def test_autotune_zstack(ctx):
    import torch
    cfg = W.ZSTACK_1024
    u = torch.from_numpy(W.field_for(cfg)).cuda()
    zs = list(W.zstack_distances(64, 0.05, 0.2))
    before = ctx.zstack(u, zs, cfg.pitch, cfg.pitch, cfg.wavelength)
    torch.cuda.synchronize()
    form, zchunk, us, _, _ = ctx.autotune(u, 64, cfg.pitch, cfg.pitch, cfg.wavelength, 0.1)
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

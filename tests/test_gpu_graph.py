"""The propagation calls captured into a HIP graph (torch.cuda.CUDAGraph) and replayed.

After one call with the same parameters has allocated the context's scratch and tables,
a call enqueues kernels only, so it can be captured. Each replay is checked bit for bit
against an eager call on the replay's input, with other eager work on the device
between the replays."""
import sys

import numpy as np
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


def fields(n, count, seed):
    import torch
    return [torch.from_numpy(W.uniform_random_field(n, seed + k)).cuda() for k in range(count)]


@pytest.mark.parametrize("kind,n", [("asm", 512), ("fresnel", 256), ("asm", 2048)])
def test_plain_call_graph_replay(ctx, kind, n):
    import torch
    note("graph %s %d" % (kind, n))
    fn = ctx.asm if kind == "asm" else ctx.fresnel
    src = fields(n, 4, 900)
    u = src[0].clone()
    out = torch.empty_like(u)
    fn(u, 8e-6, 8e-6, 532e-9, 0.2, out=out)  # allocates scratch and tables
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn(u, 8e-6, 8e-6, 532e-9, 0.2, out=out)
    other = fields(n, 1, 77)[0]
    for rep, f in enumerate(src):
        u.copy_(f)
        g.replay()
        fn(other, 8e-6, 8e-6, 532e-9, 0.3)  # eager work between replays
        torch.cuda.synchronize()
        ref = fn(f, 8e-6, 8e-6, 532e-9, 0.2)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep


def test_zstack_graph_replay(ctx):
    import torch
    n = 512
    zs = list(W.zstack_distances(16, 0.05, 0.2))
    src = fields(n, 3, 910)
    u = src[0].clone()
    out = torch.empty((len(zs), n, n), dtype=torch.complex64, device="cuda")
    ctx.zstack(u, zs, 4e-6, 4e-6, 633e-9, out=out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.zstack(u, zs, 4e-6, 4e-6, 633e-9, out=out)
    for rep, f in enumerate(src):
        u.copy_(f)
        g.replay()
        ctx.asm(f, 4e-6, 4e-6, 633e-9, 0.1)
        torch.cuda.synchronize()
        ref = ctx.zstack(f, zs, 4e-6, 4e-6, 633e-9)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep


def test_batch_graph_replay(ctx):
    import torch
    n = 256
    ins = fields(n, 8, 920)
    outs = [torch.empty_like(f) for f in ins]
    kw = dict(dx=8e-6, dy=8e-6, wavelength=532e-9, z=0.1)
    jobs = [("asm", f, o, kw) for f, o in zip(ins, outs)]
    ctx.batch(jobs)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.batch(jobs)
    for rep in range(3):
        for f in ins:
            f.mul_(1.5)
        g.replay()
        torch.cuda.synchronize()
        for f, o in zip(ins, outs):
            assert torch.equal(o, ctx.asm(f, 8e-6, 8e-6, 532e-9, 0.1)), rep


def test_point_light_source_and_fused_intensity_graph_replay(ctx):
    """The hologram sum and the fused-intensity propagation captured and replayed: each
    replay equals an eager call on the replay's inputs (eager calls between replays use no
    more points and no larger plane, so the captured scratch stays in place)."""
    import torch
    n, count = 256, 700
    clouds = [torch.from_numpy(W.pls_points(count, 950 + k, half_extent=2e-4)).cuda()
              for k in range(3)]
    pts = clouds[0].clone()
    holo = torch.empty((n, n), dtype=torch.float32, device="cuda")
    src = fields(n, 3, 960)
    u = src[0].clone()
    inten = torch.empty((n, n), dtype=torch.float32, device="cuda")
    args = (n, n, 4e-6, 4e-6, 633e-9, 1e-4, 0.0, 0.1)
    ctx.pls_cgh(pts, *args, out=holo)
    ctx.asm_intensity(u, 8e-6, 8e-6, 532e-9, 0.2, out=inten)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.pls_cgh(pts, *args, out=holo)
        ctx.asm_intensity(u, 8e-6, 8e-6, 532e-9, 0.2, out=inten)
    for rep in range(3):
        pts.copy_(clouds[rep])
        u.copy_(src[rep])
        g.replay()
        ctx.pls_cgh(clouds[(rep + 1) % 3][: count // 2].contiguous(), *args)  # eager, fewer points
        ctx.asm(src[(rep + 1) % 3], 8e-6, 8e-6, 532e-9, 0.3)
        torch.cuda.synchronize()
        ref_h = ctx.pls_cgh(clouds[rep], *args)
        ref_i = ctx.asm_intensity(src[rep], 8e-6, 8e-6, 532e-9, 0.2)
        torch.cuda.synchronize()
        assert torch.equal(holo, ref_h), rep
        assert torch.equal(inten, ref_i), rep

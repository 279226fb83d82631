"""GPU test of cwo_asm_noalloc, the entry point that allocates no device memory.

It runs the same kernels as cwo_asm with its scratch in a static device array, so its
output must equal cwo_asm's bit for bit. Two calls in a row, the second on a smaller
field, check that what the first call left in the shared array does not leak into the
second; one result is also checked against the FP64 oracle.
"""
import sys

import numpy as np
import pytest

from oracle import diffraction as D
from paper_1107_5578_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    return t


def note(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def test_noalloc_matches_cwo_asm(torch):
    from paper_1107_5578_amd import cwo
    ctx = cwo.Context(0)
    try:
        cases = [(2048, 2048, 8e-6, 532e-9, 0.5, 21), (256, 512, 10e-6, 633e-9, 0.1, 22)]
        for nx, ny, pitch, lam, z, seed in cases:
            note("noalloc %dx%d" % (nx, ny))
            u_np = W.uniform_random_field(nx, seed, ny=ny)
            u = torch.from_numpy(u_np).cuda()
            out = torch.empty_like(u)
            ref = torch.empty_like(u)
            ctx.asm_noalloc(u, pitch, pitch, lam, z, out=out)
            ctx.asm(u, pitch, pitch, lam, z, out=ref)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), "noalloc differs from cwo_asm at %dx%d" % (nx, ny)
        # the second (smaller) call against the oracle as well
        err = D.rel_l2(out.cpu().numpy(), D.asm(u_np, pitch, pitch, lam, z))
        note("  rel_l2 vs oracle %.3e" % err)
        assert err <= 1e-5
    finally:
        ctx.close()


def test_noalloc_limits(torch):
    from paper_1107_5578_amd import cwo
    ctx = cwo.Context(0)
    try:
        big = torch.zeros((4096, 4096), dtype=torch.complex64, device="cuda")
        with pytest.raises(cwo.CwoError) as e:
            ctx.asm_noalloc(big, 8e-6, out=torch.empty_like(big))
        assert e.value.status == cwo.CWO_ERR_NOMEM
        small = torch.zeros((64, 64), dtype=torch.complex64, device="cuda")
        p = cwo.make_params(64, 64, 8e-6, precision="f16")
        import ctypes
        st = cwo.load().cwo_asm_noalloc(ctx.handle, ctypes.byref(p),
                                        ctypes.c_void_p(small.data_ptr()),
                                        ctypes.c_void_p(small.data_ptr()), ctypes.c_void_p(0))
        assert st == cwo.CWO_ERR_UNSUPPORTED
    finally:
        ctx.close()

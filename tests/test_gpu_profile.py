"""Stage timing (cwo_profile): every stage of a plain propagation is timed once per call by
a pair of events that the runtime stamps from the stage's own kernels. The stage times are
positive and together fit inside the event-timed wall time of the same calls, so no stage
is counted twice and no gap between kernels is charged to a stage."""
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_stage_times_fit_the_calls():
    import torch
    from paper_1107_5578_amd import cwo, workloads as W
    ctx = cwo.Context(0)
    try:
        print("[gpu-case] stage timing, 1024^2 ASM, 20 calls", flush=True)
        sys.stdout.flush()
        u = torch.from_numpy(W.uniform_random_field(1024, 77)).cuda()
        out = torch.empty_like(u)
        for _ in range(3):
            ctx.asm(u, 8e-6, 8e-6, 532e-9, 0.2, out=out)
        torch.cuda.synchronize()
        n = 20
        stream = torch.cuda.current_stream()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        ctx.profile(True)
        start.record(stream)
        for _ in range(n):
            ctx.asm(u, 8e-6, 8e-6, 532e-9, 0.2, out=out)
        stop.record(stream)
        torch.cuda.synchronize()
        wall = start.elapsed_time(stop)
        total = 0.0
        for st in (cwo.STAGE_ROW_FWD, cwo.STAGE_COL, cwo.STAGE_ROW_INV):
            ms, cnt = ctx.profile_read(st)
            assert cnt == n, (cwo.STAGE_NAMES[st], cnt)
            assert ms > 0.0, cwo.STAGE_NAMES[st]
            total += ms
        ctx.profile(False)
        assert total <= wall * 1.02, (total, wall)
    finally:
        ctx.close()

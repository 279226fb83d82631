"""GPU tests of the serving loop (cwo_submit / cwo_poll, continuous batching).

The key property: each result is the same alone and in the mix. Every request of a
mixed stream (sizes, kinds, distances, wavelengths, same-field groups) is also run on
its own through the synchronous call, and the two outputs must agree to relative L2
<= 1e-6 (the serving slots run the same kernels; only z-stack grouping may change the
rounding order). Admission by memory and the error paths are checked too.
"""
import sys
import time

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


def test_alone_vs_mix(torch):
    from paper_1107_5578_amd import cwo
    rng = np.random.default_rng(55)
    server = cwo.Context(0, hbm_budget_bytes=256 << 20)
    alone = cwo.Context(0)
    try:
        fields = {n: torch.from_numpy(W.uniform_random_field(n, 7000 + n)).cuda()
                  for n in (64, 128, 256, 512, 1024)}
        reqs = []
        for i in range(40):
            n = int(rng.choice([64, 128, 256, 512, 1024]))
            kind = "asm" if rng.random() < 0.5 else "fresnel"
            kw = dict(dx=8e-6, wavelength=float(rng.choice([473e-9, 532e-9, 633e-9])),
                      z=float(rng.uniform(0.01, 1.0)))
            reqs.append((kind, fields[n], kw))
        # two requests on the same field back to back form a z-stack inside one batch
        reqs.insert(5, ("asm", fields[256], dict(dx=8e-6, wavelength=532e-9, z=0.2)))
        reqs.insert(6, ("asm", fields[256], dict(dx=8e-6, wavelength=532e-9, z=0.3)))
        outs = [torch.empty_like(u) for _, u, _ in reqs]
        note("serving %d mixed requests" % len(reqs))
        tickets = [server.submit(kind, u, o, **kw) for (kind, u, kw), o in zip(reqs, outs)]
        server.drain()
        worst = 0.0
        for t, (kind, u, kw), o in zip(tickets, reqs, outs):
            assert server.poll(t) == cwo.DONE
            inf = server.info(t)
            assert inf["t_submit"] <= inf["t_start"] <= inf["t_done"]
            ref = (alone.asm if kind == "asm" else alone.fresnel)(u, kw["dx"], kw["dx"],
                                                                   kw["wavelength"], kw["z"])
            torch.cuda.synchronize()
            worst = max(worst, D.rel_l2(o.cpu().numpy(), ref.cpu().numpy().astype(np.complex128)))
            server.release(t)
        note("alone vs mix: worst rel_l2 = %.3e" % worst)
        assert worst <= 1e-6
        # and one request of the mix against the FP64 oracle
        kind, u, kw = reqs[-1]
        ref = D.propagate(u.cpu().numpy(), D.ASM if kind == "asm" else D.FRESNEL, kw["dx"], kw["dx"],
                          kw["wavelength"], kw["z"])
        assert D.rel_l2(outs[-1].cpu().numpy(), ref) <= 1e-5
    finally:
        server.close()
        alone.close()


def test_alone_vs_mix_serving_sizes(torch):
    """The serving workload's sizes (512^2 ... 4096^2), each request with its own seeded field
    (seed 5000 + i), ASM and Fresnel, random z and wavelength, plus an FP16-storage pair on
    one field (16-bit requests never form a z-stack, so each must equal its own call)."""
    from paper_1107_5578_amd import cwo
    reqs = W.serving_requests(16, 1.0, seed=5, sizes=(512, 1024, 2048, 4096))
    sizes = (512, 1024, 2048, 4096)
    server = cwo.Context(0, hbm_budget_bytes=6 << 30)
    alone = cwo.Context(0)
    try:
        jobs = []
        for i, r in enumerate(reqs):
            # the request mix's kinds, distances and wavelengths, every size four times
            n = sizes[i % 4]
            u = torch.from_numpy(W.uniform_random_field(n, 5000 + i)).cuda()
            jobs.append((r.kind, u, dict(dx=r.pitch, wavelength=r.wavelength, z=r.z), "f32"))
        u16 = torch.from_numpy(W.uniform_random_field(1024, 4999)).cuda()
        for z in (0.3, 0.5):
            jobs.append(("asm", u16, dict(dx=8e-6, wavelength=532e-9, z=z), "f16"))
        outs = [torch.empty_like(u) for _, u, _, _ in jobs]
        note("serving %d requests of sizes %s" % (len(jobs), sizes))
        tickets = [server.submit(k, u, o, precision=pr, **kw)
                   for (k, u, kw, pr), o in zip(jobs, outs)]
        server.drain()
        checked = set()
        for t, (kind, u, kw, pr), o in zip(tickets, jobs, outs):
            assert server.poll(t) == cwo.DONE
            fn = alone.asm if kind == "asm" else alone.fresnel
            ref = fn(u, kw["dx"], kw["dx"], kw["wavelength"], kw["z"], precision=pr)
            torch.cuda.synchronize()
            err = D.rel_l2(o.cpu().numpy(), ref.cpu().numpy().astype(np.complex128))
            assert err <= 1e-6, (u.shape, kind, pr, err)
            n = u.shape[0]
            if pr == "f32" and n not in checked:
                # one request per size against the FP64 oracle
                note("oracle check %s %d^2" % (kind, n))
                ora = D.propagate(u.cpu().numpy(), D.ASM if kind == "asm" else D.FRESNEL,
                                  kw["dx"], kw["dx"], kw["wavelength"], kw["z"])
                e2 = D.rel_l2(o.cpu().numpy(), ora)
                note("  rel_l2 = %.3e" % e2)
                assert e2 <= 1e-5
                checked.add(n)
        assert checked == {512, 1024, 2048, 4096}
        assert server.memory_held() <= 6 << 30
    finally:
        server.close()
        alone.close()


def test_window_batches_one_geometry(torch):
    """With every slot busy (four 4096^2 requests of different pitches, one per slot),
    interleaved requests of two sizes queue up; a freed slot takes the head request and the
    queued requests of its geometry as one batch, so requests of one size share a few start
    times, and every result equals its synchronous call."""
    from paper_1107_5578_amd import cwo
    server = cwo.Context(0, hbm_budget_bytes=8 << 30)
    alone = cwo.Context(0)
    try:
        big = torch.from_numpy(W.uniform_random_field(4096, 31)).cuda()
        bouts = [torch.empty_like(big) for _ in range(4)]
        reqs = []
        for k in range(8):
            for n in (256, 512):
                u = torch.from_numpy(W.uniform_random_field(n, 9100 + 10 * n + k)).cuda()
                kind = "asm" if k % 3 else "fresnel"
                reqs.append((kind, u, dict(dx=8e-6, wavelength=532e-9, z=0.05 + 0.01 * k)))
        outs = [torch.empty_like(u) for _, u, _ in reqs]
        torch.cuda.synchronize()
        note("serving 4 blockers and %d interleaved 256^2 / 512^2 requests" % len(reqs))
        bt = [server.submit("asm", big, o, dx=p, wavelength=532e-9, z=0.3)
              for o, p in zip(bouts, (8e-6, 9e-6, 10e-6, 11e-6))]
        tickets = [server.submit(kind, u, o, **kw) for (kind, u, kw), o in zip(reqs, outs)]
        server.drain()
        for t in bt:
            assert server.poll(t) == cwo.DONE
        starts = {256: set(), 512: set()}
        for t, (kind, u, kw), o in zip(tickets, reqs, outs):
            assert server.poll(t) == cwo.DONE
            starts[u.shape[0]].add(server.info(t)["t_start"])
            fn = alone.asm if kind == "asm" else alone.fresnel
            ref = fn(u, kw["dx"], kw["dx"], kw["wavelength"], kw["z"])
            torch.cuda.synchronize()
            err = D.rel_l2(o.cpu().numpy(), ref.cpu().numpy().astype(np.complex128))
            assert err <= 1e-6, (u.shape, kind, err)
        note("distinct start times per size: %s" % {n: len(v) for n, v in starts.items()})
        # eight requests per size; at most eight per batch
        assert len(starts[256]) <= 3 and len(starts[512]) <= 3, starts
    finally:
        server.close()
        alone.close()


def test_memory_held_within_budget(torch):
    """Held device memory never exceeds the budget: 4096^2 requests (each 512 MiB of fields
    and scratch) and then 512^2 requests through a 1.25 GiB budget; idle slots give their
    4096^2 scratch back when memory is short."""
    from paper_1107_5578_amd import cwo
    budget = 1280 << 20
    server = cwo.Context(0, hbm_budget_bytes=budget)
    try:
        big = torch.from_numpy(W.uniform_random_field(4096, 61)).cuda()
        small = torch.from_numpy(W.uniform_random_field(512, 62)).cuda()
        outs_b = [torch.empty_like(big) for _ in range(3)]
        outs_s = [torch.empty_like(small) for _ in range(24)]
        tickets = [server.submit("asm", big, o, dx=8e-6, wavelength=532e-9, z=0.2 + 0.1 * i)
                   for i, o in enumerate(outs_b)]
        tickets += [server.submit("fresnel" if i % 2 else "asm", small, o, dx=8e-6,
                                  wavelength=633e-9, z=0.05 + 0.01 * i)
                    for i, o in enumerate(outs_s)]
        peak = 0
        deadline = time.time() + 120
        while time.time() < deadline:
            peak = max(peak, server.memory_held())
            if all(server.poll(t) >= cwo.DONE or server.poll(t) < 0 for t in tickets):
                break
            time.sleep(0.0005)
        server.drain()
        peak = max(peak, server.memory_held())
        note("peak held %.1f MiB of a %.1f MiB budget" % (peak / 2**20, budget / 2**20))
        assert all(server.poll(t) == cwo.DONE for t in tickets)
        assert peak <= budget
        # results are right after the slots traded their scratch
        ref = D.asm(small.cpu().numpy(), 8e-6, 8e-6, 633e-9, 0.05 + 0.01 * 22)
        assert D.rel_l2(outs_s[22].cpu().numpy(), ref) <= 1e-5
    finally:
        server.close()


def test_submit_orders_after_producer_stream(torch):
    """A field written by asynchronous kernels on the caller's stream just before submit is
    read only after they finish (cwo_submit_after, what Context.submit uses)."""
    from paper_1107_5578_amd import cwo
    server = cwo.Context(0)
    alone = cwo.Context(0)
    try:
        n = 1024
        base = torch.from_numpy(W.uniform_random_field(n, 71)).cuda()
        torch.cuda.synchronize()
        outs, fields = [], []
        for k in range(6):
            # a long chain of elementwise kernels on the current stream, then submit at once
            u = base.clone()
            for _ in range(40):
                u = u * torch.exp(torch.tensor(0.05j, dtype=torch.complex64, device="cuda"))
            fields.append(u)
            o = torch.empty_like(u)
            outs.append(o)
            server.submit("asm", u, o, dx=8e-6, wavelength=532e-9, z=0.1 + 0.05 * k)
        server.drain()
        for k, (u, o) in enumerate(zip(fields, outs)):
            ref = alone.asm(u, 8e-6, 8e-6, 532e-9, 0.1 + 0.05 * k)
            torch.cuda.synchronize()
            assert D.rel_l2(o.cpu().numpy(), ref.cpu().numpy().astype(np.complex128)) <= 1e-6
    finally:
        server.close()
        alone.close()


def test_admission_by_memory(torch):
    from paper_1107_5578_amd import cwo
    n = 512
    fp = 16 * n * n + 8 * n * 2 * n
    server = cwo.Context(0, hbm_budget_bytes=2 * fp)   # at most two requests resident at once
    try:
        u = torch.from_numpy(W.uniform_random_field(n, 3)).cuda()
        outs = [torch.empty_like(u) for _ in range(12)]
        tickets = [server.submit("asm", u, o, dx=8e-6, wavelength=532e-9, z=0.1 + 0.01 * i)
                   for i, o in enumerate(outs)]
        seen_running = 0
        deadline = time.time() + 60
        while time.time() < deadline:
            states = [server.poll(t) for t in tickets]
            seen_running = max(seen_running, sum(1 for s in states if s == cwo.RUNNING))
            if all(s == cwo.DONE for s in states):
                break
            time.sleep(0.0005)
        server.drain()
        assert all(server.poll(t) == cwo.DONE for t in tickets)
        assert seen_running <= 2
        infos = [server.info(t) for t in tickets]
        assert all(i["footprint"] == fp for i in infos)
        # FIFO admission: starts are in submission order
        starts = [i["t_start"] for i in infos]
        assert starts == sorted(starts)
        big = torch.zeros((1024, 1024), dtype=torch.complex64, device="cuda")
        with pytest.raises(cwo.CwoError) as e:
            server.submit("asm", big, torch.empty_like(big), z=0.1)
        assert e.value.status == cwo.CWO_ERR_NOMEM
        ref = D.asm(u.cpu().numpy(), 8e-6, 8e-6, 532e-9, 0.1 + 0.01 * 11)
        assert D.rel_l2(outs[11].cpu().numpy(), ref) <= 1e-5
    finally:
        server.close()


def test_ticket_errors(torch):
    from paper_1107_5578_amd import cwo
    server = cwo.Context(0)
    try:
        with pytest.raises(cwo.CwoError) as e:
            server.poll(12345)
        assert e.value.status == cwo.CWO_ERR_NOTFOUND
        u = torch.zeros((64, 64), dtype=torch.complex64, device="cuda")
        with pytest.raises(cwo.CwoError) as e:
            server.submit("fresnel", u, torch.empty_like(u), z=0.0)
        assert e.value.status == cwo.CWO_ERR_INVALID
        t = server.submit("asm", u, torch.empty_like(u), z=0.1)
        server.drain()
        server.release(t)
        with pytest.raises(cwo.CwoError) as e:
            server.release(t)
        assert e.value.status == cwo.CWO_ERR_NOTFOUND
    finally:
        server.close()

"""Benchmark of the diffraction hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]

One step = one angular-spectrum propagation of the 2048 x 2048 complex64 field
(0/1 rectangles with random phase, 8 um pitch, 532 nm, z = 0.5 m), zero-padded to
4096 x 4096, FP32: row FFT with padding, column FFT x H x IFFT, row IFFT with crop,
through the C ABI (cwo_asm). The input is resident in HBM before timing starts.

Prints one JSON line: throughput in planes/s over K timed steps (HIP events on the
launch stream, bracketed by device synchronisation), the per-kernel durations
measured live with HIP events inside the timed region, the roofline figure of the
dominant kernel, the relative L2 error of the result against the FP64 oracle, and
the oracle's own throughput on the host cores (a bounded sample: whole planes).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# vector issue: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4 clocks (one per
# clock per CU) at 2.4 GHz
VALU_PEAK_GWAVE = 256 * 2.4

# algorithmic bytes per launch of each kernel for an N x N field, M = 2N, complex64
# intermediates: row_fwd reads the field and writes the N x M spectrum rows; col reads
# and writes the N x M plane in place; row_inv reads it and writes the field.
def stage_bytes(n: int, elem: int = 8) -> dict:
    field = 8 * n * n
    plane = elem * n * (2 * n)
    return {"row_fwd": field + plane, "col": 2 * plane, "row_inv": plane + field}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in ("paper_1107_5578_amd/csrc/plane.hip", "paper_1107_5578_amd/csrc/column.hip",
                "paper_1107_5578_amd/csrc/column.hpp",
                "paper_1107_5578_amd/csrc/kernel_common.hpp",
                "paper_1107_5578_amd/csrc/fft_device.hpp", "paper_1107_5578_amd/csrc/launch.hpp",
                "paper_1107_5578_amd/csrc/rowsplit.hpp"):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_record(kernel: str):
    """The committed rocprofv3 counter record of a kernel of the 2048^2 plane, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_asm2048.json" % kernel)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec


def committed_traffic(kernel: str):
    """HBM bytes per launch from the committed counter record, or None."""
    rec = committed_record(kernel)
    return rec.get("bytes_per_launch") if rec else None


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(u_np, cfg, kind="asm", min_seconds: float = 10.0, max_planes: int = 30,
                 single_seconds: float = 8.0):
    """The FP64 oracle on the host cores, on whole planes of the same workload: first with
    every OpenMP thread, then (a shorter sample) with one thread."""
    from oracle import _native, diffraction as D
    threads = _native.max_threads()

    def sample(limit_s, max_n):
        t0 = time.perf_counter()
        ref, done = None, 0
        for _ in range(max_n):
            ref = D.propagate(u_np, kind, cfg.pitch, cfg.pitch, cfg.wavelength, cfg.z)
            done += 1
            if time.perf_counter() - t0 > limit_s:
                break
        return ref, done, time.perf_counter() - t0

    ref, done, dt = sample(min_seconds, max_planes)
    # one OpenMP thread from here on (the oracle keeps the setting of its last call)
    _native.fft2(np.zeros((16, 16), dtype=np.complex128), threads=1)
    _, done1, dt1 = sample(single_seconds, 4)
    _native.fft2(np.zeros((16, 16), dtype=np.complex128), threads=threads)
    return ref, {"value": done / dt, "unit": "planes/s", "cores": threads, "kind": "oracle",
                 "cpu_model": host_cpu_model(),
                 "sample": "%d whole %dx%d %s plane(s) of the timed workload, FP64, "
                           "%d OpenMP threads for the FFTs (%.1f s)"
                           % (done, u_np.shape[1], u_np.shape[0], kind, threads, dt),
                 "single_thread": {"value": done1 / dt1, "unit": "planes/s",
                                   "sample": "%d whole plane(s), 1 thread (%.1f s)" % (done1, dt1)}}


def time_zstack(ctx, torch, u, zs, pitch, lam, reps, warm, precision="f32"):
    """Planes/s of one z-stack call (all planes) over `reps` calls, HIP events."""
    out = torch.empty((len(zs),) + tuple(u.shape), dtype=torch.complex64, device=u.device)
    for _ in range(warm):
        ctx.zstack(u, zs, pitch, pitch, lam, kind="asm", out=out, precision=precision)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(u.device)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        ctx.zstack(u, zs, pitch, pitch, lam, kind="asm", out=out, precision=precision)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del out
    return len(zs) * 1000.0 / ms, ms


def time_call(torch, stream, fn, reps, warm):
    """Milliseconds per call of fn over `reps` calls, HIP events on the launch stream."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def other_forms(ctx, torch, W, u, u_np, cfg, stream, with_oracle):
    """The other diffraction forms and the epilogues on the same 2048^2 field: planes/s,
    algorithmic bytes and GB/s (and the error against the oracle when it is run)."""
    n = u.shape[0]
    res = {}
    out = torch.empty_like(u)

    def rec(name, ms, alg_bytes, extra=None):
        r = {"ms": round(ms, 4), "planes_per_s": round(1000.0 / ms, 1), "alg_bytes": alg_bytes,
             "GBps": round(alg_bytes / (ms * 1e-3) / 1e9, 1)}
        r.update(extra or {})
        res[name] = r

    # shifted angular spectrum, band-limited, far beyond the critical distance
    z_bl = 3.0
    from paper_1107_5578_amd import cwo
    wx, wy = cwo.band_limit(n, n, cfg.pitch, cfg.pitch, cfg.wavelength, z_bl)
    sh = (1.2e-3, -0.4e-3, 0.0, wx, 0.0, wy)
    ms = time_call(torch, stream, lambda: ctx.asm_shifted(u, cfg.pitch, cfg.pitch, cfg.wavelength,
                                                          z_bl, *sh, out=out), 50, 5)
    extra = {"z_m": z_bl, "offset_m": [sh[0], sh[1]], "band_width_per_m": [wx, wy]}
    if with_oracle:
        from oracle import shifted_asm as S
        ref = S.propagate(u_np, cfg.pitch, cfg.pitch, cfg.wavelength, z_bl, *sh)
        extra["rel_l2_vs_oracle"] = float("%.3e" % rel_l2(out.cpu().numpy(), ref))
    rec("asm_shifted", ms, 80 * n * n, extra)

    # Fresnel, Fourier form: one unpadded FFT, in place on the output plane
    ms = time_call(torch, stream, lambda: ctx.fresnel_fourier(u, cfg.pitch, cfg.pitch,
                                                              cfg.wavelength, cfg.z, out=out), 100, 5)
    extra = {"z_m": cfg.z}
    if with_oracle:
        from oracle import fresnel_fourier as F
        ref = F.propagate(u_np, cfg.pitch, cfg.pitch, cfg.wavelength, cfg.z)
        extra["rel_l2_vs_oracle"] = float("%.3e" % rel_l2(out.cpu().numpy(), ref))
    rec("fresnel_fourier", ms, 32 * n * n, extra)

    # shifted Fresnel: destination pitch 1.5x, window moved off axis
    p1 = 1.5 * cfg.pitch
    offs = (0.0, 0.0, 2.0e-3, -1.0e-3)
    ms = time_call(torch, stream, lambda: ctx.fresnel_shifted(u, cfg.pitch, cfg.pitch, p1, p1,
                                                              cfg.wavelength, cfg.z, *offs, out=out),
                   50, 5)
    extra = {"z_m": cfg.z, "dst_pitch_m": p1, "dst_centre_m": [offs[2], offs[3]]}
    if with_oracle:
        from oracle import shifted_fresnel as SF
        rows = [0, n // 3, n // 2, n - 1]
        ref = SF.propagate(u_np, cfg.pitch, cfg.pitch, p1, p1, cfg.wavelength, cfg.z, *offs,
                           rows=rows)
        extra["rel_l2_vs_oracle_rows"] = float("%.3e" % rel_l2(out.cpu().numpy()[rows], ref))
    rec("fresnel_shifted", ms, 80 * n * n, extra)

    # epilogues on the propagated plane: intensity, then the 8-bit min-max image
    def epi():
        i = ctx.intensity(out)
        return ctx.scale(i, 255.0, u8=True)

    ms = time_call(torch, stream, epi, 100, 5)
    rec("intensity_scale_u8", ms, 21 * n * n)

    # intensity fused into the last pass vs a propagation followed by the epilogue
    inten = torch.empty((n, n), dtype=torch.float32, device=u.device)
    ms_f = time_call(torch, stream, lambda: ctx.asm_intensity(u, cfg.pitch, cfg.pitch,
                                                              cfg.wavelength, cfg.z, out=inten),
                     100, 5)
    ms_s = time_call(torch, stream, lambda: ctx.intensity(ctx.asm(u, cfg.pitch, cfg.pitch,
                                                                  cfg.wavelength, cfg.z, out=out)),
                     100, 5)
    rec("asm_intensity_fused", ms_f, 76 * n * n,
        {"separate_ms": round(ms_s, 4), "fused_vs_separate": round(ms_s / ms_f, 3)})

    # point-light-source hologram (direct sum, arithmetic-bound): the paper's hologram
    # geometry and point counts, synthetic point clouds
    pc = W.PLS_2048
    pls = {"workload": "%dx%d hologram, %g um pitch, %g nm, object offset (%g, %g, %g) m, "
                       "synthetic points in a +-4 mm cube" % (pc.n, pc.n, pc.pitch * 1e6,
                                                             pc.wavelength * 1e9, pc.ox, pc.oy,
                                                             pc.oz)}
    for count in pc.counts:
        pts_np = W.pls_points(count, 7)
        pts = torch.from_numpy(pts_np).to(u.device)
        h = torch.empty((pc.n, pc.n), dtype=torch.float32, device=u.device)
        ms = time_call(torch, stream, lambda: ctx.pls_cgh(pts, pc.n, pc.n, pc.pitch, pc.pitch,
                                                          pc.wavelength, pc.ox, pc.oy, pc.oz,
                                                          out=h), 3 if count > 5000 else 10, 1)
        terms = count * pc.n * pc.n
        e = {"ms": round(ms, 3), "terms_per_s": float("%.4g" % (terms / (ms * 1e-3)))}
        if with_oracle:
            from oracle import pls as PL
            rows = [0, pc.n // 2]
            ref = PL.cgh(pts_np, pc.n, pc.n, pc.pitch, pc.pitch, pc.wavelength, pc.ox, pc.oy,
                         pc.oz, rows=rows)
            e["rel_l2_vs_oracle_rows"] = float("%.3e" % rel_l2(h.cpu().numpy()[rows], ref))
        pls[str(count)] = e
        del pts, h
    res["pls_cgh"] = pls
    return res


def rel_l2(y, ref):
    import numpy as np
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    return float(np.linalg.norm((y - ref).ravel()) / np.linalg.norm(ref.ravel()))


def serve_bench(ctx_cls, torch, W, dev, count, budget=8 << 30, rates=(0.5, 0.8, 0.95)):
    """Serving: a stream of mixed requests (sizes 512..4096^2, ASM/Fresnel 50/50,
    z ~ U[0.01, 1] m, wavelength in {473, 532, 633} nm, 8 um pitch) through cwo_submit /
    cwo_poll under an HBM budget. Every request reads a field of its own: 10k distinct
    fields do not fit, so each size has a ring of FIELD_RING distinct seeded fields and
    successive requests of one size take successive fields. A serving batch takes requests
    of one size, the oldest queued ones of that size, at most 8 of them (the library's
    default; CWO_SERVE_MAX_BATCH must stay unset or at most FIELD_RING), so no batch holds
    two requests on one field and none can be merged into a z-stack. Outputs rotate through
    a ring per size (a buffer is reused only after its previous request is done)."""
    FIELD_RING = 8
    reqs = W.serving_requests(count, 1.0, seed=5)
    sizes = sorted({r.n for r in reqs})
    fields = {n: [torch.from_numpy(W.uniform_random_field(n, 5000 + FIELD_RING * k + i)).to(dev)
                  for i in range(FIELD_RING)] for k, n in enumerate(sizes)}
    seq = {n: 0 for n in sizes}
    req_field = []
    for r in reqs:
        req_field.append(fields[r.n][seq[r.n] % FIELD_RING])
        seq[r.n] += 1
    ring = 40
    outs = {n: [torch.empty_like(fields[n][0]) for _ in range(ring)] for n in sizes}

    def run(arrivals):
        srv = ctx_cls(0, hbm_budget_bytes=budget)
        owner = {n: [None] * ring for n in sizes}
        used = {n: 0 for n in sizes}
        tickets = []
        t0 = time.perf_counter()
        for r, f, ta in zip(reqs, req_field, arrivals):
            if ta is not None:
                while time.perf_counter() - t0 < ta:
                    pass
            k = used[r.n] % ring
            used[r.n] += 1
            prev = owner[r.n][k]
            while prev is not None and srv.poll(prev) < 2:
                time.sleep(0.0001)
            t = srv.submit(r.kind, f, outs[r.n][k], dx=r.pitch, wavelength=r.wavelength, z=r.z)
            owner[r.n][k] = t
            tickets.append(t)
        srv.drain()
        infos = [srv.info(t) for t in tickets]
        srv.close()
        lat = np.array([i["t_done"] - i["t_submit"] for i in infos]) * 1e3
        span = max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)
        return {"requests": len(infos), "req_per_s": round(len(infos) / span, 1),
                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "mean_ms": round(float(lat.mean()), 3)}

    # plain per-call form on one stream, same requests in order (first 2000)
    plain_ctx = ctx_cls(0)
    nplain = min(2000, count)
    for r, f in zip(reqs[:8], req_field):
        (plain_ctx.asm if r.kind == "asm" else plain_ctx.fresnel)(
            f, r.pitch, r.pitch, r.wavelength, r.z, out=outs[r.n][0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r, f in zip(reqs[:nplain], req_field):
        (plain_ctx.asm if r.kind == "asm" else plain_ctx.fresnel)(
            f, r.pitch, r.pitch, r.wavelength, r.z, out=outs[r.n][0])
    torch.cuda.synchronize()
    plain_rps = nplain / (time.perf_counter() - t0)
    plain_ctx.close()

    closed = run([None] * count)
    cap = closed["req_per_s"]
    out = {"workload": "%d requests, sizes %s^2 uniform, ASM/Fresnel 50/50, z~U[0.01,1] m, "
                       "lambda in {473,532,633} nm, 8 um, HBM budget %d GiB, a ring of %d "
                       "distinct fields per size (no serving batch holds two requests on one "
                       "field)" % (count, "/".join(str(n) for n in sizes), budget >> 30,
                                   FIELD_RING),
           "plain_per_call_req_per_s": round(plain_rps, 1),
           "closed_loop": closed, "served_vs_plain": round(cap / plain_rps, 3), "open_loop": {}}
    for f in rates:
        rng = np.random.default_rng(5)
        gaps = rng.exponential(1.0 / (f * cap), size=count)
        arr = list(np.cumsum(gaps) - gaps[0])
        out["open_loop"]["%.2f" % f] = dict(run(arr), offered_req_per_s=round(f * cap, 1))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--settle-ms", type=float, default=250.0,
                    help="repeat the step for this wall time before the warm-up steps (0: none)")
    ap.add_argument("--kind", choices=["asm", "fresnel"], default="asm",
                    help="transfer function of the timed plane (the headline metric is asm)")
    ap.add_argument("--n", type=int, default=0,
                    help="field size other than the headline 2048 (a side measurement)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the z-stack (batched form) measurements")
    ap.add_argument("--precision", choices=["f32", "f16", "bf16"], default="f32",
                    help="storage of the padded planes (arithmetic is always FP32)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests in the serving measurement (0 skips it)")
    ap.add_argument("--no-gs", action="store_true",
                    help="skip the ping-pong (GS) iteration measurement")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the other diffraction forms and the epilogues")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this size three times (a plain copy "
                         "kernel of known traffic, to calibrate profiler byte counters)")
    ap.add_argument("--pls-points", type=int, default=0,
                    help="time only the point-light-source hologram of the 2048^2 geometry with "
                         "this many points (--steps calls after --warmup) and print one line")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(planes would shard across GPUs with no exchange; see the design notes). "
              "Run with --gpus 1.", file=sys.stderr, flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1107_5578_amd import cwo, workloads as W

    if args.pls_points > 0:
        pc = W.PLS_2048
        dev = torch.device("cuda:0")
        ctx = cwo.Context(0)
        stream = torch.cuda.current_stream(dev)
        pts = torch.from_numpy(W.pls_points(args.pls_points, 7)).to(dev)
        h = torch.empty((pc.n, pc.n), dtype=torch.float32, device=dev)
        ms = time_call(torch, stream, lambda: ctx.pls_cgh(pts, pc.n, pc.n, pc.pitch, pc.pitch,
                                                          pc.wavelength, pc.ox, pc.oy, pc.oz,
                                                          out=h), args.steps, args.warmup)
        terms = args.pls_points * pc.n * pc.n
        print(json.dumps({"metric": "PLS hologram terms/s at 2048^2", "points": args.pls_points,
                          "ms": round(ms, 4), "terms_per_s": float("%.4g" % (terms / (ms * 1e-3))),
                          "steps": args.steps, "warmup": args.warmup}), flush=True)
        ctx.close()
        return

    cfg = W.PLANE_2048
    n = args.n or cfg.n
    u_np = W.field_for(cfg, n)
    dev = torch.device("cuda:0")
    ctx = cwo.Context(0)
    u = torch.from_numpy(u_np).to(dev)
    out = torch.empty_like(u)
    stream = torch.cuda.current_stream(dev)

    prop = ctx.asm if args.kind == "asm" else ctx.fresnel

    def step():
        prop(u, cfg.pitch, cfg.pitch, cfg.wavelength, cfg.z, out=out, precision=args.precision)

    # settle: the same step repeated for a fixed wall time before the counted warm-up, so
    # that a short timed region measures the device in its steady (clocked-up) state
    if args.settle_ms > 0:
        t_end = time.perf_counter() + args.settle_ms * 1e-3
        while time.perf_counter() < t_end:
            for _ in range(8):
                step()
            torch.cuda.synchronize()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # the timed region: K steps, HIP events on the launch stream, device sync around it
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        step()
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    # the same K steps again with the library's per-kernel HIP events on that stream
    ctx.profile(True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        step()
    stop.record(stream)
    torch.cuda.synchronize()
    profiled_ms = start.elapsed_time(stop)
    kernels = {}
    for stage in (cwo.STAGE_ROW_FWD, cwo.STAGE_COL, cwo.STAGE_ROW_INV):
        ms, cnt = ctx.profile_read(stage)
        kernels[cwo.STAGE_NAMES[stage]] = {"avg_us": 1000.0 * ms / max(cnt, 1), "launches": cnt}
    ctx.profile(False)

    ms_per_step = total_ms / args.steps
    value = 1000.0 / ms_per_step

    sb = stage_bytes(n, 8 if args.precision == "f32" else 4)
    for name, rec in kernels.items():
        rec["alg_bytes"] = sb[name]
        rec["GBps"] = sb[name] / (rec["avg_us"] * 1e-6) / 1e9
    dominant = max(kernels, key=lambda k: kernels[k]["avg_us"])
    d = kernels[dominant]
    traffic = committed_traffic(dominant)
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(d["GBps"], 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(d["GBps"] / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "plane_alg_bytes": sum(sb.values()),
                "plane_GBps": round(sum(sb.values()) / (ms_per_step * 1e-3) / 1e9, 1)}
    # the same kernel against the vector-issue peak: its committed SQ_INSTS_VALU count per
    # launch (wave instructions, same source hash) over its live average duration; one wave
    # instruction per clock per CU is the peak (packed FP32 is not used)
    rec = committed_record(dominant) if n == cfg.n and args.kind == "asm" else None
    if rec and rec.get("valu_wave_instructions"):
        achieved = rec["valu_wave_instructions"] / (d["avg_us"] * 1e-6)
        roofline["issue"] = {"bound": "alu", "achieved": round(achieved / 1e9, 1),
                             "peak": VALU_PEAK_GWAVE, "unit": "G wave-instructions/s",
                             "frac": round(achieved / 1e9 / VALU_PEAK_GWAVE, 4),
                             "valu_wave_instructions": rec["valu_wave_instructions"]}

    batched = None
    if not args.no_batched and args.kind == "asm" and args.precision == "f32":
        # batched form: the same field to 64 distances in one cwo_zstack call, against the
        # same 64 distances as 64 plain calls (the plain figure above is one distance)
        zs = list(W.zstack_distances(64, 0.05, 0.5))
        z_form, z_chunk, _, _, _ = ctx.autotune(u, 64, cfg.pitch, cfg.pitch, cfg.wavelength, cfg.z)
        z_pps, z_ms = time_zstack(ctx, torch, u, zs, cfg.pitch, cfg.wavelength, 5, 2)
        batched = {"form": "cwo_zstack, one %dx%d field to 64 distances in [0.05, 0.5] m" % (n, n),
                   "planes_per_s": round(z_pps, 1), "ms_per_stack": round(z_ms, 4),
                   "vs_plain": round(z_pps / value, 3),
                   "schedule": {"row_form": z_form, "zchunk": z_chunk}}
        c3 = W.ZSTACK_1024
        u3 = torch.from_numpy(W.field_for(c3)).to(dev)
        z3 = list(W.zstack_distances(64, 0.05, 0.2))
        # the library's autotuner picks the row-pass form and the chunk size for this stack
        form, zchunk, _, _, _ = ctx.autotune(u3, 64, c3.pitch, c3.pitch, c3.wavelength, 0.1)
        c3_pps, c3_ms = time_zstack(ctx, torch, u3, z3, c3.pitch, c3.wavelength, 10, 2)
        batched["zstack_1024x64"] = {"planes_per_s": round(c3_pps, 1), "ms_per_stack": round(c3_ms, 4),
                                     "schedule": {"row_form": form, "zchunk": zchunk},
                                     "workload": "1024x1024 speckle, 4um, 633nm, 64 z in [0.05, 0.2] m"}
        # the same stack with FP16 / BF16 storage of the spectrum and the planes (autotuned
        # for that precision), each plane's error against the complex64 stack
        ref3 = ctx.zstack(u3, z3, c3.pitch, c3.pitch, c3.wavelength, kind="asm")
        for prec in ("f16", "bf16"):
            pf, pz, _, _, _ = ctx.autotune(u3, 64, c3.pitch, c3.pitch, c3.wavelength, 0.1,
                                           precision=prec)
            p_pps, p_ms = time_zstack(ctx, torch, u3, z3, c3.pitch, c3.wavelength, 10, 2, prec)
            y3 = ctx.zstack(u3, z3, c3.pitch, c3.pitch, c3.wavelength, kind="asm", precision=prec)
            err = float((torch.linalg.vector_norm(y3 - ref3) /
                         torch.linalg.vector_norm(ref3)).item())
            batched["zstack_1024x64"][prec + "_storage"] = {
                "planes_per_s": round(p_pps, 1), "ms_per_stack": round(p_ms, 4),
                "schedule": {"row_form": pf, "zchunk": pz}, "rel_l2_vs_complex64": float("%.3e" % err)}
            del y3
        del ref3
        del u3
        # 64 independent fields, each at its own distance (and every third one Fresnel): one
        # cwo_batch (one launch per pass, a transfer function per plane) vs the same 64
        # propagations as plain calls
        batched["independent_fields"] = {}
        zk = [float(z) for z in W.zstack_distances(64, 0.05, 0.5)]
        kinds = ["fresnel" if k % 3 == 1 else "asm" for k in range(64)]
        for ni in (n, 512):
            fields = [torch.from_numpy(W.uniform_random_field(ni, 800 + k)).to(dev) for k in range(64)]
            outs = [torch.empty_like(f) for f in fields]
            jobs = [(kd, f, o, dict(dx=cfg.pitch, dy=cfg.pitch, wavelength=cfg.wavelength, z=z))
                    for kd, f, o, z in zip(kinds, fields, outs, zk)]
            b_ms = time_call(torch, stream, lambda: ctx.batch(jobs), 5, 2)

            def plain():
                for kd, f, o, z in zip(kinds, fields, outs, zk):
                    (ctx.asm if kd == "asm" else ctx.fresnel)(f, cfg.pitch, cfg.pitch,
                                                               cfg.wavelength, z, out=o)

            p_ms = time_call(torch, stream, plain, 5, 2)
            batched["independent_fields"]["%d" % ni] = {
                "planes_per_s": round(64 * 1000.0 / b_ms, 1),
                "plain_planes_per_s": round(64 * 1000.0 / p_ms, 1),
                "vs_plain": round(p_ms / b_ms, 3),
                "workload": "64 independent %dx%d uniform random fields, 64 distances in "
                            "[0.05, 0.5] m, ASM with every third plane Fresnel" % (ni, ni)}
            del fields, outs
        # the same work captured once into a HIP graph and replayed (launch overhead and
        # host work paid once): the 1024^2 x 64 z-stack, 64 independent 512^2 fields in one
        # cwo_batch, and 64 plain 512^2 calls
        graph = {}
        u3 = torch.from_numpy(W.field_for(c3)).to(dev)
        o3 = torch.empty((64,) + tuple(u3.shape), dtype=torch.complex64, device=dev)
        f512 = [torch.from_numpy(W.uniform_random_field(512, 830 + k)).to(dev) for k in range(64)]
        o512 = [torch.empty_like(f) for f in f512]
        kw = dict(dx=cfg.pitch, dy=cfg.pitch, wavelength=cfg.wavelength, z=cfg.z)
        jobs = [("asm", f, o, kw) for f, o in zip(f512, o512)]
        cases = {
            "zstack_1024x64": (lambda: ctx.zstack(u3, z3, c3.pitch, c3.pitch, c3.wavelength, out=o3), 64),
            "independent_512x64": (lambda: ctx.batch(jobs), 64),
            "plain_512x64": (lambda: [ctx.asm(f, cfg.pitch, cfg.pitch, cfg.wavelength, cfg.z,
                                              out=o) for f, o in zip(f512, o512)], 64),
        }
        for name, (fn, planes) in cases.items():
            fn()
            torch.cuda.synchronize()
            eager_ms = time_call(torch, stream, fn, 20, 2)
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                fn()
            graph_ms = time_call(torch, torch.cuda.current_stream(dev), g.replay, 20, 2)
            graph[name] = {"eager_planes_per_s": round(planes * 1000.0 / eager_ms, 1),
                           "graph_planes_per_s": round(planes * 1000.0 / graph_ms, 1),
                           "graph_vs_eager": round(eager_ms / graph_ms, 3)}
            del g
        batched["graph_replay"] = graph
        del u3, o3, f512, o512

    gs = None
    if not args.no_gs and args.kind == "asm" and n == cfg.n and args.precision == "f32":
        # 200 ping-pong iterations (400 propagations) between two 2048^2 planes 0.1 m apart
        a1, a2, u0 = W.gs_problem(2048)
        ta1 = torch.from_numpy(a1).to(dev)
        ta2 = torch.from_numpy(a2).to(dev)
        tu = torch.from_numpy(u0).to(dev)
        g = W.GS_2048
        gs = {"workload": "2048x2048 rectangles targets 0.1 m apart, 8um, 532nm, 200 iterations"}
        for prec in ("f32", "f16", "bf16"):
            # storage of the padded spectrum between passes; arithmetic stays FP32
            tp = tu.clone()
            ctx.gs(tp.clone(), ta1, ta2, g.pitch, g.pitch, g.wavelength, g.z, iterations=5,
                   precision=prec)
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            errs = ctx.gs(tp, ta1, ta2, g.pitch, g.pitch, g.wavelength, g.z, iterations=200,
                          precision=prec)
            b.record(stream)
            torch.cuda.synchronize()
            gms = a.elapsed_time(b)
            e = errs.cpu().numpy()
            # per-kernel times of 20 more iterations (library HIP events on the stream)
            ctx.profile(True)
            ctx.gs(tp, ta1, ta2, g.pitch, g.pitch, g.wavelength, g.z, iterations=20,
                   precision=prec)
            stages = {}
            for st in (cwo.STAGE_COL, cwo.STAGE_ROW_GS):
                ms, cnt = ctx.profile_read(st)
                stages[cwo.STAGE_NAMES[st]] = round(1000.0 * ms / max(cnt, 1), 2)
            ctx.profile(False)
            gs[prec + "_storage"] = {
                "ms_total": round(gms, 3), "ms_per_iteration": round(gms / 200, 4),
                "propagations_per_s": round(400 * 1000.0 / gms, 1),
                "E_0": float("%.5f" % e[0]), "E_199": float("%.5f" % e[-1]),
                "kernel_us_with_events": stages}
            del tp
        del ta1, ta2, tu

    forms = None
    if not args.no_forms and args.kind == "asm" and n == cfg.n and args.precision == "f32":
        forms = other_forms(ctx, torch, W, u, u_np, cfg, stream, not args.no_cpu_baseline)

    serve = None
    if args.serve_requests > 0 and args.kind == "asm" and n == cfg.n and args.precision == "f32":
        serve = serve_bench(cwo.Context, torch, W, dev, args.serve_requests)

    y = out.cpu().numpy()
    line = {
        "metric": "%s planes/s at %d^2 fp32 (plain per-call form)" % (args.kind.upper(), n),
        "value": round(value, 2),
        "unit": "planes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_ms": args.settle_ms,
        "ms_per_step": round(ms_per_step, 5),
        "ms_per_step_with_kernel_events": round(profiled_ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "f32" else "f32 (%s storage)" % args.precision,
        "data": "synthetic",
        "config": {"workload": "%s-%d: %dx%d complex64 rectangles+random phase, pitch 8um, "
                               "532nm, z=0.5m, padded to %dx%d, plain per-call form"
                               % (args.kind, n, n, n, 2 * n, 2 * n),
                   "n": n, "padded": 2 * n, "pitch_m": cfg.pitch, "wavelength_m": cfg.wavelength,
                   "z_m": cfg.z, "seed": cfg.seed},
        "kernels": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kernels.items()},
        "roofline": roofline,
    }
    if batched is not None:
        line["batched"] = batched
    if gs is not None:
        line["gs_pingpong"] = gs
    if forms is not None:
        line["other_forms"] = forms
    if serve is not None:
        line["serving"] = serve
    if not args.no_cpu_baseline:
        ref, base = cpu_baseline(u_np, cfg, args.kind)
        from oracle import diffraction as D
        line["rel_l2_vs_oracle"] = float("%.3e" % D.rel_l2(y, ref))
        line["cpu_baseline"] = base
    print(json.dumps(line), flush=True)
    if args.copy_probe_mib > 0:
        nbytes = args.copy_probe_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "copies": 3}), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

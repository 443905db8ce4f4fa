#!/usr/bin/env python3
"""Benchmark: FP32 acoustic leapfrog with the 25-point star on one MI355X.

Workload (one benchmark step = one complete simulation): 1024 x 1024 x 512
interior, 4-cell zero Dirichlet halo, layered velocity model (8 horizontal
layers, speeds U[1500, 4500] m/s, seed 0), dx = 10 m, dt at CFL 0.4, Ricker
15 Hz source at the grid centre, 500 time steps from zero wavefields; three
FP32 fields resident (p, p_prev/p_next, v).

Prints one JSON line: GPts/s (point-updates per second), the HBM roofline
of the dominant kernel measured with HIP events on the launch stream, and the
FP64 CPU oracle timed on the host cores on a bounded sample of the workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GPts/s + % HBM roofline, 25-pt star FP32 vs FP16-store; p50/p99 shot latency"
HBM_PEAK_GBS = 8000.0
NX, NY, NZ, NSTEPS = 1024, 1024, 512, 500
BYTES_PER_POINT = 16          # read p, p_prev, v; write p_next (FP32)
EV_GROUP = 10                 # leapfrog launches per timing event pair
FLOPS_PER_POINT = 49          # paper's 2*points-1 convention for star3d4r


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the sources that define the timed kernel, its helpers, its
    argument layout and its tile choice."""
    h = hashlib.sha256()
    for name in ("star25.hip", "kcommon.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2309_04671_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "k_star25_wave_1024x1024x512_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(min_seconds=10.0):
    """The FP64 oracle on a 1024 x 1024 x 128 slab of the same model (same
    per-point work), stepping until at least min_seconds of CPU work."""
    import numpy as np
    import oracle
    import synth
    nx, ny, nz = NX, NY, 128
    v = synth.layered_velocity(nx, ny, nz, 0)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    co = synth.star25_coeffs()
    src = np.array([[nx // 2, ny // 2, nz // 2]], np.int32)
    prev = np.zeros((nz + 8, ny + 8, nx + 8))
    cur = np.zeros_like(prev)
    w = synth.ricker(64, dt)
    steps, elapsed = 0, 0.0
    while elapsed < min_seconds and steps < 64:
        t0 = time.perf_counter()
        r = oracle.wave_run(co, v, dt, dx, 2, src=src, amp=w[steps:steps + 2, None], prev=prev, cur=cur)
        elapsed += time.perf_counter() - t0
        prev, cur = r["prev"], r["cur"]
        steps += 2
    pts = nx * ny * nz * steps
    cores = oracle.num_threads()
    # the same loop nest on one core: 2 steps of a 1024 x 1024 x 16 slab
    n1 = 16
    v1 = np.ascontiguousarray(v[:n1])
    p1 = np.zeros((n1 + 8, ny + 8, nx + 8))
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.wave_run(co, v1, dt, dx, 2, prev=p1, cur=p1.copy())
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(cores)
    return {"value": round(pts / elapsed / 1e9, 4), "unit": "GPts/s", "cores": cores,
            "kind": "oracle",
            "sample": "%dx%dx%d slab of the same layered model, %d FP64 leapfrog steps, %.1f s"
                      % (nx, ny, nz, steps, elapsed),
            "one_core_value": round(nx * ny * n1 * 2 / t1 / 1e9, 4),
            "one_core_sample": "%dx%dx%d slab, 2 steps, %.2f s" % (nx, ny, n1, t1)}


def leg_storage(torch, lib, fields, synth, steps=2, nt=1000, n=512):
    """FP32 vs FP16-store vs BF16-store leapfrog on n^3, nt steps (same model,
    same source); GPts/s and HBM fraction at each form's algorithmic bytes."""
    out = {}
    vel = synth.layered_velocity(n, n, n, 0)
    dx = 10.0
    dt = synth.cfl_dt(vel, dx)
    gv = lib.grid_init(n, n, n, lib.SP_F32)
    V = fields.Field(gv).set_interior(vel)
    del vel
    amp = torch.tensor(synth.ricker(nt, dt, 15.0)[:, None], dtype=torch.float32, device="cuda")
    src = lib.make_sources([[n // 2, n // 2, n // 2]], amp.data_ptr(), 1)
    co = lib.coeffs(synth.star25_coeffs())
    stream = torch.cuda.current_stream()
    for name, dtype, bpp in (("fp32", lib.SP_F32, 16), ("fp16_store", lib.SP_F16, 10),
                             ("bf16_store", lib.SP_BF16, 10)):
        g = lib.grid_init(n, n, n, dtype)
        ws = fields.WaveState(g)
        ev = []
        for it in range(steps + 1):
            ws.reset()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            lib.sp_wave_step(g, co, dt, dx, gv, V.ptr, ws.st, nt, src=src, stream=stream)
            e1.record(stream)
            if it > 0:
                ev.append((e0, e1))
        torch.cuda.synchronize()
        ms = sum(a.elapsed_time(b) for a, b in ev) / len(ev)
        gpts = n ** 3 * nt / (ms / 1e3) / 1e9
        out[name] = {"gpts": round(gpts, 2), "ms_per_sim": round(ms, 2),
                     "bytes_per_point": bpp,
                     "hbm_frac": round(gpts * bpp / HBM_PEAK_GBS, 4),
                     "finite": bool(torch.isfinite(ws.cur().interior().float()).all())}
        del ws
    out["fp16_vs_fp32_speed"] = round(out["fp16_store"]["gpts"] / out["fp32"]["gpts"], 3)
    out["bf16_vs_fp32_speed"] = round(out["bf16_store"]["gpts"] / out["fp32"]["gpts"], 3)
    out["config"] = "%d^3, %d steps, layered v seed 0, Ricker 15 Hz at centre" % (n, nt)
    return out


# FLOPs per point of the accuracy-study kernels as the paper counts them
# (2P - 1 for P taps; the four Jacobi kernels carry one extra operation).
SUITE_FLOPS = {"j2d5pt": 10, "j2d9pt-gol": 18, "j2d9pt": 18, "j3d27pt": 54}
VALU_PEAK_GFLOPS = 78600.0      # FP32 FMA on all 256 CUs without packed-FP32 forms


def leg_suite(torch, lib, fields, synth, sweeps=10, apply_only=False):
    """Stencil suite throughput: the 25-point sp_stencil_apply at 512^3 and
    1024x1024x512, and every suite kernel through sp_apply (3D: 512^3; 2D:
    one 8192^2 plane), `sweeps` ping-pong sweeps each; GPts/s, GB/s at 8 B
    per point, GFLOP/s, and the fraction of the binding peak (HBM 8 TB/s or
    the 78.6 TFLOP/s FP32 VALU).  apply_only: the 25-point apply alone (a
    short run for counter collection)."""
    import numpy as np
    stream = torch.cuda.current_stream()
    out = {}

    def timed(g, fn):
        # The GPU needs tens of milliseconds of continuous load before its
        # clocks settle (40 sweeps of 512^3 are only 8 ms): time 40 sweeps,
        # continue for about 150 ms of sweeps, then take the median of three
        # timed batches.
        a, b = fields.Field(g), fields.Field(g)
        a.set_interior(torch.rand((g.nz, g.ny, g.nx), generator=torch.Generator().manual_seed(0)))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn(g, a, b, 40)
        e1.record(stream)
        torch.cuda.synchronize()
        extra = int(150.0 / max(e0.elapsed_time(e1) / 40, 1e-3))
        if extra > 0:
            fn(g, a, b, min(extra, 20000))
        ms = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn(g, a, b, sweeps)
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1) / sweeps)
        ok = bool(torch.isfinite(b.interior()).all())
        return sorted(ms)[1], ok

    def record(name, g, ms, flops, ok):
        gpts = g.nx * g.ny * g.nz / (ms / 1e3) / 1e9
        gbs, gfl = gpts * 8, gpts * flops
        bound = "alu" if flops * HBM_PEAK_GBS / 8 > VALU_PEAK_GFLOPS else "hbm"
        frac = gfl / VALU_PEAK_GFLOPS if bound == "alu" else gbs / HBM_PEAK_GBS
        out[name] = {"grid": [g.nx, g.ny, g.nz], "gpts": round(gpts, 2), "us_per_sweep": round(ms * 1e3, 1),
                     "gbs_at_8B": round(gbs, 1), "gflops": round(gfl, 1), "flops_per_point": flops,
                     "bound": bound, "frac": round(frac, 4), "finite": ok}

    # The FD8 weights scaled by 1 / sum |c|: the same kernel and cost, and
    # repeated sweeps stay finite (the unscaled operator grows ~19.5x per sweep).
    c8 = synth.star25_coeffs()
    norm = abs(c8["center"]) + 2 * sum(abs(x) for k in ("ax", "ay", "az") for x in c8[k])
    co = lib.coeffs({"center": c8["center"] / norm, **{k: [x / norm for x in c8[k]] for k in ("ax", "ay", "az")}})
    # one 64^3 sweep is latency-bound (1.5 MB fits in L2); time per sweep
    # over 1000 back-to-back sweeps
    g = lib.grid_init(64, 64, 64)
    a, b = fields.Field(g), fields.Field(g)
    a.set_interior(torch.rand((64, 64, 64), generator=torch.Generator().manual_seed(0)))
    lib.sp_stencil_apply(g, co, 2000, a.ptr, b.ptr, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lib.sp_stencil_apply(g, co, 1000, a.ptr, b.ptr, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    out["apply25_64^3_latency"] = {"us_per_sweep": round(e0.elapsed_time(e1), 2),
                                   "note": "1000 back-to-back sweeps, latency-bound (1-plane z-chunks)"}
    for n3 in ((512, 512, 512), (1024, 1024, 512)):
        g = lib.grid_init(*n3)
        ms, ok = timed(g, lambda g, a, b, k: lib.sp_stencil_apply(g, co, k, a.ptr, b.ptr, stream=stream))
        record("apply25_%dx%dx%d" % n3, g, ms, 49, ok)
    if apply_only:
        out["config"] = ("median of 3 batches of %d sweeps each after about 150 ms of warm-up sweeps; "
                         "inputs U[0,1) FP32; the FD8 weights over sum |c|" % sweeps)
        return out
    # NEXT-2 A/B on equal terms: the accumulating z-stream (sp_apply,
    # star3d4r) with the very weights and input of the register-queue
    # apply25 at 512^3 above, so both sweep the same data.
    wab = np.zeros((9, 9, 9))
    wab[4, 4, 4] = c8["center"] / norm
    for r in range(1, 5):
        wab[4, 4, 4 + r] = wab[4, 4, 4 - r] = c8["ax"][r - 1] / norm
        wab[4, 4 + r, 4] = wab[4, 4 - r, 4] = c8["ay"][r - 1] / norm
        wab[4 + r, 4, 4] = wab[4 - r, 4, 4] = c8["az"][r - 1] / norm
    for n3 in ((512, 512, 512), (1024, 1024, 512)):
        g = lib.grid_init(*n3)
        ms, ok = timed(g, lambda g, a, b, k: lib.sp_apply(g, "star", wab, a.ptr, b.ptr, k, stream=stream))
        record("semi_stencil_star3d4r_fd8_%dx%dx%d" % n3, g, ms, 49, ok)
        torch.cuda.empty_cache()
    for name in sorted(synth.SUITE):
        kind, ndim, r = synth.SUITE[name]
        w = synth.suite_weights(name, 0)
        g = lib.grid_init(512, 512, 512) if ndim == 3 else lib.grid_init_2d(8192, 8192)
        ms, ok = timed(g, lambda g, a, b, k: lib.sp_apply(g, kind, w, a.ptr, b.ptr, k, stream=stream))
        flops = SUITE_FLOPS.get(name, 2 * int(np.count_nonzero(w)) - 1)
        record(name, g, ms, flops, ok)
        torch.cuda.empty_cache()
    out["config"] = ("median of 3 batches of %d sweeps each after about 150 ms of warm-up sweeps; inputs U[0,1) FP32; apply25 with "
                     "the FD8 weights over sum |c|, the suite with seeded positive weights (sum 1)" % sweeps)
    return out


def leg_storage_vs_fp32(torch, lib, fields, synth, n=512, nt=1000, n_e=400):
    """Each storage form against the plain FP32 form on the same GPU after nt
    steps of the n^3 storage workload (rel-L2, max abs and RMSD of the final
    field, FP64 sums), and the drift of the discrete energy between step n_e
    (source finished) and step nt, evaluated in FP64 on the GPU from decoded
    FP32 copies of (u^{n-1}, u^n).  The FP64-oracle errors of the same forms
    are measured by the storage-error tests."""
    import numpy as np
    vel = synth.layered_velocity(n, n, n, 0)
    dx = 10.0
    dt = synth.cfl_dt(vel, dx)
    gv = lib.grid_init(n, n, n, lib.SP_F32)
    V = fields.Field(gv).set_interior(vel)
    del vel
    amp = torch.tensor(synth.ricker(nt, dt, 15.0)[:, None], dtype=torch.float32, device="cuda")
    src = lib.make_sources([[n // 2, n // 2, n // 2]], amp.data_ptr(), 1)
    co = lib.coeffs(synth.star25_coeffs())
    F0, F1 = fields.Field(gv), fields.Field(gv)
    e_out = torch.zeros(1, dtype=torch.float64, device="cuda")
    e_ws = torch.zeros(max(int(lib.load().sp_energy_ws_bytes(gv)) // 8, 1), dtype=torch.float64,
                       device="cuda")

    def energy(ws):
        F0.set_interior(ws.decoded("prev"))
        F1.set_interior(ws.decoded("cur"))
        lib.sp_energy(gv, co, dt, dx, gv, V.ptr, F0.ptr, F1.ptr, e_out.data_ptr(), e_ws.data_ptr())
        torch.cuda.synchronize()
        return float(e_out.item())

    out = {"config": "%d^3, %d steps, layered v seed 0, Ricker 15 Hz at centre; errors of the final "
                     "field against the FP32 form on the same GPU; energy drift between steps %d and %d"
                     % (n, nt, n_e, nt)}
    ref = None
    for name, dtype in (("fp32", lib.SP_F32), ("fp16_store", lib.SP_F16), ("bf16_store", lib.SP_BF16)):
        g = lib.grid_init(n, n, n, dtype)
        ws = fields.WaveState(g)
        lib.sp_wave_step(g, co, dt, dx, gv, V.ptr, ws.st, n_e, src=src)
        e_a = energy(ws)
        lib.sp_wave_step(g, co, dt, dx, gv, V.ptr, ws.st, nt - n_e, src=src)
        e_b = energy(ws)
        rec = {"energy_drift": float((e_b - e_a) / e_a)}
        if ref is None:
            ref = ws.decoded()
            rec["peak"] = float(np.max(np.abs(ref)))
        else:
            d = ws.decoded() - ref
            rec.update(rel_l2_vs_fp32=float(np.linalg.norm(d) / np.linalg.norm(ref)),
                       max_abs_vs_fp32=float(np.max(np.abs(d))), rmsd_vs_fp32=float(np.sqrt(np.mean(d * d))))
            del d
        out[name] = rec
        del ws
    return out


def oracle_cores():
    import oracle
    return oracle.num_threads()


def leg_storage_vs_oracle(torch, lib, fields, synth, n=128, nt=1000):
    """The three storage forms against the FP64 oracle after nt steps of the
    n^3 storage workload (same model, source and wavelet as the 512^3 legs):
    rel-L2, max abs and RMSD of the final field.  The oracle run is timed on
    the host cores (it is this leg's CPU baseline)."""
    import numpy as np
    import oracle
    vel = synth.layered_velocity(n, n, n, 0)
    dx = 10.0
    dt = synth.cfl_dt(vel, dx)
    amp32 = synth.ricker(nt, dt, 15.0)[:, None].astype(np.float32)
    src_xyz = np.array([[n // 2, n // 2, n // 2]], np.int32)
    co_d = synth.star25_coeffs()
    t0 = time.perf_counter()
    r = oracle.wave_run(co_d, vel, dt, dx, nt, src=src_xyz, amp=amp32.astype(np.float64))
    t_or = time.perf_counter() - t0
    ref = oracle.interior(r["cur"]).copy()
    del r
    gv = lib.grid_init(n, n, n, lib.SP_F32)
    V = fields.Field(gv).set_interior(vel)
    amp = torch.tensor(amp32, device="cuda")
    src = lib.make_sources(src_xyz, amp.data_ptr(), 1)
    co = lib.coeffs(co_d)
    nref = float(np.linalg.norm(ref))
    out = {"config": "%d^3, %d steps, layered v seed 0, Ricker 15 Hz at centre; final field "
                     "against the FP64 oracle" % (n, nt),
           "peak": float(np.max(np.abs(ref))),
           "oracle": {"value": round(n ** 3 * nt / t_or / 1e9, 4), "unit": "GPts/s",
                      "seconds": round(t_or, 2), "cores": oracle_cores(), "kind": "oracle",
                      "sample": "the whole %d^3 x %d-step run" % (n, nt)}}
    for name, dtype in (("fp32", lib.SP_F32), ("fp16_store", lib.SP_F16), ("bf16_store", lib.SP_BF16)):
        g = lib.grid_init(n, n, n, dtype)
        ws = fields.WaveState(g)
        lib.sp_wave_step(g, co, dt, dx, gv, V.ptr, ws.st, nt, src=src)
        torch.cuda.synchronize()
        d = ws.decoded().astype(np.float64) - ref
        out[name] = {"rel_l2_vs_oracle": float(np.linalg.norm(d) / nref),
                     "max_abs_vs_oracle": float(np.max(np.abs(d))),
                     "rmsd_vs_oracle": float(np.sqrt(np.mean(d * d)))}
        del ws, d
    return out


def oracle_small_and_adjoint(synth):
    """The oracle beside the small forms, timed on the host cores: one
    25-point sweep at 64^3, the misfit gradient at 48^3 x 200 steps
    (the gradient check's size), and bounded samples of the full-size ones:
    the checkpointed gradient at 256^3 over 24 steps (the adjoint workload's
    grid) and 10 leapfrog steps at 512^3 (the storage forms' grid)."""
    import numpy as np
    import oracle
    u = oracle.padded(synth.uniform_field((64, 64, 64), 0))
    co = synth.star25_coeffs()
    reps = 0
    t0 = time.perf_counter()
    while reps < 20 or time.perf_counter() - t0 < 1.0:
        oracle.laplacian(u, co)
        reps += 1
    t_c0 = (time.perf_counter() - t0) / reps
    n, nt = 48, 200
    v = synth.gaussian_bump(synth.layered_velocity(n, n, n, 0), (24, 24, 24), 4.0, 0.10)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    src = np.array([[24, 24, 8]], np.int32)
    rec = synth.receiver_plane(n, n, n - 8, 2)
    amp = synth.ricker(nt, dt, 15.0)[:, None]
    obs = np.zeros((nt, len(rec)))
    t0 = time.perf_counter()
    oracle.adjoint_grad(co, v, dt, dx, nt, src, amp, rec, obs)
    t_adj = time.perf_counter() - t0
    # the 256^3 adjoint workload, 24 steps with a checkpoint every 6
    n3, nt3, c3 = 256, 24, 6
    v0, _ = synth.adjoint_models(n3)
    dt3 = synth.cfl_dt(v0, dx)
    src3 = np.array([[n3 // 2, n3 // 2, 8]], np.int32)
    rec3 = synth.receiver_plane(n3, n3, 8, 2)
    amp3 = synth.ricker(nt3, dt3, 15.0)[:, None]
    t0 = time.perf_counter()
    oracle.adjoint_grad_ckpt(co, v0, dt3, dx, nt3, src3, amp3, rec3, np.zeros((nt3, len(rec3))), c3)
    t_adj3 = time.perf_counter() - t0
    del v0
    # the 512^3 storage workload, 10 FP64 leapfrog steps
    n5, nt5 = 512, 10
    v5 = synth.layered_velocity(n5, n5, n5, 0)
    dt5 = synth.cfl_dt(v5, dx)
    t0 = time.perf_counter()
    oracle.wave_run(co, v5, dt5, dx, nt5, src=np.array([[n5 // 2] * 3], np.int32),
                    amp=synth.ricker(nt5, dt5, 15.0)[:, None])
    t_5 = time.perf_counter() - t0
    del v5
    cores = oracle_cores()
    return ({"value": round(64 ** 3 / t_c0 / 1e9, 4), "unit": "GPts/s", "us_per_sweep": round(t_c0 * 1e6, 1),
             "cores": cores, "kind": "oracle", "sample": "%d sweeps of 64^3" % reps},
            {"value": round(n ** 3 * nt / t_adj / 1e9, 4), "unit": "GPts/s (time steps of the gradient)",
             "seconds": round(t_adj, 2), "cores": cores, "kind": "oracle",
             "sample": "misfit gradient at %d^3 x %d steps, every state kept" % (n, nt)},
            {"value": round(n3 ** 3 * nt3 / t_adj3 / 1e9, 4), "unit": "GPts/s (time steps of the gradient)",
             "seconds": round(t_adj3, 2), "cores": cores, "kind": "oracle",
             "sample": "misfit gradient at %d^3 x %d steps, checkpoint every %d (forward, recompute, "
                       "adjoint and FP64 sum)" % (n3, nt3, c3)},
            {"value": round(n5 ** 3 * nt5 / t_5 / 1e9, 4), "unit": "GPts/s",
             "seconds": round(t_5, 2), "cores": cores, "kind": "oracle",
             "sample": "%d FP64 leapfrog steps at %d^3" % (nt5, n5)})


def leg_adjoint(torch, lib, fields, synth, n=256, nt=1000, ckpt=32):
    """Misfit gradient at n^3 x nt (checkpoint every ckpt steps): wall time of
    forward + backward against the plain forward run."""
    import numpy as np
    from paper_2309_04671_amd.adjoint import WaveOp, WaveProblem
    v0, v_obs = synth.adjoint_models(n)
    dx = 10.0
    dt = synth.cfl_dt(v0, dx)
    src = np.array([[n // 2, n // 2, 8]], np.int32)
    rec = synth.receiver_plane(n, n, 8, 2)
    amp = synth.ricker(nt, dt, 15.0)[:, None]
    prob = WaveProblem(n, n, n, synth.star25_coeffs(), dt, dx, nt, src, amp, rec, ckpt=ckpt)
    with torch.no_grad():
        d_obs = WaveOp.apply(torch.tensor(v_obs, device="cuda"), prob).double()
    vt = torch.tensor(v0, device="cuda")
    # plain forward
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.no_grad():
        WaveOp.apply(vt, prob)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    def fwd_bwd():
        vv = vt.clone().requires_grad_(True)
        tr = WaveOp.apply(vv, prob)
        J = 0.5 * ((tr.double() - d_obs) ** 2).sum()
        J.backward()
        return J, vv.grad

    # the first call also allocates the recompute ring and gradient buffers
    torch.cuda.reset_peak_memory_stats()
    t0 = time.perf_counter()
    fwd_bwd()
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    peak_gb = torch.cuda.max_memory_allocated() / 1e9
    t0 = time.perf_counter()
    J, g = fwd_bwd()
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    bytes_per_step = 68      # forward 16 + recompute 16 + fused adjoint step 36 (B/pt)
    return {"config": "%d^3, %d steps, checkpoint every %d, %d receivers" % (n, nt, ckpt, len(rec)),
            "forward_s": round(t_fwd, 4), "forward_backward_s": round(t_all, 4),
            "first_call_s": round(t_first, 4),
            "peak_memory_gb": round(peak_gb, 2),
            "ratio_vs_forward": round(t_all / t_fwd, 3),
            "effective_gbs": round(n ** 3 * nt * bytes_per_step / t_all / 1e9, 1),
            "misfit": float(J.detach()), "grad_finite": bool(torch.isfinite(g).all()),
            "grad_norm": float(g.double().norm())}



# The paper's own timings of this kernel (inner region of its Acoustic ISO
# kernel, 750 x 994 x 300 grid, 10,000 iterations, "Kernel" column of the
# CSL time-measurement table in its evaluation of runtime performance), in
# seconds, with the device each ran on.  Context only: other hardware.
PAPER_KERNEL_S = {"NVIDIA H100, CUDA f4 template": 45.0160, "AMD MI210, HIP gmem template": 138.1122,
                  "Cerebras CS-2, CSL": 0.4685, "AMD EPYC 9684X (192 cores), OpenMP loop": 269.4177}


def leg_paper(torch, lib, fields, synth, nt=10000):
    """The paper's timing workload on this GPU: the leapfrog (inner region,
    zero Dirichlet frame) on a 750 x 994 x 300 grid for 10,000 iterations,
    FP32, layered model and Ricker source at the centre as in the headline
    workload; kernel time from HIP events around the whole run, next to the
    paper's own kernel times on its hardware."""
    nx, ny, nz = 750, 994, 300
    g = lib.grid_init(nx, ny, nz)
    v = synth.layered_velocity(nx, ny, nz, 0)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    V = fields.Field(g).set_interior(v)
    del v
    amp = torch.tensor(synth.ricker(nt, dt, 15.0)[:, None], dtype=torch.float32, device="cuda")
    src = lib.make_sources([[nx // 2, ny // 2, nz // 2]], amp.data_ptr(), 1)
    co = lib.coeffs(synth.star25_coeffs())
    ws = fields.WaveState(g)
    stream = torch.cuda.current_stream()
    lib.sp_wave_step(g, co, dt, dx, g, V.ptr, ws.st, 200, src=src, stream=stream)   # warm-up
    ws.reset()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lib.sp_wave_step(g, co, dt, dx, g, V.ptr, ws.st, nt, src=src, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3
    finite = bool(torch.isfinite(ws.cur().interior()).all())
    pts = nx * ny * nz * nt
    out = {"config": "750x994x300, %d leapfrog iterations, FP32, layered v seed 0, Ricker 15 Hz at centre" % nt,
           "kernel_s": round(t, 4), "gpts": round(pts / t / 1e9, 2),
           "hbm_frac_at_16B": round(16 * pts / t / 1e9 / HBM_PEAK_GBS, 4), "finite": finite,
           "paper_kernel_s": PAPER_KERNEL_S,
           "paper_gpts": {k: round(pts / s / 1e9, 2) for k, s in PAPER_KERNEL_S.items()}}
    del ws, V
    return out


def leg_fused(torch, lib, fields, synth, nt=100):
    """Two leapfrog steps per sweep (sp_wave_step_fused) against the
    single-step sweep on the 1024x1024x512 workload, nt steps each after a
    warm-up run, median of 3.  Reported as effective bytes: the single-step
    algorithmic 16 B per point-step over the measured time, and the fused
    sweep's own 10 B per point-step (u^n, u^{n-1}, v read once, u^{n+1} and
    u^{n+2} written, per two steps)."""
    nx, ny, nz = NX, NY, NZ
    g = lib.grid_init(nx, ny, nz)
    v = synth.layered_velocity(nx, ny, nz, 0)
    V = fields.Field(g).set_interior(v)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    del v
    amp = torch.tensor(synth.ricker(nt, dt)[:, None], dtype=torch.float32, device="cuda")
    src = lib.make_sources([[nx // 2, ny // 2, nz // 2]], amp.data_ptr(), 1)
    co = lib.coeffs(synth.star25_coeffs())
    ws = fields.WaveState(g, spares=True)
    stream = torch.cuda.current_stream()
    runs = {"single_step": lambda: lib.sp_wave_step(g, co, dt, dx, g, V.ptr, ws.st, nt, src=src,
                                                    stream=stream),
            "fused_two_steps": lambda: lib.sp_wave_step_fused(g, co, dt, dx, g, V.ptr, ws.st, nt,
                                                              ws.spare, src=src, stream=stream)}
    out = {}
    pts = nx * ny * nz
    for name, fn in runs.items():
        ws.reset()
        fn()
        ms = []
        for _ in range(3):
            ws.reset()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1) / nt)
        m = sorted(ms)[1]
        out[name] = {"us_per_step": round(m * 1e3, 1), "gpts": round(pts / m / 1e6, 1),
                     "effective_gbs_at_16B": round(16 * pts / m / 1e6, 1)}
    f = out["fused_two_steps"]
    f["algorithmic_gbs_at_10B"] = round(10 * pts / (f["us_per_step"] * 1e3), 1)
    f["vs_single_step"] = round(out["single_step"]["us_per_step"] / f["us_per_step"], 3)
    out["config"] = "1024x1024x512, %d steps, 64x48 regions (56x40 tiles), median of 3" % nt
    del ws, V
    return out


def leg_pml(torch, lib, fields, synth, nt=100, width=32):
    """Leapfrog with the absorbing layer on the 1024x1024x512 workload (layer
    of `width` cells on every face): the seven-region map (inner box by the
    streaming kernel, six slabs by the layer kernel), the two-region map
    (the six slabs in one launch), the unified map (layer kernel everywhere)
    and the plain leapfrog, nt steps each after a
    warm-up run; the layer kernel's own rate at its 28 B per point."""
    import numpy as np
    nx, ny, nz = NX, NY, NZ
    g = lib.grid_init(nx, ny, nz)
    v = synth.layered_velocity(nx, ny, nz, 0)
    V = fields.Field(g).set_interior(v)
    dx = 10.0
    dt = synth.cfl_dt(v, dx)
    E = fields.Field(g)
    lib.sp_pml_profile(g, width, synth.pml_eta_max(float(v.max()), width, dx), E.ptr)
    del v
    PSI = fields.Field(g)
    amp = torch.tensor(synth.ricker(nt, dt)[:, None], dtype=torch.float32, device="cuda")
    src = lib.make_sources([[nx // 2, ny // 2, nz // 2]], amp.data_ptr(), 1)
    co = lib.coeffs(synth.star25_coeffs())
    ws = fields.WaveState(g)
    stream = torch.cuda.current_stream()
    alpha = np.pi * 15.0
    runs = {"plain": lambda: lib.sp_wave_step(g, co, dt, dx, g, V.ptr, ws.st, nt, src=src, stream=stream),
            "seven_region": lambda: lib.sp_wave_step_pml(g, co, dt, dx, g, V.ptr, ws.st, nt,
                                                         lib.make_pml(width, E.ptr, PSI.ptr, alpha, 1),
                                                         src=src, stream=stream),
            "two_region": lambda: lib.sp_wave_step_pml(g, co, dt, dx, g, V.ptr, ws.st, nt,
                                                       lib.make_pml(width, E.ptr, PSI.ptr, alpha, 2),
                                                       src=src, stream=stream),
            "unified": lambda: lib.sp_wave_step_pml(g, co, dt, dx, g, V.ptr, ws.st, nt,
                                                    lib.make_pml(width, E.ptr, PSI.ptr, alpha, 0),
                                                    src=src, stream=stream)}
    out = {}
    for name, fn in runs.items():
        ws.reset()
        fn()
        ms = []
        for _ in range(3):
            ws.reset()
            PSI.buf.zero_()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1) / nt)
        m = sorted(ms)[1]
        out[name] = {"us_per_step": round(m * 1e3, 1), "gpts": round(nx * ny * nz / m / 1e6, 1)}
    inner = (nx - 2 * width) * (ny - 2 * width) * (nz - 2 * width)
    layer_pts = nx * ny * nz - inner
    layer_us = out["seven_region"]["us_per_step"] - out["plain"]["us_per_step"] * inner / (nx * ny * nz)
    out["layer_kernel"] = {"points": layer_pts, "us_per_step_est": round(layer_us, 1),
                           "gbs_at_28B": round(28 * layer_pts / (layer_us * 1e3), 1),
                           "note": "layer time = seven-region step minus the inner box at the plain rate"}
    out["config"] = "1024x1024x512, layer %d cells, alpha pi*15 1/s, %d steps, median of 3" % (width, nt)
    return out


SERVE_SHAPES = [(128, 128, 128), (192, 192, 160), (256, 256, 256), (384, 384, 256)]


def _serve_requests(torch, lib, serve, synth, n, seed0):
    """Seeded request stream: grid uniform over the four shapes, steps
    U{200..2000}, FP32 or FP16 storage by a fair coin, layered v and source
    position per request (seed 1000 + id), receivers on z = 8 every 4th cell."""
    import numpy as np
    reqs = []
    for i in range(n):
        rid = seed0 + i
        rng = np.random.default_rng(1000 + rid)
        nx, ny, nz = SERVE_SHAPES[int(rng.integers(0, 4))]
        nsteps = int(rng.integers(200, 2001))
        dtype = lib.SP_F16 if rng.integers(0, 2) else lib.SP_F32
        v = synth.layered_velocity(nx, ny, nz, 1000 + rid)
        dt = synth.cfl_dt(v, 10.0)
        src = synth.random_points(nx, ny, nz, 1, 5000 + rid, margin=8)
        amp = synth.ricker(nsteps, dt, 15.0)[:, None]
        rec = synth.receiver_plane(nx, ny, 8, 4)
        shot = serve.Shot(v, dt, 10.0, nsteps, synth.star25_coeffs(), src, amp, rec=rec,
                          dtype=dtype, final=False)
        reqs.append(shot)
    torch.cuda.synchronize()
    return reqs


def leg_serve(torch, lib, fields, synth, nreq=96, loads=(0.5, 0.8, 1.0), budget_gb=200.0, slots=32,
              chunk=16):
    """Served shot stream (continuous batching): capacity from a saturating
    batch, then a Poisson stream of nreq requests at each offered load (a
    fraction of that capacity); latency = done - submit per request.  The
    top-level figures are those at load 0.8; `loads` holds all three."""
    import numpy as np
    from paper_2309_04671_amd import serve
    budget = int(budget_gb * 1e9)
    arena = budget + (256 << 20)
    cl = serve.ServeClient(arena_bytes=arena, budget_bytes=budget, max_slots=slots, chunk_steps=chunk)
    # capacity: a saturating batch submitted at once
    sat = _serve_requests(torch, lib, serve, synth, 24, 100000)
    t0 = time.perf_counter()
    for s in sat:
        cl.submit(s)
    cl.drain()
    cap_s = time.perf_counter() - t0
    capacity = sum(s.points for s in sat) / cap_s / 1e9
    del sat

    def stream(rho, seed0):
        reqs = _serve_requests(torch, lib, serve, synth, nreq, seed0)
        mean_pts = float(np.mean([s.points for s in reqs]))
        rate = rho * capacity * 1e9 / mean_pts                 # requests per second
        gaps = np.random.default_rng(7 + seed0).exponential(1.0 / rate, nreq)
        t_arr = time.perf_counter() + np.cumsum(gaps)
        for s, ta in zip(reqs, t_arr):
            d = ta - time.perf_counter()
            if d > 0:
                time.sleep(d)
            cl.submit(s)
        cl.drain()
        lat, waits, done_t, sub_t = [], [], [], []
        for s in reqs:
            ok, st = cl.poll(s.ticket)
            if not ok or st.state != lib.SP_SHOT_DONE:
                raise RuntimeError("served shot failed: state %d error %d" % (st.state, st.error))
            lat.append(st.t_done - st.t_submit)
            waits.append(st.t_admit - st.t_submit)
            done_t.append(st.t_done)
            sub_t.append(st.t_submit)
        makespan = max(done_t) - min(sub_t)
        lat = np.array(lat)
        res = {"p50_latency_s": round(float(np.percentile(lat, 50)), 4),
               "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
               "mean_admit_wait_s": round(float(np.mean(waits)), 4),
               "aggregate_gpts": round(sum(s.points for s in reqs) / makespan / 1e9, 1),
               "makespan_s": round(makespan, 3)}
        return res, reqs

    per_load = {}
    main_reqs = None
    for k, rho in enumerate(loads):
        res, reqs = stream(rho, 0 if abs(rho - 0.8) < 1e-9 else 1000 * (k + 1))
        per_load["%.1f" % rho] = res
        if abs(rho - 0.8) < 1e-9:
            main_reqs = reqs
        else:
            del reqs
    # two requests of the load-0.8 stream re-run alone must reproduce their
    # traces bit for bit
    solo_equal = True
    if main_reqs is not None:
        small = sorted(range(nreq), key=lambda i: main_reqs[i].points)[:2]
        for i in small:
            s = main_reqs[i]
            ref = s.traces.clone()
            s.traces.zero_()
            cl2 = serve.ServeClient(arena_bytes=4 << 30, max_slots=1, chunk_steps=chunk)
            cl2.submit(s)
            cl2.drain()
            cl2.close()
            solo_equal = solo_equal and bool(torch.equal(ref, s.traces))
    cl.close()
    out = {"config": "%d requests per load, Poisson arrivals at %s of capacity, shapes %s, steps U{200..2000}, "
                     "FP32/FP16 50/50, budget %.0f GB, %d slots, %d-step chunks"
                     % (nreq, "/".join("%.0f%%" % (100 * r) for r in loads), SERVE_SHAPES, budget_gb, slots,
                        chunk),
           "capacity_gpts": round(capacity, 1)}
    out.update(per_load.get("0.8", {}))
    out["loads"] = per_load
    out["solo_equal_sampled"] = solo_equal
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed simulations (500 time steps each)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--nt", type=int, default=NSTEPS,
                    help="time steps per simulation (default: the workload's 500; fewer only for "
                         "profiling runs)")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"],
                    help="wavefield storage of the headline run (f32 is the benchmark; the others "
                         "only for profiling runs)")
    ap.add_argument("--grid", default=None, metavar="NXxNYxNZ",
                    help="override the headline grid (profiling runs only)")
    ap.add_argument("--no-headline", action="store_true",
                    help="skip the headline run (profiling runs of the extra legs)")
    ap.add_argument("--legs", default="storage,storage_error,storage_oracle,adjoint,paper,fused,pml,suite,serve",
                    help="extra measurements after the headline run (comma list; '' for none)")
    ap.add_argument("--calibrate-copy", type=float, default=0.0, metavar="GIB",
                    help="instead of the benchmark, copy a GIB-sized buffer 4 times with torch "
                         "(reference kernel for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X and has no "
              "multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2309_04671_amd import fields, lib

    lib.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.calibrate_copy > 0:
        n = int(args.calibrate_copy * (1 << 30))
        a = torch.ones(n, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "torch copy", "bytes_read_per_launch": n,
                          "bytes_written_per_launch": n, "launches": 4}))
        return
    nt = args.nt
    nx, ny, nz = (NX, NY, NZ) if not args.grid else (int(a) for a in args.grid.split("x"))
    sdt = {"f32": lib.SP_F32, "f16": lib.SP_F16, "bf16": lib.SP_BF16}[args.dtype]
    if args.no_headline:
        args.steps = 0

    log("setting up %dx%dx%d" % (nx, ny, nz))
    gv = lib.grid_init(nx, ny, nz, lib.SP_F32)
    g = lib.grid_init(nx, ny, nz, sdt)
    vel = synth.layered_velocity(nx, ny, nz, 0)
    dx = 10.0
    dt = synth.cfl_dt(vel, dx)
    V = fields.Field(gv).set_interior(vel)
    del vel
    ws = fields.WaveState(g)
    w = synth.ricker(nt, dt, 15.0)
    amp = torch.tensor(w[:, None], dtype=torch.float32, device=dev)
    src = lib.make_sources([[nx // 2, ny // 2, nz // 2]], amp.data_ptr(), 1)
    co = lib.coeffs(synth.star25_coeffs())
    ev = []

    def simulate(timed):
        ws.reset()
        if not timed:
            lib.sp_wave_step(g, co, dt, dx, gv, V.ptr, ws.st, nt, src=src, stream=stream)
            return
        # one call per group of EV_GROUP steps with a HIP event pair around
        # it on the launch stream: the launches of one call run back to back,
        # so the group's time over its launch count is the average launch
        # duration (an event pair around every single launch would leave a
        # ~10 us gap before each kernel and cost the wall clock 0.7 %)
        for k0 in range(0, nt, EV_GROUP):
            k = min(EV_GROUP, nt - k0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            lib.sp_wave_step(g, co, dt, dx, gv, V.ptr, ws.st, k, src=src, stream=stream)
            e1.record(stream)
            ev.append((e0, e1, k))

    for i in range(args.warmup if args.steps else 0):
        simulate(False)
        torch.cuda.synchronize()
        log("warmup %d done" % i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        simulate(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log("timed %d simulations in %.3f s" % (args.steps, wall))
    if args.steps and not bool(torch.isfinite(ws.cur().interior().float()).all()):
        raise RuntimeError("non-finite wavefield")

    npts = nx * ny * nz
    bpp = BYTES_PER_POINT if sdt == lib.SP_F32 else 10
    steps_done = max(args.steps, 1)
    gpts = npts * nt * args.steps / max(wall, 1e-9) / 1e9
    kern_ms = sum(a.elapsed_time(b) for a, b, _ in ev)   # one event pair per launch group
    launches = sum(k for _, _, k in ev)
    launch_s = kern_ms / 1e3 / launches if ev else float("nan")
    achieved = bpp * npts / launch_s / 1e9 if ev else 0.0
    traffic = measured_traffic() if (sdt == lib.SP_F32 and (nx, ny, nz) == (NX, NY, NZ)) else None

    out = {
        "metric": METRIC,
        "value": round(gpts, 3),
        "unit": "GPts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / steps_done * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "acoustic leapfrog, 25-point star, %dx%dx%d %s storage, %d time "
                               "steps, layered v (8 layers, seed 0), Ricker 15 Hz at centre, CFL 0.4"
                               % (nx, ny, nz, args.dtype.upper(), nt),
                   "grid": [nx, ny, nz], "time_steps": nt, "global_batch": 1,
                   "step": "one full simulation"},
        "roofline": {"bound": "hbm", "kernel": "k_star25 (WAVE)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "avg_launch_us": round(launch_s * 1e6, 2) if ev else None,
                     "bytes_per_launch": bpp * npts},
        "hbm_frac_of_wall": round(gpts * bpp / HBM_PEAK_GBS, 4),
        "gflops": round(gpts * FLOPS_PER_POINT, 1),
    }
    del ws, V
    torch.cuda.empty_cache()
    legs = [x for x in args.legs.split(",") if x]
    forms = {}
    if "storage" in legs:
        log("storage forms at 512^3")
        forms["storage_512"] = leg_storage(torch, lib, fields, synth)
    if "storage_error" in legs:
        log("storage forms against FP32 at 512^3")
        forms["storage_vs_fp32_512"] = leg_storage_vs_fp32(torch, lib, fields, synth)
        torch.cuda.empty_cache()
    if "storage_oracle" in legs:
        log("storage forms against the FP64 oracle at 128^3")
        forms["storage_vs_oracle_128"] = leg_storage_vs_oracle(torch, lib, fields, synth)
        torch.cuda.empty_cache()
    if "adjoint" in legs:
        log("adjoint gradient at 256^3")
        forms["adjoint_256"] = leg_adjoint(torch, lib, fields, synth)
    if "paper" in legs:
        log("the paper's timing workload")
        forms["paper_workload"] = leg_paper(torch, lib, fields, synth)
        torch.cuda.empty_cache()
    if "fused" in legs:
        log("two steps per sweep")
        forms["fused"] = leg_fused(torch, lib, fields, synth)
        torch.cuda.empty_cache()
    if "pml" in legs:
        log("absorbing layer")
        forms["pml"] = leg_pml(torch, lib, fields, synth)
        torch.cuda.empty_cache()
    if "suite" in legs:
        log("stencil suite")
        forms["suite"] = leg_suite(torch, lib, fields, synth)
    elif "apply" in legs:                  # the 25-point apply alone (counter runs)
        log("25-point apply")
        forms["apply"] = leg_suite(torch, lib, fields, synth, apply_only=True)
    if "serve" in legs:
        log("served shot stream")
        torch.cuda.empty_cache()
        forms["serve"] = leg_serve(torch, lib, fields, synth)
    if forms:
        out["forms"] = forms
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline()
        if forms:
            c0, adj, adj256, st512 = oracle_small_and_adjoint(synth)
            if "suite" in forms or "apply" in forms:
                forms["suite" if "suite" in forms else "apply"]["apply25_64^3_latency"]["oracle"] = c0
            if "adjoint_256" in forms:
                forms["adjoint_256"]["oracle_48"] = adj
                forms["adjoint_256"]["oracle_256"] = adj256
            if "storage_512" in forms:
                forms["storage_512"]["oracle"] = st512
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

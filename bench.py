"""Benchmark: SSP-RK3 steps of the gradient-based-reconstruction solver on the
13M-cell jet-shaped workload, one MI355X.

A step is one full pass of the hot path: the CFL reduction, then three
RHS evaluations (cell gradients and Ducros sensor, xi/eta/zeta interface
sweeps with characteristic MP reconstruction, HLLC and alpha-damping
viscous flux) each followed by an SSP-RK3 stage. Inputs (grid metrics and
the state) are resident in HBM before timing starts.

The headline roofline is one RHS evaluation against its algorithmic bytes
(Q in, interface metrics in, Res out, and the sensor's cell metrics: 440 B
per cell for 3-D Navier-Stokes in FP64), next to the counter-measured bytes
and the bandwidth a streaming triad reaches on the same device. Further legs:
FP32-bulk and MIG4 on the same workload, the bounded spatial jet, the
deforming 128^3 grid, the batched many-grid workload, the serving loop, and
the CPU oracle on the host (all threads and one).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-batch]
                  [--no-bounded] [--no-serve]

Prints ONE JSON line on stdout (everything else goes to stderr).
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

NI, NJ, NK = 400, 180, 180
PARAMS = dict(viscous=True, limiter="ducros", theta_c=0.5, Re=1.144e6, Mref=1.0)
CFL = 0.2
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
PAPER_CONTEXT = {
    "cell_rhs_per_s": 1.26e8,
    "source": "derived from the paper's 34.5 h for 13M cells x 400,000 SSP-RK3 steps on one A100 "
              "(FP64, MEG6 + alpha-damping, real jet with sponge/BCs); context, not this workload",
}

# Algorithmic bytes per cell per RHS evaluation: what any implementation
# must move between HBM and the chip for one RHS, i.e. Q in, the interface
# metrics of the three face families in, Res out; the Ducros sensor adds the
# nine cell metrics it needs and a moving grid the temporal face metrics.
def alg_bytes_per_cell_rhs(ndim=3, viscous=True, sensor=True, moving=False, fp32_res=False):
    nvar = ndim + 2
    per_family = ndim if not viscous else ndim + ndim * ndim  # hatted + unhatted face metrics
    b = nvar * 8 + ndim * per_family * 8 + nvar * (4 if fp32_res else 8)
    if sensor:
        b += ndim * ndim * 8
    if moving:
        b += ndim * 8
    return b


ALG_BYTES_PER_CELL_RHS = alg_bytes_per_cell_rhs()  # 440 B: 3-D NS, FP64, static, sensor on

# Bytes per cell each kernel class of this implementation moves when every
# one of its inputs is read once and every output written once, counting the
# intermediates this design keeps in HBM (primitives, the 12 cell gradients,
# theta, Res between sweeps, the stage buffers). These are the
# implementation's own bytes, reported per kernel beside the measured
# counter traffic; the headline roofline uses the algorithmic bytes above.
IMPL_BYTES_PER_CELL = {
    "prims": 40 + 48,                     # Q -> rho, u, v, w, p, T
    "cell_grad": 32 + 72 + 96 + 1,        # u, v, w, T, 9 cell metrics -> 12 gradients, sensor flag
    # the sweeps run zeta, eta, xi: zeta writes Res, eta adds to it, and xi,
    # last, applies the SSP-RK3 stage
    "sweep_zeta": 40 + 96 + 64 + 8 + 1 + 40,  # 5 primitives (T formed from rho, p), 12 face
                                              # metrics, 8 tangential grads, T', sensor flag
                                              # -> Res out
    "sweep_eta": 40 + 96 + 64 + 8 + 1 + 80,   # ... Res in and out
    # with the stage fused: Res in; Q, Qn, J in ((1/J)_t too on moving
    # grids); Q out; the next stage's primitives out in two of the three
    # stages
    "sweep_xi": 40 + 96 + 64 + 8 + 1 + 40 + 88 + 40 + (2 * 48) / 3,
    "rk_stage": 40 + 80 + 40 + 8 + 8,     # Qn, Q in/out, Res, J, (1/J)_t
    # gbr_step forms the first stage's primitives in the time-step pass
    "cfl": 40 + 72 + 48,                  # Q, 9 cell metrics (temporal ones: moving grids only) -> primitives
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest():
    h = hashlib.sha256()
    for f in ("gbr_rhs.hip", "gbr_device.hpp", "gbr_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2303_10785_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes per launch of each kernel class from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a streaming-kernel
    calibration), or None if absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_jet13m.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_digest") != source_digest():
        return None
    out = {}
    for k, v in vals.items():
        if k.endswith("_bytes_per_launch") and not k.endswith("_alg_bytes_per_launch"):
            out[k[: -len("_bytes_per_launch")]] = float(v)
    return out


def triad_probe(dev, n=1 << 26, reps=20):
    """Achievable HBM bandwidth: the library's STREAM-triad probe a = b + s c
    over three arrays of n doubles (24 n bytes per launch), best of reps
    launches timed with events on the current stream."""
    import torch

    from paper_2303_10785_amd import gbr

    a = torch.empty(n, dtype=torch.float64, device=dev)
    b = torch.rand(n, dtype=torch.float64, device=dev)
    c = torch.rand(n, dtype=torch.float64, device=dev)
    for _ in range(3):
        gbr.gbr_probe_triad(a, b, c, 0.5)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        gbr.gbr_probe_triad(a, b, c, 0.5)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    ok = bool(torch.equal(a[:4096], b[:4096] + 0.5 * c[:4096]))
    del a, b, c
    torch.cuda.empty_cache()
    gbs = 24.0 * n / best / 1e9
    log(f"bench: triad probe {gbs:.0f} GB/s ({24 * n / 2**30:.2f} GiB per launch, best of {reps})")
    return {"GBps": gbs, "bytes_per_launch": 24 * n, "best_ms": best * 1e3, "check": ok}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(grid, Q):
    """The oracle as it stands, timed for one RHS evaluation of the full
    workload (its metrics computed beforehand, not timed) on every host thread
    the process may use and on one thread."""
    import oracle

    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    oracle.set_num_threads(threads)
    log(f"cpu baseline: oracle metrics on {NI}x{NJ}x{NK} ({threads} threads)")
    m = oracle.metrics(grid, **PARAMS)
    ncell = NI * NJ * NK
    log("cpu baseline: timing one oracle RHS on all threads")
    t0 = time.perf_counter()
    oracle.rhs(grid, m, Q, **PARAMS)
    t = time.perf_counter() - t0
    log("cpu baseline: timing one oracle RHS on one thread")
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    oracle.rhs(grid, m, Q, **PARAMS)
    t1 = time.perf_counter() - t0
    oracle.set_num_threads(threads)
    log(f"cpu baseline: {t:.2f} s on {threads} threads, {t1:.2f} s on one")
    return {"value": ncell / t, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"one RHS evaluation of the full {NI}x{NJ}x{NK} jet workload "
                      f"(NS, Ducros-gated MP, FP64), metrics precomputed; {t:.2f} s on {threads} threads",
            "single_core": {"value": ncell / t1, "unit": "cell-updates/s", "cores": 1, "seconds": t1},
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0))}


def fp32_bulk_leg(G64, grid, Q0, args, dev, ncell):
    import torch

    from paper_2303_10785_amd import gbr

    Q = torch.from_numpy(Q0).to(dev)
    r64 = torch.empty_like(Q)
    G64.rhs(Q, r64)
    G = gbr.Grid(grid, precision="fp32_bulk", **PARAMS)
    G.metrics(torch.from_numpy(grid["xyz"]).to(dev))
    r32 = torch.empty(Q.shape, dtype=torch.float32, device=dev)
    G.rhs(Q, r32)
    torch.cuda.synchronize()
    err = 0.0
    for v in range(Q.shape[0]):
        s = r64[v].abs().max().item()
        err = max(err, (r32[v].double() - r64[v]).abs().max().item() / s)
    del r64, r32
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        G.step(Q, CFL, gbr.GBR_DT_CFL, dt_out=dt)
    gbr.gbr_timing_enable(G.h, True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        G.step(Q, CFL, gbr.GBR_DT_CFL, dt_out=dt)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    kern = gbr.gbr_timing_collect(G.h)
    gbr.gbr_timing_enable(G.h, False)
    state = G.check_state()
    G.close()
    log(f"bench fp32-bulk: {ms:.3f} ms/step, one-RHS max rel err vs FP64 {err:.3e}")
    return {"ms_per_step": ms, "value": ncell * 3 / (ms * 1e-3), "unit": "cell-updates/s",
            "rhs_max_rel_err_vs_fp64": err, "state_ok": state == gbr.GBR_OK,
            "kernels_ms_per_launch": {k: v[0] / v[1] for k, v in kern.items() if v[1]}}


def mig4_leg(grid, Q0, args, dev, ncell):
    """The same jet workload with the MIG4 scheme (IG4 gradients and
    IG4-based metrics): step time and kernel breakdown."""
    import torch

    from paper_2303_10785_amd import gbr

    G = gbr.Grid(grid, scheme="mig4", **PARAMS)
    gbr.gbr_timing_enable(G.h, True)
    G.metrics(torch.from_numpy(grid["xyz"]).to(dev))
    metrics_ms = gbr.gbr_timing_collect(G.h)["metrics"][0]
    Q = torch.from_numpy(Q0).to(dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        G.step(Q, CFL, gbr.GBR_DT_CFL, dt_out=dt)
    gbr.gbr_timing_collect(G.h)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        G.step(Q, CFL, gbr.GBR_DT_CFL, dt_out=dt)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    kern = gbr.gbr_timing_collect(G.h)
    state = G.check_state()
    G.close()
    log(f"bench mig4: {ms:.3f} ms/step, metrics {metrics_ms:.1f} ms")
    return {"ms_per_step": ms, "value": ncell * 3 / (ms * 1e-3), "unit": "cell-updates/s", "dtype": "f64",
            "metrics_ms": metrics_ms, "state_ok": state == gbr.GBR_OK,
            "kernels_ms_per_launch": {k: v[0] / v[1] for k, v in kern.items() if v[1]}}


def bounded_leg(args, dev):
    """Spatial jet with boundaries (Sec. 6, App. C, Sec. 8.3): the jet grid
    with 6 ghost layers on each side of every direction (the same 400x180x180
    interior cells), Dirichlet inflow on the xi-low side (the jet state held
    in its ghost cells), zero-gradient outflow on the other five sides with
    sponge layers 20 cells deep (sigma_max 2, quadratic) relaxing to the
    ambient state; same physics and CFL as the periodic workload. Step time,
    interior cell-updates/s and the boundary kernels' share."""
    import torch

    import workloads as W
    from paper_2303_10785_amd import gbr
    ng = W.NG
    g = W.bounded(W.jet3d((NI + 2 * ng, NJ + 2 * ng, NK + 2 * ng)),
                  [("inflow", "outflow"), ("outflow", "outflow"), ("outflow", "outflow")])
    Q0 = W.jet_ic(g)
    sig = W.sponge_sigma(g, width=20, amp=2.0, power=2.0, sides=[(0, 1), (1, 0), (1, 1), (2, 0), (2, 1)])
    G = gbr.Grid(g, **PARAMS)
    gbr.gbr_timing_enable(G.h, True)
    G.metrics(torch.from_numpy(g["xyz"]).to(dev))
    metrics_ms = gbr.gbr_timing_collect(G.h)["metrics"][0]
    G.set_sponge(torch.from_numpy(sig).to(dev), (1.0, 0.0, 0.0, 0.0, 1.0 / 1.4))
    Q = torch.from_numpy(Q0).to(dev)
    del Q0, sig
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        G.step(Q, CFL, gbr.GBR_DT_CFL, dt_out=dt)
    gbr.gbr_timing_collect(G.h)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        G.step(Q, CFL, gbr.GBR_DT_CFL, dt_out=dt)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / args.steps
    kern = gbr.gbr_timing_collect(G.h)
    state = G.check_state()
    G.close()
    interior = NI * NJ * NK
    log(f"bench bounded: {ms:.3f} ms/step, metrics {metrics_ms:.1f} ms")
    return {"workload": f"bounded jet, {NI}x{NJ}x{NK} interior cells + {ng} ghost layers per side, "
                        "inflow / zero-gradient outflow, sponge layers 20 cells",
            "ms_per_step": ms, "value": interior * 3 / (ms * 1e-3), "unit": "interior cell-updates/s",
            "dtype": "f64", "metrics_ms": metrics_ms, "state_ok": state == gbr.GBR_OK,
            "kernels_ms_per_launch": {k: v[0] / v[1] for k, v in kern.items() if v[1]},
            "kernels_ms_per_step": {k: v[0] / args.steps for k, v in kern.items() if v[1]}}


def moving_leg(args, dev):
    """Deforming-grid workload (Sec. 8.2): the 128^3 sinusoidally deforming
    grid (A = 1.5, L = 12, n = 4, omega = 1, seeded +-0.2-cell node noise),
    3-D Navier-Stokes, Re 1e4, MP limiter, uniform M = 0.5 flow, CFL 0.2;
    every step recomputes the metrics, temporal metrics and GCL rate at t^n
    from device-side coordinates. Step time, the metrics' share and the
    freestream drift max |v|, |w| after the timed steps."""
    import math

    import torch

    import workloads as W
    from paper_2303_10785_amd import gbr
    n = 128
    mv = W.Deforming3D((n, n, n), L=12.0, A=1.5, nmode=4, omega=1.0, rand=0.2, seed=7)
    params = dict(viscous=True, limiter="mp", Re=1e4, Mref=0.5)
    g0 = mv.at(0.0)
    Q = torch.from_numpy(W.uniform_flow(g0, 1.0, 1.0, 0.0, 0.0, 1.0 / (1.4 * 0.25))).to(dev)
    G = gbr.Grid(g0, **params)
    base = torch.from_numpy(mv.base).to(dev)
    mode = torch.from_numpy(mv.mode).to(dev)
    w = 2 * math.pi * mv.omega
    t = torch.zeros(1, dtype=torch.float64, device=dev)  # mesh time, kept on the device

    def step():
        G.step(Q, 0.2, gbr.GBR_DT_CFL, xyz=base + torch.sin(w * t) * mode,
               xyz_t=(w * torch.cos(w * t)) * mode, t=t)  # the library advances t by dt

    for _ in range(args.warmup):
        step()
    gbr.gbr_timing_enable(G.h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    kern = gbr.gbr_timing_collect(G.h)
    state = G.check_state()
    G.close()
    q = Q.cpu().numpy()
    drift = float(max(abs(q[2] / q[0]).max(), abs(q[3] / q[0]).max()))
    ncell = n ** 3
    log(f"bench moving: {ms:.3f} ms/step, drift {drift:.2e}")
    return {"workload": "128^3 deforming grid, metrics every step, 3-D Navier-Stokes freestream, MP, CFL 0.2",
            "ms_per_step": ms, "value": ncell * 3 / (ms * 1e-3), "unit": "cell-updates/s", "dtype": "f64",
            "metrics_ms_per_step": kern.get("metrics", (0.0, 0))[0] / args.steps,
            "freestream_max_v_w": drift, "state_ok": state == gbr.GBR_OK,
            "note": "the mesh coordinates and velocities are formed on the device each step (two "
                    "elementwise torch passes, included in the step time)"}


BATCH_STEPS = 100
BATCH_CFL = 0.4


def batched_leg(dev, per_solve_leg=True):
    """Many-small-grids workload: 256 periodic wavy 2-D Euler grids of
    32^2..512^2 cells (vortex / Sod-vortex states), MP limiter, CFL 0.4 per
    grid, 100 SSP-RK3 steps each. Timed as one batch (graph replay, tile
    autotuned) in FP32-bulk and FP64, and as 256 separate FP64 solves through
    gbr_step; the FP32-bulk results are compared per problem with the FP64
    ones."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2303_10785_amd import gbr

    t0 = time.perf_counter()
    cases = W.batch2d()
    cells = sum(g["n"][0] * g["n"][1] for g, _, _ in cases)
    log(f"bench batched: {len(cases)} grids, {cells} cells, generated in {time.perf_counter() - t0:.1f}s")

    def grids_for(precision):
        hs = []
        for g, _, _ in cases:
            h = gbr.Grid(g, precision=precision, viscous=False, limiter="mp")
            h.metrics(torch.from_numpy(g["xyz"]).to(dev))
            hs.append(h)
        return hs

    def states():
        return [torch.from_numpy(Q).to(dev) for _, Q, _ in cases]

    def timed(fn):
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        fn()
        stop.record()
        torch.cuda.synchronize()
        return start.elapsed_time(stop) * 1e-3

    out = {"workload": f"{len(cases)} periodic wavy 2-D Euler grids, N^2 cells with N = round(2^U(5,9)) "
                       f"({cells} cells total), Shu vortex / Sod+vortex, MP limiter, "
                       f"{BATCH_STEPS} SSP-RK3 steps each at CFL {BATCH_CFL}",
           "grids": len(cases), "cells": cells, "steps_per_solve": BATCH_STEPS}
    finals = {}
    for precision in ("fp32_bulk", "fp64"):
        hs = grids_for(precision)
        Qs = states()
        B = gbr.Batch(hs, Qs, tile=gbr.GBR_TILE_AUTO)
        B.run(1, BATCH_CFL)  # captures the step graph
        for q, (_, Q, _) in enumerate(cases):
            Qs[q].copy_(torch.from_numpy(Q))
        torch.cuda.synchronize()
        sec = timed(lambda: B.run(BATCH_STEPS, BATCH_CFL))
        _, _, tile = B.query()
        ok = all(h.check_state() == gbr.GBR_OK for h in hs)
        finals[precision] = [x.cpu().numpy() for x in Qs]
        out[f"batched_{precision}"] = {
            "seconds": sec, "solves_per_s": len(cases) / sec,
            "cell_updates_per_s": cells * 3 * BATCH_STEPS / sec, "tile": gbr.TILE_NAMES[tile],
            "state_ok": ok}
        log(f"bench batched {precision}: {sec:.3f} s, {len(cases) / sec:.1f} solves/s, tile {gbr.TILE_NAMES[tile]}")
        B.close()
        if precision == "fp64" and per_solve_leg:
            # the same 256 problems solved one after another through gbr_step
            Qs = states()
            dt = torch.zeros(1, dtype=torch.float64, device=dev)

            def per_solve():
                for h, Q in zip(hs, Qs):
                    for _ in range(BATCH_STEPS):
                        h.step(Q, BATCH_CFL, gbr.GBR_DT_CFL, dt_out=dt)
            sec1 = timed(per_solve)
            ok1 = all(h.check_state() == gbr.GBR_OK for h in hs)
            dev64 = max(float(np.abs(Q.cpu().numpy() - f).max() / max(np.abs(f).max(), 1e-300))
                        for Q, f in zip(Qs, finals["fp64"]))
            out["per_solve_fp64"] = {"seconds": sec1, "solves_per_s": len(cases) / sec1,
                                     "cell_updates_per_s": cells * 3 * BATCH_STEPS / sec1,
                                     "state_ok": ok1, "max_rel_diff_vs_batched_fp64": dev64}
            log(f"bench per-solve fp64: {sec1:.3f} s, {len(cases) / sec1:.1f} solves/s")
        for h in hs:
            h.close()
        del Qs
        torch.cuda.empty_cache()
    errs = []
    for a, b in zip(finals["fp32_bulk"], finals["fp64"]):
        errs.append(max(float(np.abs(a[v] - b[v]).max() / np.abs(b[v]).max()) for v in range(b.shape[0])))
    out["fp32_vs_fp64_per_problem_max_rel_err"] = {"max": max(errs), "median": float(np.median(errs))}
    if per_solve_leg:
        out["speedup_batched_fp32_vs_per_solve_fp64"] = (out["batched_fp32_bulk"]["solves_per_s"]
                                                         / out["per_solve_fp64"]["solves_per_s"])
    return out


SERVE_BURST = 30
SERVE_PACED = 80


def serving_leg(dev):
    """Serving workload (Poisson stream of 2-D 64^2..1024^2 and 3-D
    64^3..256^3 wavy-grid Euler requests, 20..500 SSP-RK3 steps each, FP64 or
    FP32-bulk, admitted against 0.8 x the free HBM), bounded in time: the first
    SERVE_BURST requests of the seeded trace arrive at once to measure the
    served capacity, then the first SERVE_PACED requests arrive at the
    trace's own Poisson times rescaled so that the offered load is 0.8 x that
    capacity. Reports latency and queue-wait percentiles, solves/s and
    offered against achieved cell-updates/s for the paced run."""
    import torch

    from paper_2303_10785_amd import serve

    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    trace = serve.make_trace(SERVE_PACED)
    ex = serve.GpuExecutor()
    t0 = time.perf_counter()
    burst = serve.run(serve.rescale(trace[:SERVE_BURST], 1e9), ex, budget, log=log)
    cap = burst["achieved_cell_updates_per_s"]
    log(f"bench serving: burst of {SERVE_BURST} in {time.perf_counter() - t0:.1f} s, capacity {cap:.3e} cell-RHS/s")
    offered = sum(r.work for r in trace) / max(r.arrival for r in trace)
    factor = 0.8 * cap / offered
    t0 = time.perf_counter()
    paced = serve.run(serve.rescale(trace, factor), ex, budget, log=log)
    ex.close()
    log(f"bench serving: paced {SERVE_PACED} requests in {time.perf_counter() - t0:.1f} s, "
        f"p50/p99 latency {paced['latency_p50_s']:.2f}/{paced['latency_p99_s']:.2f} s")
    return {"workload": f"Poisson trace (seed 5) of 2-D 64^2..1024^2 / 3-D 64^3..256^3 wavy-grid Euler requests, "
                        f"20..500 SSP-RK3 steps, FP64 or FP32-bulk, HBM budget 0.8 x free",
            "budget_bytes": budget,
            "capacity_burst": dict(burst, requests_in_burst=SERVE_BURST),
            "paced": dict(paced, rate_per_s=50.0 * factor, offered_over_capacity=0.8),
            "latency_p50_s": paced["latency_p50_s"], "latency_p99_s": paced["latency_p99_s"],
            "queue_wait_p50_s": paced["queue_wait_p50_s"], "queue_wait_p99_s": paced["queue_wait_p99_s"],
            "solves_per_s": paced["solves_per_s"],
            "offered_cell_updates_per_s": paced["offered_cell_updates_per_s"],
            "achieved_cell_updates_per_s": paced["achieved_cell_updates_per_s"],
            "all_states_ok": burst["all_states_ok"] and paced["all_states_ok"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched many-grid leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-per-solve", action="store_true",
                    help="skip the batched leg's comparison with 256 separate gbr_step solves (counter "
                         "runs of the batched kernels, where its many small launches dominate)")
    ap.add_argument("--no-bounded", action="store_true",
                    help="skip the bounded spatial-jet and deforming-grid legs (they launch the same kernels "
                         "at other sizes, so profiles of the periodic workload leave them out)")
    args = ap.parse_args()
    if args.gpus != 1:
        log(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
            "(the build targets a single MI355X; multi-GPU sharding is a design note).")
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2303_10785_amd import gbr

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"bench: generating {NI}x{NJ}x{NK} jet grid and state")
    grid = W.jet3d((NI, NJ, NK))
    Q0 = W.jet_ic(grid)
    G = gbr.Grid(grid, **PARAMS)
    xyz = torch.from_numpy(grid["xyz"]).to(dev)
    G.metrics(xyz)
    del xyz
    Q = torch.from_numpy(Q0).to(dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    ncell = NI * NJ * NK

    # a streaming pass over the state (518 MB read, 518 MB written, outside
    # the timed region; torch's elementwise negation, a copy with a sign
    # flip): the calibration kernel for the HBM counter runs of profiles/
    calib = torch.neg(Q)
    del calib
    log(f"bench: {args.warmup} warmup steps")
    for _ in range(args.warmup):
        G.step(Q, CFL, gbr.GBR_DT_CFL, dt_out=dt)
    torch.cuda.synchronize()
    if G.check_state() != gbr.GBR_OK:
        raise RuntimeError("non-physical state during warmup")

    log(f"bench: timing {args.steps} steps")
    gbr.gbr_timing_enable(G.h, True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        G.step(Q, CFL, gbr.GBR_DT_CFL, dt_out=dt)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(stop)
    kern = gbr.gbr_timing_collect(G.h)
    # diagnostics of the final state (vorticity, Q-criterion, |grad rho|, KE and
    # enstrophy averages), timed separately from the steps
    fields = torch.empty((5, NK, NJ, NI), dtype=torch.float64, device=dev)
    integ = torch.empty(3, dtype=torch.float64, device=dev)
    G.diagnostics(Q, fields, integ)
    diag = gbr.gbr_timing_collect(G.h)["diagnostics"]
    diag_ms = diag[0] / max(diag[1], 1)
    del fields
    gbr.gbr_timing_enable(G.h, False)
    state = G.check_state()
    if state != gbr.GBR_OK:
        raise RuntimeError(f"non-physical state in the timed steps ({state})")
    ms_per_step = ms_total / args.steps
    value = ncell * 3 * args.steps / (ms_total * 1e-3)
    log(f"bench: {ms_per_step:.3f} ms/step (wall {1e3 * wall / args.steps:.3f}), "
        f"{value:.4e} cell-RHS/s, dt {dt.item():.4e}")

    breakdown = {}
    for k, (ms, cnt) in kern.items():
        if cnt:
            breakdown[k] = {"ms_per_launch": ms / cnt, "launches_per_step": cnt / args.steps,
                            "share": ms / ms_total}
    # headline roofline: one RHS evaluation (gradients and the three sweeps,
    # with a third of the step's time-step pass) against the algorithmic
    # bytes per cell-RHS; its duration is the timed step over three
    traffic = read_traffic()
    rhs_s = ms_per_step * 1e-3 / 3
    achieved = ALG_BYTES_PER_CELL_RHS * ncell / rhs_s / 1e9
    measured = None
    if traffic is not None and all(k in traffic for k in breakdown if k in IMPL_BYTES_PER_CELL):
        measured = sum(traffic[k] * b["launches_per_step"] for k, b in breakdown.items()
                       if k in IMPL_BYTES_PER_CELL) / 3
    for k, b in breakdown.items():
        if k in IMPL_BYTES_PER_CELL:
            b["impl_bytes_per_cell"] = IMPL_BYTES_PER_CELL[k]
            b["impl_GBps"] = IMPL_BYTES_PER_CELL[k] * ncell / (b["ms_per_launch"] * 1e-3) / 1e9
            b["impl_frac"] = b["impl_GBps"] / HBM_PEAK_GBS
            if traffic is not None and k in traffic:
                b["measured_bytes_per_launch"] = traffic[k]
                b["measured_GBps"] = traffic[k] / (b["ms_per_launch"] * 1e-3) / 1e9
    triad = triad_probe(dev)
    roofline = {"bound": "hbm", "kernel": "rhs (cell gradients + zeta, eta, xi sweeps, 1/3 of the time-step pass)",
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured,
                "alg_bytes_per_cell_rhs": ALG_BYTES_PER_CELL_RHS, "alg_bytes_per_launch": ALG_BYTES_PER_CELL_RHS * ncell,
                "ms_per_launch": rhs_s * 1e3,
                "measured_bytes_per_cell_rhs": measured / ncell if measured is not None else None,
                "measured_GBps": measured / rhs_s / 1e9 if measured is not None else None,
                "achievable": triad["GBps"], "frac_of_achievable": achieved / triad["GBps"],
                "achievable_probe": "STREAM triad a = b + s c over 3 x 2^26 doubles (gbr_probe_triad)"}

    # FP32-bulk on the same workload: step time and the error of one RHS
    # against the FP64 path (which matches the oracle to 1e-12)
    fp32 = fp32_bulk_leg(G, grid, Q0, args, dev, ncell)
    mig4 = mig4_leg(grid, Q0, args, dev, ncell)
    bounded = None if args.no_bounded else bounded_leg(args, dev)
    moving = None if args.no_bounded else moving_leg(args, dev)

    line = {
        "metric": "cell-updates/s per RHS at 13M cells (% HBM peak); batched solves/s + p99 latency",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded jet-shaped grid and tanh jet state with 1% velocity noise)",
        "config": {"workload": f"jet-shaped stretched periodic curvilinear grid {NI}x{NJ}x{NK} "
                               f"({ncell} cells), 3-D Navier-Stokes with alpha-damping, "
                               f"Ducros-gated MP limiter, HLLC, SSP-RK3 at CFL {CFL}, FP64",
                   "cells": ncell, "rhs_per_step": 3},
        "roofline": roofline,
        "kernels": breakdown,
        "fp32_bulk": fp32,
        "mig4": mig4,
        "bounded": bounded,
        "moving": moving,
        "diagnostics": {"ms": diag_ms, "kinetic_energy": float(integ[0]), "enstrophy": float(integ[1]),
                        "volume": float(integ[2])},
        "paper_context": PAPER_CONTEXT,
    }
    G.close()
    del Q
    torch.cuda.empty_cache()
    line["batched"] = None if args.no_batch else batched_leg(dev, per_solve_leg=not args.no_per_solve)
    torch.cuda.empty_cache()
    line["serving"] = None if args.no_serve else serving_leg(dev)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(grid, Q0)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Serving loop for many independent solve requests on one GPU.

A request asks for ``steps`` SSP-RK3 steps of one periodic grid (2-D or 3-D
Euler with the MP limiter, FP64 or FP32-bulk). Requests arrive as a Poisson
stream; the server

* admits them first-in first-out while their device bytes (``gbr_grid_bytes``
  plus the state and the transient coordinates) fit an HBM budget,
* runs every admitted request in a group with a HIP stream of its own: the
  2-D requests of one precision form one continuous batch (``gbr_batch``),
  each 3-D request steps through ``gbr_step``. Groups advance independently
  and overlap on the device: whenever a group's last launch has completed
  (polled through an event, never by synchronising the device), its finished
  members retire and it is relaunched with its current members for the
  smallest remaining step count of them (capped), so no request overshoots
  and a 2-D request that arrived meanwhile joins its batch at that boundary,
* retires finished requests, releases their bytes and records latency.

The scheduling logic (``Scheduler``, ``run``) is plain Python and is tested
on the CPU with a simulated executor; ``GpuExecutor`` drives the C ABI.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

GAMMA = 1.4
CFL_2D = 0.4
CFL_3D = 0.2
TICK_STEPS = 25  # largest number of steps a group advances per tick


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds from the start of the trace
    ndim: int
    n: int                  # cells per side
    steps: int
    precision: str          # "fp64" or "fp32_bulk"
    ic: str                 # "vortex", "sod" (2-D) or "column" (3-D)
    seed: int
    # filled in by the server
    bytes: int = 0
    admitted: float | None = None
    done: float | None = None
    remaining: int = 0
    state_ok: bool | None = None

    @property
    def ncell(self):
        return self.n ** self.ndim

    @property
    def nvar(self):
        return self.ndim + 2

    @property
    def work(self):
        """Cell-RHS evaluations the request asks for."""
        return self.ncell * 3 * self.steps

    @property
    def group(self):
        return ("2d", self.precision) if self.ndim == 2 else ("3d", self.rid)


def make_trace(count=600, rate=50.0, seed=5, p2d=0.5, n2d=(64, 1024), n3d=(64, 256), steps=(20, 500),
               p_fp32=0.5):
    """Poisson arrivals at ``rate`` per second; 2-D with probability p2d and N
    log-uniform in n2d, else 3-D with N log-uniform in n3d; steps uniform in
    the closed range; FP32-bulk with probability p_fp32; 2-D states split
    between vortex and Sod+vortex."""
    rng = np.random.default_rng(2303_10785 + seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += float(rng.exponential(1.0 / rate))
        two = rng.uniform() < p2d
        lo, hi = n2d if two else n3d
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        st = int(rng.integers(steps[0], steps[1] + 1))
        prec = "fp32_bulk" if rng.uniform() < p_fp32 else "fp64"
        ic = ("vortex" if rng.uniform() < 0.5 else "sod") if two else "column"
        out.append(Request(rid, t, 2 if two else 3, n, st, prec, ic, int(rng.integers(1 << 30))))
    return out


def rescale(trace, factor):
    """The same requests with arrival times divided by ``factor`` (rate x factor)."""
    return [dataclasses.replace(r, arrival=r.arrival / factor) for r in trace]


def percentile(xs, q):
    if not xs:
        return None
    return float(np.percentile(np.asarray(xs, dtype=float), q))


class Scheduler:
    """FIFO admission under a byte budget and per-group tick planning."""

    def __init__(self, budget_bytes, bytes_of, tick_steps=TICK_STEPS):
        self.budget = int(budget_bytes)
        self.bytes_of = bytes_of
        self.tick_steps = int(tick_steps)
        self.used = 0
        self.queue = []      # arrived, not admitted (FIFO)
        self.active = {}     # rid -> Request
        self.finished = []

    def arrive(self, req):
        req.bytes = int(self.bytes_of(req))
        if req.bytes > self.budget:
            raise ValueError(f"request {req.rid} needs {req.bytes} B, more than the whole budget")
        req.remaining = req.steps
        self.queue.append(req)

    def admit(self, now):
        """Admit queued requests in arrival order while the head fits."""
        out = []
        while self.queue and self.used + self.queue[0].bytes <= self.budget:
            r = self.queue.pop(0)
            r.admitted = now
            self.used += r.bytes
            self.active[r.rid] = r
            out.append(r)
        return out

    def plan(self, busy=()):
        """{group: (steps, rids)} for every group with active members that is
        not in ``busy``: the members advance together by the smallest
        remaining count among them, at most tick_steps."""
        groups = {}
        for r in self.active.values():
            g = r.group
            if g in busy:
                continue
            k, rids = groups.get(g, (self.tick_steps, []))
            groups[g] = (min(k, r.remaining), rids + [r.rid])
        return groups

    def advanced(self, rids, k, now):
        """Record that the requests ``rids`` advanced k steps; returns the
        requests that finished."""
        done = []
        for rid in rids:
            r = self.active[rid]
            r.remaining -= k
            if r.remaining < 0:
                raise RuntimeError(f"request {r.rid} overshot")
            if r.remaining == 0:
                r.done = now
                self.used -= r.bytes
                del self.active[r.rid]
                self.finished.append(r)
                done.append(r)
        return done


def run(trace, executor, budget_bytes, tick_steps=TICK_STEPS, clock=time.perf_counter, sleep=time.sleep,
        log=None, log_every=20.0, poll_s=2e-4):
    """Serve ``trace`` in real time (arrival times relative to the start) and
    drain it. Returns a summary dict. ``log`` (a callable taking a string)
    receives a progress line every ``log_every`` seconds.

    The executor enqueues a group's steps without waiting (``launch``) and
    reports whether they have completed (``done``); the loop admits arrivals,
    retires finished requests and relaunches idle groups as soon as each of
    these becomes possible, and sleeps ``poll_s`` when nothing changed."""
    sched = Scheduler(budget_bytes, executor.bytes_of, tick_steps)
    pending = sorted(trace, key=lambda r: r.arrival)
    t0 = clock()
    launches = 0
    inflight = {}  # group -> (steps, rids) of its launch in flight
    last_log = 0.0
    while pending or sched.queue or sched.active or inflight:
        now = clock() - t0
        if log is not None and now - last_log >= log_every:
            last_log = now
            log(f"[serve] t={now:.1f}s done={len(sched.finished)}/{len(trace)} active={len(sched.active)} "
                f"queued={len(sched.queue)} pending={len(pending)} used={sched.used / 2**30:.1f}GiB")
        progressed = False
        for g in list(inflight):
            if executor.done(g):
                k, rids = inflight.pop(g)
                for r in sched.advanced(rids, k, clock() - t0):
                    r.state_ok = executor.retire(r)
                progressed = True
        while pending and pending[0].arrival <= now:
            sched.arrive(pending.pop(0))
        for r in sched.admit(clock() - t0):
            executor.admit(r)
            progressed = True
        for g, (k, rids) in sched.plan(busy=inflight).items():
            executor.launch(g, rids, k)
            inflight[g] = (k, rids)
            launches += 1
            progressed = True
        if not progressed:
            wait = poll_s
            if not inflight and pending:
                wait = max(poll_s, min(pending[0].arrival - (clock() - t0), 0.05))
            sleep(wait)
    makespan = clock() - t0
    fin = sched.finished
    lat = [r.done - r.arrival for r in fin]
    wait = [r.admitted - r.arrival for r in fin]
    span = max(r.arrival for r in trace) if trace else 0.0
    work = sum(r.work for r in fin)
    return {
        "requests": len(fin),
        "launches": launches,
        "makespan_s": makespan,
        "trace_span_s": span,
        "latency_p50_s": percentile(lat, 50),
        "latency_p99_s": percentile(lat, 99),
        "queue_wait_p50_s": percentile(wait, 50),
        "queue_wait_p99_s": percentile(wait, 99),
        "solves_per_s": len(fin) / makespan if makespan > 0 else None,
        "offered_cell_updates_per_s": work / span if span > 0 else None,
        "achieved_cell_updates_per_s": work / makespan if makespan > 0 else None,
        "all_states_ok": all(r.state_ok for r in fin),
    }


# ---------------------------------------------------------------------------
# request inputs, generated on the device (no method arithmetic here)
# ---------------------------------------------------------------------------
def _wavy_nodes(torch, n, ndim, L, amp, dev):
    s = torch.arange(n + 1, dtype=torch.float64, device=dev) / n
    if ndim == 2:
        et, xi = torch.meshgrid(s, s, indexing="ij")
        w = torch.sin(2 * math.pi * et) * torch.sin(2 * math.pi * xi)
        return [L * (xi + amp * w), L * (et + amp * w)]
    ze, et, xi = torch.meshgrid(s, s, s, indexing="ij")
    sx, sy, sz = (torch.sin(2 * math.pi * a) for a in (xi, et, ze))
    return [L * (xi + amp * sy * sz), L * (et + amp * sz * sx), L * (ze + amp * sx * sy)]


def _centroids(nodes, ndim):
    out = []
    for X in nodes:
        if ndim == 2:
            out.append(0.25 * (X[:-1, :-1] + X[:-1, 1:] + X[1:, :-1] + X[1:, 1:]))
        else:
            c = (X[:-1, :-1, :-1] + X[:-1, :-1, 1:] + X[:-1, 1:, :-1] + X[:-1, 1:, 1:]
                 + X[1:, :-1, :-1] + X[1:, :-1, 1:] + X[1:, 1:, :-1] + X[1:, 1:, 1:])
            out.append(0.125 * c)
    return out


def _vortex(torch, x, y, xc, yc, eps, gamma):
    dx, dy = x - xc, y - yc
    f = torch.exp(0.5 * (1.0 - (dx * dx + dy * dy)))
    du = -eps / (2 * math.pi) * f * dy
    dv = eps / (2 * math.pi) * f * dx
    T = 1.0 - (gamma - 1.0) * eps * eps / (8 * gamma * math.pi ** 2) * f * f
    return du, dv, T ** (1.0 / (gamma - 1.0)), T ** (gamma / (gamma - 1.0))


def request_inputs(req, dev, L=10.0):
    """(grid dict for gbr.Grid, coordinates [3][...], conserved state) on ``dev``."""
    import torch

    amp = 0.05
    nodes = _wavy_nodes(torch, req.n, req.ndim, L, amp, dev)
    cen = _centroids(nodes, req.ndim)
    if req.ndim == 2:
        x, y = cen
        xyz = torch.stack([x, y, torch.zeros_like(x)]).reshape(3, 1, req.n, req.n).contiguous()
    else:
        x, y = cen[0], cen[1]
        xyz = torch.stack(cen).contiguous()
    du, dv, rf, pf = _vortex(torch, x, y, 0.5 * L, 0.5 * L, 5.0 if req.ic != "sod" else 2.0, GAMMA)
    if req.ic == "sod":
        left = x < 0.5 * L - 1e-9 * L  # a column on the split takes the right state
        rho = torch.where(left, 1.0, 0.125) * rf
        p = torch.where(left, 1.0, 0.1) * pf
        u, v = du, dv
    else:
        rho, p = rf, pf
        u, v = 1.0 + du, 1.0 + dv
    w = torch.zeros_like(u)
    if req.ic == "column":
        g = torch.Generator(device="cpu").manual_seed(req.seed)
        noise = (torch.rand((3,) + tuple(u.shape), generator=g, dtype=torch.float64) * 2 - 1).to(dev)
        u, v, w = u + 0.01 * noise[0], v + 0.01 * noise[1], w + 0.01 * noise[2]
    E = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    comps = [rho, rho * u, rho * v] + ([rho * w] if req.ndim == 3 else []) + [E]
    Q = torch.stack(comps)
    if req.ndim == 2:
        Q = Q.reshape(4, 1, req.n, req.n)
    Q = Q.contiguous()
    off = [[L, 0.0, 0.0], [0.0, L, 0.0], [0.0, 0.0, L if req.ndim == 3 else 1.0]]
    grid = {"n": (req.n, req.n, req.n if req.ndim == 3 else 1), "ndim": req.ndim, "off": off}
    return grid, xyz, Q


class GpuExecutor:
    """Runs admitted requests through the C ABI on the current device. Each
    2-D batch group has a stream of its own, and so does each active 3-D
    request (taken from a pool that grows on demand); a group's launch ends
    with an event on its stream, which ``done`` polls."""

    def __init__(self, dev=None, tile=None, keep_results=False):
        import torch

        from . import gbr
        self.torch, self.gbr = torch, gbr
        self.dev = dev or torch.device("cuda", torch.cuda.current_device())
        self.tile = tile or {"fp64": gbr.GBR_TILE_16X16, "fp32_bulk": gbr.GBR_TILE_16X16}
        self.keep = keep_results
        self.setup = torch.cuda.Stream(device=self.dev)  # inputs and metrics of new requests
        self.free_streams = []
        self.streams = {}   # group -> stream
        self.live = {}      # rid -> (Grid, Q, req)
        self.batches = {}   # 2-D group -> (Batch, rids)
        self.events = {}    # group -> event of its last launch
        self.results = {}   # rid -> final state (host), if keep_results

    def bytes_of(self, req):
        cfg = self.gbr.make_config((req.n, req.n, req.n if req.ndim == 3 else 1), req.ndim,
                                   [[1, 0, 0], [0, 1, 0], [0, 0, 1]], precision=req.precision)
        return self.gbr.gbr_grid_bytes(cfg) + (req.nvar + 3) * req.ncell * 8

    def _stream_of(self, group):
        if group not in self.streams:
            self.streams[group] = self.free_streams.pop() if self.free_streams else \
                self.torch.cuda.Stream(device=self.dev)
        return self.streams[group]

    def admit(self, req):
        """Inputs and metrics on the setup stream (gbr_metrics waits for that
        stream only), then the grid is rebound to its group's stream."""
        torch = self.torch
        with torch.cuda.stream(self.setup):
            grid, xyz, Q = request_inputs(req, self.dev)
            h = self.gbr.Grid(grid, precision=req.precision, viscous=False, limiter="mp")
            h.metrics(xyz)
            del xyz
        lane = self._stream_of(req.group)
        self.gbr.gbr_set_stream(h.h, lane.cuda_stream)
        self.live[req.rid] = (h, Q, req)

    def launch(self, group, rids, k):
        torch, gbr = self.torch, self.gbr
        lane = self._stream_of(group)
        if group[0] == "3d":
            h, Q, _ = self.live[group[1]]
            for _ in range(k):
                h.step(Q, CFL_3D, gbr.GBR_DT_CFL)
        else:
            rids = sorted(rids)
            if group not in self.batches or self.batches[group][1] != rids:
                self._drop_batch(group)
                b = gbr.Batch([self.live[r][0] for r in rids], [self.live[r][1] for r in rids],
                              tile=self.tile[group[1]])
                self.batches[group] = (b, rids)
            self.batches[group][0].run(k, CFL_2D, gbr.GBR_DT_CFL, graph=True)
        ev = torch.cuda.Event()
        ev.record(lane)
        self.events[group] = ev

    def done(self, group):
        ev = self.events.get(group)
        return ev is None or ev.query()

    def _drop_batch(self, group):
        if group in self.batches:
            self.batches[group][0].close()
            del self.batches[group]

    def retire(self, req):
        h, Q, _ = self.live.pop(req.rid)
        ok = h.check_state() == self.gbr.GBR_OK  # waits for the group's stream (idle here)
        if self.keep:
            with self.torch.cuda.stream(self._stream_of(req.group)):
                self.results[req.rid] = Q.cpu().numpy()
        if req.ndim == 2 and req.group in self.batches and req.rid in self.batches[req.group][1]:
            self._drop_batch(req.group)
        h.close()
        del Q
        if req.ndim == 3:
            self.events.pop(req.group, None)
            self.free_streams.append(self.streams.pop(req.group))
        return ok

    def close(self):
        for g in list(self.batches):
            self._drop_batch(g)
        for rid in list(self.live):
            self.live.pop(rid)[0].close()
        self.torch.cuda.synchronize()


def main(argv=None):
    import argparse
    import json
    import sys

    import torch

    ap = argparse.ArgumentParser(description="Serve a Poisson trace of solve requests on one GPU.")
    ap.add_argument("--requests", type=int, default=600)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--budget-frac", type=float, default=0.8, help="HBM budget as a fraction of free memory")
    ap.add_argument("--n2d", type=int, nargs=2, default=(64, 1024))
    ap.add_argument("--n3d", type=int, nargs=2, default=(64, 256))
    ap.add_argument("--steps", type=int, nargs=2, default=(20, 500))
    ap.add_argument("--paced", action="store_true",
                    help="also replay the trace at 0.8x the capacity measured by the first run")
    a = ap.parse_args(argv)
    free, _ = torch.cuda.mem_get_info()
    budget = int(a.budget_frac * free)
    trace = make_trace(a.requests, a.rate, n2d=tuple(a.n2d), n3d=tuple(a.n3d), steps=tuple(a.steps))
    ex = GpuExecutor()
    out = {"budget_bytes": budget, "trace": {"requests": a.requests, "rate_per_s": a.rate,
                                             "n2d": a.n2d, "n3d": a.n3d, "steps": a.steps}}

    def log(msg):
        print(msg, file=sys.stderr, flush=True)
    out["burst"] = run(trace, ex, budget, log=log)
    print(json.dumps(out["burst"]), flush=True)
    if a.paced:
        cap = out["burst"]["achieved_cell_updates_per_s"]
        offered = out["burst"]["offered_cell_updates_per_s"]
        factor = 0.8 * cap / offered
        out["paced"] = run(rescale(trace, factor), ex, budget, log=log)
        out["paced"]["rate_per_s"] = a.rate * factor
    ex.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

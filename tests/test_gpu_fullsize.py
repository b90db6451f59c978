"""Parity at the full workload sizes, in the launch configuration bench.py
times: the 400x180x180 jet-shaped grid (13M cells) and the 128^3 deforming
Navier-Stokes freestream grid. Every element is compared with the FP64 oracle
(which runs on the host cores); the 100-step freestream property is checked on
the GPU alone.
"""
import time

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = 1e-12
JET = (400, 180, 180)
JET_PARAMS = dict(viscous=True, limiter="ducros", theta_c=0.5, Re=1.144e6, Mref=1.0)
C2_PARAMS = dict(viscous=True, limiter="mp", Re=1e4, Mref=0.5)


@pytest.fixture(scope="module")
def gbr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_10785_amd import gbr as G
    G.lib()
    return G


def say(*a):
    print(*a, flush=True)


def rel_whole(gpu, ref):
    """Max error over the whole RHS relative to its largest component."""
    return float(np.abs(gpu - ref).max()) / float(np.abs(ref).max())


def rel(gpu, ref):
    """Max over variables of the error relative to that variable's scale."""
    worst = 0.0
    for v in range(ref.shape[0]):
        s = float(np.abs(ref[v]).max())
        d = float(np.abs(gpu[v] - ref[v]).max())
        worst = max(worst, d / s if s > 0 else d)
    return worst


@pytest.fixture(scope="module")
def jet(gbr):
    t0 = time.time()
    g = W.jet3d(JET)
    Q = W.jet_ic(g)
    say(f"[jet] generated {JET} in {time.time() - t0:.1f}s; oracle metrics ...")
    m = oracle.metrics(g, **JET_PARAMS)
    say(f"[jet] oracle metrics done at {time.time() - t0:.1f}s")
    h = gbr.Grid(g, **JET_PARAMS)
    h.metrics(torch.from_numpy(g["xyz"]).cuda())
    torch.cuda.synchronize()
    yield g, Q, m, h
    h.close()


def test_jet_metrics_full(gbr, jet):
    g, Q, m, h = jet
    groups = {
        "face_hat": [(oracle.M_FHAT(f, c), gbr.SLOT_FACE_HAT(f, c)) for f in range(3) for c in range(3)],
        "face_unhat": [(oracle.M_FUNHAT(f, e, c), gbr.SLOT_FACE_UNHAT(f, e, c))
                       for f in range(3) for e in range(3) for c in range(3)],
        "cell_unhat": [(oracle.M_UNHAT(e, c), gbr.SLOT_CELL_UNHAT(e, c)) for e in range(3) for c in range(3)],
        "jac": [(oracle.M_J, gbr.SLOT_CELL_J)],
    }
    for name, pairs in groups.items():
        scale = max(float(np.abs(m[o]).max()) for o, _ in pairs)
        worst = 0.0
        for o, s in pairs:
            worst = max(worst, float(np.abs(h.metric(s).cpu().numpy() - m[o]).max()) / scale)
        say(f"[jet metrics] {name}: max rel err {worst:.3e}")
        assert worst <= TOL, name


def test_jet_rhs_full(gbr, jet):
    g, Q, m, h = jet
    Qd = torch.from_numpy(Q).cuda()
    res = torch.empty_like(Qd)
    h.rhs(Qd, res)
    torch.cuda.synchronize()
    assert h.check_state() == gbr.GBR_OK
    t0 = time.time()
    ref = oracle.rhs(g, m, Q, **JET_PARAMS)
    e = rel(res.cpu().numpy(), ref)
    say(f"[jet rhs] 13M cells, oracle {time.time() - t0:.1f}s, max rel err {e:.3e}")
    assert e <= TOL


def test_jet_step_full(gbr, jet):
    """One SSP-RK3 step at CFL 0.2 (the step bench.py times)."""
    g, Q, m, h = jet
    Qd = torch.from_numpy(Q).cuda()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    h.step(Qd, 0.2, gbr.GBR_DT_CFL, dt_out=dt)
    torch.cuda.synchronize()
    q_ref, dt_ref = oracle.step(g, m, Q, 0.2, **JET_PARAMS)
    e = rel(Qd.cpu().numpy(), q_ref)
    say(f"[jet step] max rel err {e:.3e}, dt {dt.item():.6e} vs {dt_ref:.6e}")
    assert e <= TOL
    assert abs(dt.item() - dt_ref) <= TOL * dt_ref


def test_jet_fp32_bulk_full(gbr, jet):
    """FP32-bulk RHS on the full jet workload against the FP64 oracle."""
    g, Q, m, _ = jet
    h = gbr.Grid(g, precision="fp32_bulk", **JET_PARAMS)
    h.metrics(torch.from_numpy(g["xyz"]).cuda())
    Qd = torch.from_numpy(Q).cuda()
    res = torch.empty(Qd.shape, dtype=torch.float32, device="cuda")
    h.rhs(Qd, res)
    torch.cuda.synchronize()
    h.close()
    ref = oracle.rhs(g, m, Q, **JET_PARAMS)
    e = rel(res.double().cpu().numpy(), ref)
    say(f"[jet fp32 rhs] max rel err vs FP64 oracle {e:.3e}")
    assert e <= 2e-4


def _config2():
    return W.Deforming3D((128, 128, 128), L=12.0, A=1.5, nmode=4, omega=1.0, rand=0.2, seed=2)


def test_config2_rhs_full(gbr):
    """128^3 deforming randomized grid, uniform Mach 0.5 NS flow: one RHS
    (dominated by the GCL term) matches the oracle. The rho v and rho w
    components vanish exactly for this flow (both sides hold round-off
    only), so the error is taken relative to the largest RHS component."""
    mv = _config2()
    g = mv.at(0.1)
    pinf = 1.0 / (1.4 * 0.25)
    Q = W.uniform_flow(g, 1.0, 1.0, 0.0, 0.0, pinf)
    h = gbr.Grid(g, **C2_PARAMS)
    h.metrics(torch.from_numpy(g["xyz"]).cuda(), torch.from_numpy(g["xyz_t"]).cuda())
    Qd = torch.from_numpy(Q).cuda()
    res = torch.empty_like(Qd)
    h.rhs(Qd, res)
    torch.cuda.synchronize()
    jac = h.metric(gbr.SLOT_CELL_J).cpu().numpy()
    ijt = h.metric(gbr.SLOT_CELL_INVJT).cpu().numpy()
    h.close()
    m = oracle.metrics(g, **C2_PARAMS)
    ref = oracle.rhs(g, m, Q, **C2_PARAMS)
    got = res.cpu().numpy()
    e = rel_whole(got, ref)
    bal = np.abs(jac * (got - ijt * Q)).max()
    say(f"[config2 rhs] max rel err {e:.3e}; |J (Res - (1/J)_t Q)| max {bal:.3e}")
    assert e <= TOL
    assert bal <= 1e-12


def test_config2_freestream_100_steps(gbr):
    """3-D Navier-Stokes freestream on the 128^3 grid deforming in time
    (dynamic GCL), Re 1e4, 100 SSP-RK3 steps: v and w stay at round-off."""
    mv = _config2()
    pinf = 1.0 / (1.4 * 0.25)
    g0 = mv.at(0.0)
    Q = W.uniform_flow(g0, 1.0, 1.0, 0.0, 0.0, pinf)
    h = gbr.Grid(g0, **C2_PARAMS)
    base = torch.from_numpy(mv.base).cuda()
    mode = torch.from_numpy(mv.mode).cuda()
    Qd = torch.from_numpy(Q).cuda()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    w = 2 * np.pi * mv.omega
    t = 0.0
    t0 = time.time()
    for s in range(100):
        xyz = (base + np.sin(w * t) * mode).contiguous()
        xyz_t = ((w * np.cos(w * t)) * mode).contiguous()
        h.step(Qd, 0.2, gbr.GBR_DT_CFL, xyz=xyz, xyz_t=xyz_t, dt_out=dt)
        t += dt.item()
    torch.cuda.synchronize()
    st = h.check_state()
    h.close()
    rho, u, v, ww, p = oracle.prim_from_Q(Qd.cpu().numpy())
    vmax = max(np.abs(v).max(), np.abs(ww).max())
    say(f"[config2] 100 steps to t={t:.4f} in {time.time() - t0:.1f}s: max |v|,|w| {vmax:.3e}, "
        f"max |rho-1| {np.abs(rho - 1).max():.3e}")
    assert st == gbr.GBR_OK
    assert vmax <= 1e-12


def test_bounded_jet_freestream_full(gbr):
    """The bench's bounded spatial jet (400x180x180 interior cells, 6 ghost
    layers per side, inflow / zero-gradient outflow, sponge layers) at full
    size: a uniform flow, held in the inflow ghosts and used as the sponge
    reference, gives a zero interior RHS (App. C metrics keep the discrete
    metric identities) and stays uniform over three steps."""
    ng = W.NG
    g = W.bounded(W.jet3d((JET[0] + 2 * ng, JET[1] + 2 * ng, JET[2] + 2 * ng)),
                  [("inflow", "outflow"), ("outflow", "outflow"), ("outflow", "outflow")])
    state = (1.0, 0.5, 0.1, -0.1, 1.0 / 1.4)
    Q0 = W.uniform_flow(g, *state)
    sig = W.sponge_sigma(g, width=20, amp=2.0, power=2.0, sides=[(0, 1), (1, 0), (1, 1), (2, 0), (2, 1)])
    h = gbr.Grid(g, **JET_PARAMS)
    h.metrics(torch.from_numpy(g["xyz"]).cuda())
    h.set_sponge(torch.from_numpy(sig).cuda(), state)
    Q = torch.from_numpy(Q0).cuda()
    res = torch.empty_like(Q)
    h.rhs(Q, res)
    torch.cuda.synchronize()
    inner = (slice(None),) + oracle.interior(g)
    scale = 3.0 * float(h.metric(gbr.SLOT_FACE_HAT(0, 0)).abs().max())
    r = float(res.cpu().numpy()[inner].__abs__().max())
    say(f"[bounded jet full] freestream interior |Res| {r:.3e} (scale {scale:.3e})")
    assert r <= 1e-13 * scale
    for _ in range(3):
        h.step(Q, 0.2, gbr.GBR_DT_CFL)
    assert h.check_state() == gbr.GBR_OK
    d = float((Q.cpu() - torch.from_numpy(Q0)).abs().max())
    say(f"[bounded jet full] 3 steps: max |Q - Q0| {d:.3e}")
    h.close()
    assert d <= 1e-12

"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerance: the FP64 path must match the oracle to a max relative error of
1e-12 per evaluation, measured per variable as max|gpu - oracle| / max|oracle|
(metrics: per family of slots, normalised by the family's largest magnitude).
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def gbr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_10785_amd import gbr as G
    G.lib()
    return G


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def say(*a):
    print(*a, flush=True)


def rel(gpu, ref):
    worst = 0.0
    for v in range(ref.shape[0]):
        s = float(np.abs(ref[v]).max())
        d = float(np.abs(gpu[v] - ref[v]).max())
        worst = max(worst, d / s if s > 0 else d)
    return worst


# oracle slot -> GPU slot, grouped in families normalised together
def slot_families(G):
    fam = {}
    fam["cell_hat"] = [(oracle.M_HAT(d, c), G.SLOT_CELL_HAT(d, c)) for d in range(3) for c in range(3)]
    fam["cell_unhat"] = [(oracle.M_UNHAT(d, c), G.SLOT_CELL_UNHAT(d, c)) for d in range(3) for c in range(3)]
    fam["invj"] = [(oracle.M_INVJ, G.SLOT_CELL_INVJ)]
    fam["j"] = [(oracle.M_J, G.SLOT_CELL_J)]
    fam["cell_t"] = [(oracle.M_HATT(d), G.SLOT_CELL_HATT(d)) for d in range(3)]
    fam["cell_unhat_t"] = [(oracle.M_UNHATT(d), G.SLOT_CELL_UNHATT(d)) for d in range(3)]
    fam["invjt"] = [(oracle.M_INVJT, G.SLOT_CELL_INVJT)]
    for f in range(3):
        fam[f"face{f}_hat"] = [(oracle.M_FHAT(f, c), G.SLOT_FACE_HAT(f, c)) for c in range(3)]
        fam[f"face{f}_t"] = [(oracle.M_FHATT(f), G.SLOT_FACE_HATT(f))]
        fam[f"face{f}_unhat"] = [(oracle.M_FUNHAT(f, e, c), G.SLOT_FACE_UNHAT(f, e, c))
                                 for e in range(3) for c in range(3)]
    return fam


def metric_errors(G, grid_h, m_ref, ndim):
    out = {}
    for name, pairs in slot_families(G).items():
        if ndim == 2 and name.startswith("face2"):
            continue
        ref = np.stack([m_ref[o] for o, _ in pairs])
        gpu = np.stack([grid_h.metric(s).cpu().numpy() for _, s in pairs])
        scale = np.abs(ref).max()
        d = np.abs(gpu - ref).max()
        out[name] = d / scale if scale > 1e-300 else d
    return out


GRIDS = {
    "wavy2d_64": lambda: W.wavy2d((64, 64), L=10.0, amp=0.1),
    "wavy2d_37x23_rand": lambda: W.wavy2d((37, 23), L=4.0, amp=0.08, rand=0.2, seed=3),
    "random3d_21x13x9": lambda: W.random3d((21, 13, 9), amp=0.2, seed=5),
    "deforming3d_16": lambda: W.Deforming3D((16, 16, 16), A=0.75, nmode=2, rand=0.2, seed=7).at(0.13),
    "jet3d_48x20x18": lambda: W.jet3d((48, 20, 18)),
    "tiny3d_4x3x2": lambda: W.random3d((4, 3, 2), amp=0.1, seed=8),
    "thin3d_7x1x5": lambda: W.random3d((7, 1, 5), amp=0.1, seed=9),
}


@pytest.mark.parametrize("name", list(GRIDS))
def test_metrics_parity(gbr, name):
    g = GRIDS[name]()
    say(f"[metrics] {name} n={g['n']} moving={g['xyz_t'] is not None}")
    h = gbr.Grid(g)
    h.metrics(dev(g["xyz"]), dev(g["xyz_t"]) if g["xyz_t"] is not None else None)
    torch.cuda.synchronize()
    errs = metric_errors(gbr, h, oracle.metrics(g), g["ndim"])
    h.close()
    bad = {k: v for k, v in errs.items() if not v <= TOL}
    assert not bad, bad


CASES = [
    # name, grid, state, params
    ("c1_vortex_euler_mp", "wavy2d_64", lambda g: W.shu_vortex(g, eps=5.0, xc=5.0, yc=5.0),
     dict(limiter="mp")),
    ("2d_rough_ns_ducros", "wavy2d_37x23_rand", lambda g: W.random_rough_state(g, seed=1),
     dict(viscous=True, limiter="ducros", theta_c=0.3, Re=200.0)),
    ("2d_rough_euler_none", "wavy2d_37x23_rand", lambda g: W.random_rough_state(g, seed=2),
     dict(limiter="none")),
    ("3d_rough_ns_mp", "random3d_21x13x9", lambda g: W.random_rough_state(g, seed=3),
     dict(viscous=True, limiter="mp", Re=100.0, Mref=0.5)),
    ("3d_rough_euler_ducros", "random3d_21x13x9", lambda g: W.random_rough_state(g, seed=4),
     dict(limiter="ducros", theta_c=0.4)),
    ("3d_smooth_euler_none", "random3d_21x13x9", lambda g: W.random_smooth_state(g, seed=5),
     dict(limiter="none")),
    ("3d_moving_ns_mp", "deforming3d_16", lambda g: W.random_smooth_state(g, seed=6),
     dict(viscous=True, limiter="mp", Re=1e4, Mref=0.5)),
    ("jet_ns_ducros", "jet3d_48x20x18", lambda g: W.jet_ic(g),
     dict(viscous=True, limiter="ducros", Re=1.144e6)),
    ("tiny_ns_mp", "tiny3d_4x3x2", lambda g: W.random_rough_state(g, seed=7),
     dict(viscous=True, limiter="mp", Re=50.0)),
    ("thin_ns_ducros", "thin3d_7x1x5", lambda g: W.random_rough_state(g, seed=8),
     dict(viscous=True, limiter="ducros", theta_c=0.2, Re=50.0)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_rhs_parity(gbr, case):
    name, gname, state, params = case
    g = GRIDS[gname]()
    Q = state(g)
    say(f"[rhs] {name} grid={gname} n={g['n']} params={params}")
    h = gbr.Grid(g, **params)
    h.metrics(dev(g["xyz"]), dev(g["xyz_t"]) if g["xyz_t"] is not None else None)
    Qd = dev(Q)
    res = torch.empty_like(Qd)
    h.rhs(Qd, res)
    torch.cuda.synchronize()
    assert h.check_state() == gbr.GBR_OK
    m = oracle.metrics(g, **params)
    ref = oracle.rhs(g, m, Q, **params)
    got = res.cpu().numpy()
    h.close()
    e = rel(got, ref)
    say(f"[rhs] {name} max rel err {e:.3e}")
    assert e <= TOL


def test_rhs_is_deterministic(gbr):
    g = GRIDS["jet3d_48x20x18"]()
    Q = W.jet_ic(g)
    h = gbr.Grid(g, viscous=True, limiter="ducros", Re=1.144e6)
    h.metrics(dev(g["xyz"]))
    Qd = dev(Q)
    r1, r2 = torch.empty_like(Qd), torch.empty_like(Qd)
    h.rhs(Qd, r1)
    h.rhs(Qd, r2)
    torch.cuda.synchronize()
    h.close()
    assert torch.equal(r1, r2)


@pytest.mark.parametrize("precision,scheme", [("fp64", "meg6"), ("fp32_bulk", "meg6"), ("fp64", "mig4")])
def test_steps_are_deterministic(gbr, precision, scheme):
    """Two grid handles stepped alike give bitwise-equal states and time
    steps: every reduction (the time-step minimum, the sensor gather) is
    order-independent. Multi-tile lines along xi (130 cells: one 127-cell
    tile and a tail tile) and the Ducros-gated limiter."""
    g = W.jet3d((130, 40, 36))
    Q = W.jet_ic(g)
    params = dict(viscous=True, limiter="ducros", Re=1.144e6, precision=precision, scheme=scheme)
    say(f"[determinism] jet 130x40x36 {precision} {scheme}, 5 steps")
    out = []
    for _ in range(2):
        h = gbr.Grid(g, **params)
        h.metrics(dev(g["xyz"]))
        Qd = dev(Q)
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        dts = []
        for _ in range(5):
            h.step(Qd, 0.2, gbr.GBR_DT_CFL, dt_out=dt)
            dts.append(dt.clone())
        torch.cuda.synchronize()
        assert h.check_state() == gbr.GBR_OK
        h.close()
        out.append((Qd, torch.cat(dts)))
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])


def test_step_parity_config1_vortex(gbr):
    """2-D Euler isentropic vortex (strength 5) on the periodic 64x64 wavy
    grid, gradient-based reconstruction + MP + HLLC, SSP-RK3 at CFL 0.4,
    10 steps: state and time step after every step match the oracle."""
    g = GRIDS["wavy2d_64"]()
    Q = W.shu_vortex(g, eps=5.0, xc=5.0, yc=5.0)
    params = dict(limiter="mp")
    say("[step] config1 vortex 64x64, 10 steps CFL 0.4")
    h = gbr.Grid(g, **params)
    h.metrics(dev(g["xyz"]))
    m = oracle.metrics(g, **params)
    Qd = dev(Q)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    for s in range(10):
        h.step(Qd, 0.4, gbr.GBR_DT_CFL, dt_out=dt)
        Q, dt_ref = oracle.step(g, m, Q, 0.4, **params)
        torch.cuda.synchronize()
        e = rel(Qd.cpu().numpy(), Q)
        assert e <= TOL, (s, e)
        assert abs(dt.item() - dt_ref) <= TOL * dt_ref
    assert h.check_state() == gbr.GBR_OK
    h.close()


def test_step_parity_moving_grid(gbr):
    """3-D NS on a deforming randomized grid: metrics recomputed every step
    inside gbr_step from the caller's coordinates at t^n."""
    mv = W.Deforming3D((20, 18, 16), A=0.75, nmode=2, rand=0.2, seed=11)
    params = dict(viscous=True, limiter="mp", Re=1e4, Mref=0.5)
    g0 = mv.at(0.0)
    Q = W.random_smooth_state(g0, seed=9, amp=0.05)
    say("[step] moving 20x18x16 NS, 3 steps")
    h = gbr.Grid(g0, **params)
    m = oracle.metrics(g0, **params)
    Qd = dev(Q)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = 0.0
    for s in range(3):
        gt = mv.at(t)
        h.step(Qd, 0.2, gbr.GBR_DT_CFL, xyz=dev(gt["xyz"]), xyz_t=dev(gt["xyz_t"]), dt_out=dt)
        Q, dt_ref = oracle.step(gt, m, Q, 0.2, **params)
        torch.cuda.synchronize()
        e = rel(Qd.cpu().numpy(), Q)
        assert e <= TOL, (s, e)
        assert abs(dt.item() - dt_ref) <= TOL * dt_ref
        t += dt_ref
    h.close()


def test_rk_stage_and_cfl_entry_points(gbr):
    """gbr_cfl and gbr_rk_stage called directly match the oracle's stages."""
    g = GRIDS["random3d_21x13x9"]()
    Q0 = W.random_smooth_state(g, seed=12)
    params = dict(viscous=True, limiter="ducros", theta_c=0.1, Re=300.0)
    h = gbr.Grid(g, **params)
    h.metrics(dev(g["xyz"]))
    m = oracle.metrics(g, **params)
    Qn, Q = dev(Q0), dev(Q0)
    res = torch.empty_like(Q)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    h.cfl(Qn, 0.25, dt)
    torch.cuda.synchronize()
    dt_ref = 0.25 * oracle.cfl_min(g, m, Q0, **params)
    assert abs(dt.item() - dt_ref) <= TOL * dt_ref
    Qr = Q0.copy()
    for s in range(3):
        h.rhs(Q, res)
        h.rk_stage(s, dt, Qn, Q, res)
        r = oracle.rhs(g, m, Qr, **params)
        Qr = oracle.rk_stage(g, m, s, dt_ref, Q0, Qr, r, **params)
        torch.cuda.synchronize()
        assert rel(Q.cpu().numpy(), Qr) <= TOL
    h.close()


def test_step_advances_time_per_grid(gbr):
    """gbr_step adds each step's dt to the caller's per-grid device time
    (App. B: t^{n+1} = t^n + dt), in CFL and fixed-dt modes, for several
    grids in one call; the time and dt outputs may not alias."""
    gs = [GRIDS["random3d_21x13x9"](), GRIDS["wavy2d_37x23_rand"]()]
    hs, Qs, ts, dts = [], [], [], []
    for q, g in enumerate(gs):
        h = gbr.Grid(g, limiter="mp")
        h.metrics(dev(g["xyz"]))
        hs.append(h)
        Qs.append(dev(W.random_smooth_state(g, seed=40 + q)))
        ts.append(torch.full((1,), 0.25 * (q + 1), dtype=torch.float64, device="cuda"))
        dts.append(torch.zeros(1, dtype=torch.float64, device="cuda"))
    expect = [0.25, 0.5]
    for s in range(4):
        mode, val = (gbr.GBR_DT_CFL, 0.3) if s % 2 == 0 else (gbr.GBR_DT_FIXED, 1e-3)
        gbr.gbr_step([h.h for h in hs], Qs, val, mode, dt_out=dts, t=ts)
        torch.cuda.synchronize()
        for q in range(2):
            expect[q] += dts[q].item()
            assert ts[q].item() == expect[q], (s, q, ts[q].item(), expect[q])
    with pytest.raises(gbr.GbrError) as ei:
        hs[0].step(Qs[0], 0.3, gbr.GBR_DT_CFL, dt_out=ts[0], t=ts[0])
    assert ei.value.status == gbr.GBR_E_ARG
    for h in hs:
        h.close()


def test_nonphysical_state_is_reported(gbr):
    g = GRIDS["random3d_21x13x9"]()
    Q = W.random_smooth_state(g, seed=13)
    Q[0, 3, 4, 5] = -0.5  # negative density set on the host
    h = gbr.Grid(g, limiter="mp")
    h.metrics(dev(g["xyz"]))
    Qd = dev(Q)
    res = torch.empty_like(Qd)
    h.rhs(Qd, res)
    assert h.check_state() == gbr.GBR_E_STATE
    assert "non-physical" in gbr.gbr_last_error(h.h)
    # flags are cleared by the check
    h.rhs(dev(W.random_smooth_state(g, seed=13)), res)
    assert h.check_state() == gbr.GBR_OK
    h.close()


def test_folded_grid_reports_jacobian(gbr):
    g = W.uniform3d((8, 8, 8))
    xyz = g["xyz"].copy()
    xyz[0, :, :, 3], xyz[0, :, :, 4] = g["xyz"][0, :, :, 5], g["xyz"][0, :, :, 2]
    h = gbr.Grid(g)
    with pytest.raises(gbr.GbrError) as ei:
        h.metrics(dev(xyz))
    assert ei.value.status == gbr.GBR_E_JACOBIAN
    h.close()


def test_argument_errors(gbr):
    g = W.uniform3d((6, 6, 6))
    h = gbr.Grid(g)
    Qd = dev(W.uniform_flow(g))
    with pytest.raises(gbr.GbrError) as ei:
        h.rhs(Qd, Qd)  # aliasing
    assert ei.value.status == gbr.GBR_E_ARG
    with pytest.raises(gbr.GbrError):
        h.rk_stage(3, Qd, Qd, Qd, Qd)
    mv = gbr.Grid(dict(g, xyz_t=np.zeros_like(g["xyz"])))
    with pytest.raises(gbr.GbrError) as ei:
        mv.metrics(dev(g["xyz"]))  # moving grid without velocities
    assert ei.value.status == gbr.GBR_E_ARG
    h.close()
    mv.close()


# ---------------------------------------------------------------------------
# FP32-bulk: reconstruction, limiter, HLLC and viscous flux in float; Q,
# metrics, J, (1/J)_t and the RK accumulation in double. Compared with the
# FP64 oracle under the stated bounds.
# ---------------------------------------------------------------------------
FP32_RHS_TOL = 2e-4     # per-variable max relative error of one RHS
FP32_STEP_TOL = 1e-5    # per-variable max relative error of Q after 10 steps

FP32_CASES = [
    ("c1_vortex_euler_mp", "wavy2d_64", lambda g: W.shu_vortex(g, eps=5.0, xc=5.0, yc=5.0),
     dict(limiter="mp")),
    ("3d_smooth_ns_mp", "random3d_21x13x9", lambda g: W.random_smooth_state(g, seed=5),
     dict(viscous=True, limiter="mp", Re=100.0, Mref=0.5)),
    ("3d_moving_ns_mp", "deforming3d_16", lambda g: W.random_smooth_state(g, seed=6),
     dict(viscous=True, limiter="mp", Re=1e4, Mref=0.5)),
    ("jet_ns_ducros", "jet3d_48x20x18", lambda g: W.jet_ic(g),
     dict(viscous=True, limiter="ducros", Re=1.144e6)),
]


@pytest.mark.parametrize("case", FP32_CASES, ids=[c[0] for c in FP32_CASES])
def test_fp32_bulk_rhs_within_bound(gbr, case):
    name, gname, state, params = case
    g = GRIDS[gname]()
    Q = state(g)
    say(f"[fp32 rhs] {name} n={g['n']}")
    h = gbr.Grid(g, precision="fp32_bulk", **params)
    h.metrics(dev(g["xyz"]), dev(g["xyz_t"]) if g["xyz_t"] is not None else None)
    Qd = dev(Q)
    res = torch.empty(Qd.shape, dtype=torch.float32, device="cuda")
    h.rhs(Qd, res)
    torch.cuda.synchronize()
    assert h.check_state() == gbr.GBR_OK
    h.close()
    ref = oracle.rhs(g, oracle.metrics(g, **params), Q, **params)
    e = rel(res.double().cpu().numpy(), ref)
    say(f"[fp32 rhs] {name} max rel err vs FP64 oracle {e:.3e}")
    assert e <= FP32_RHS_TOL


def test_fp32_bulk_rhs_after_metric_update(gbr):
    """FP32-bulk flux kernels read a float copy of the metrics: after a second
    metric evaluation (a deforming grid at a later time) the RHS must use the
    new metrics. Compared with the FP64 oracle at the second time."""
    mv = W.Deforming3D((16, 14, 12), A=0.75, nmode=2, rand=0.2, seed=8)
    params = dict(viscous=True, limiter="mp", Re=1e4, Mref=0.5)
    g0, g1 = mv.at(0.0), mv.at(0.23)
    Q = W.random_smooth_state(g1, seed=9)
    h = gbr.Grid(g0, precision="fp32_bulk", **params)
    h.metrics(dev(g0["xyz"]), dev(g0["xyz_t"]))
    h.metrics(dev(g1["xyz"]), dev(g1["xyz_t"]))
    Qd = dev(Q)
    res = torch.empty(Qd.shape, dtype=torch.float32, device="cuda")
    h.rhs(Qd, res)
    torch.cuda.synchronize()
    h.close()
    ref = oracle.rhs(g1, oracle.metrics(g1, **params), Q, **params)
    e = rel(res.double().cpu().numpy(), ref)
    say(f"[fp32 rhs] after a metric update, max rel err vs FP64 oracle {e:.3e}")
    assert e <= FP32_RHS_TOL


def test_fp32_bulk_steps_config1(gbr):
    g = GRIDS["wavy2d_64"]()
    Q = W.shu_vortex(g, eps=5.0, xc=5.0, yc=5.0)
    h = gbr.Grid(g, precision="fp32_bulk", limiter="mp")
    h.metrics(dev(g["xyz"]))
    m = oracle.metrics(g, limiter="mp")
    Qd = dev(Q)
    for _ in range(10):
        h.step(Qd, 0.4, gbr.GBR_DT_CFL)
        Q, _ = oracle.step(g, m, Q, 0.4, limiter="mp")
    torch.cuda.synchronize()
    e = rel(Qd.cpu().numpy(), Q)
    say(f"[fp32 step] config1 10 steps max rel err {e:.3e}")
    h.close()
    assert e <= FP32_STEP_TOL


def test_fp32_bulk_freestream_moving(gbr):
    """FP32-bulk keeps freestream to single-precision round-off on a deforming
    randomized grid (the metrics and GCL terms stay in double)."""
    mv = W.Deforming3D((16, 16, 16), A=0.75, nmode=2, rand=0.2, seed=6)
    g = mv.at(0.0)
    pinf = 1.0 / (1.4 * 0.25)
    Q = W.uniform_flow(g, 1.0, 1.0, 0.0, 0.0, pinf)
    h = gbr.Grid(g, precision="fp32_bulk", viscous=True, limiter="mp", Mref=0.5, Re=1e4)
    Qd = dev(Q)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = 0.0
    for _ in range(10):
        gt = mv.at(t)
        h.step(Qd, 0.2, gbr.GBR_DT_CFL, xyz=dev(gt["xyz"]), xyz_t=dev(gt["xyz_t"]), dt_out=dt)
        torch.cuda.synchronize()
        t += dt.item()
    rho, u, v, w, p = oracle.prim_from_Q(Qd.cpu().numpy())
    vmax = max(np.abs(v).max(), np.abs(w).max())
    say(f"[fp32 freestream] max |v|,|w| after 10 moving steps {vmax:.3e}")
    h.close()
    assert vmax < 1e-5


# xi line lengths around the sweep's tiling: lines are cut into 127-cell
# tiles and a remainder below 32 cells goes to a 32-face tail tile in the
# same launch. 31: tail only; 32, 64: one partial full tile; 127: one exact
# tile; 128: a tile and a 1-cell tail; 158: a tile and the largest tail (31);
# 159: two tiles, the second partial; 254: two exact tiles.
XI_LENGTHS = [31, 32, 64, 127, 128, 158, 159, 254]


@pytest.mark.parametrize("ni", XI_LENGTHS)
def test_xi_tiling_rhs_and_steps(gbr, ni):
    """One RHS and two SSP-RK3 steps (the last xi sweep of each stage applies
    the stage and forms the next primitives) match the oracle on an
    ni x 5 x 4 randomized grid with a rough state, NS with the Ducros gate."""
    g = W.random3d((ni, 5, 4), amp=0.1, seed=20 + ni)
    Q = W.random_rough_state(g, seed=30 + ni)
    params = dict(viscous=True, limiter="ducros", theta_c=0.2, Re=100.0)
    say(f"[xi tiling] ni={ni} n={g['n']}")
    h = gbr.Grid(g, **params)
    h.metrics(dev(g["xyz"]))
    m = oracle.metrics(g, **params)
    Qd = dev(Q)
    res = torch.empty_like(Qd)
    h.rhs(Qd, res)
    torch.cuda.synchronize()
    e_rhs = rel(res.cpu().numpy(), oracle.rhs(g, m, Q, **params))
    dt = 2e-4
    for s in range(2):
        h.step(Qd, dt, gbr.GBR_DT_FIXED)
        Q, _ = oracle.step(g, m, Q, dt, dt_mode=oracle.DT_FIXED, **params)
    torch.cuda.synchronize()
    e_step = rel(Qd.cpu().numpy(), Q)
    say(f"[xi tiling] ni={ni}: rhs max rel err {e_rhs:.3e}, state after 2 steps {e_step:.3e}")
    assert h.check_state() == gbr.GBR_OK
    h.close()
    assert e_rhs <= TOL and e_step <= TOL


def test_grouped_tile_order_parity(gbr):
    """The tiled kernels take their tile from a block index permuted in runs
    of 256 blocks (neighbouring tiles grouped on one XCD); blocks past the
    last full run keep their order. On a 270 x 64 x 64 grid every tiled
    kernel has full runs and a partial one (cell gradients 272 blocks, xi
    sweep 4608 with two 127-cell tiles and a 16-cell tail per line, eta and
    zeta sweeps 5440 each): one RHS and one SSP-RK3 step match the oracle
    element by element, NS with the Ducros-gated limiter."""
    g = W.random3d((270, 64, 64), amp=0.1, seed=41)
    Q = W.random_rough_state(g, seed=42)
    params = dict(viscous=True, limiter="ducros", theta_c=0.3, Re=500.0)
    say(f"[grouped tiles] n={g['n']}")
    h = gbr.Grid(g, **params)
    h.metrics(dev(g["xyz"]))
    m = oracle.metrics(g, **params)
    Qd = dev(Q)
    res = torch.empty_like(Qd)
    h.rhs(Qd, res)
    torch.cuda.synchronize()
    e_rhs = rel(res.cpu().numpy(), oracle.rhs(g, m, Q, **params))
    dt = 1e-4
    h.step(Qd, dt, gbr.GBR_DT_FIXED)
    Q1, _ = oracle.step(g, m, Q, dt, dt_mode=oracle.DT_FIXED, **params)
    torch.cuda.synchronize()
    e_step = rel(Qd.cpu().numpy(), Q1)
    say(f"[grouped tiles] rhs max rel err {e_rhs:.3e}, state after 1 step {e_step:.3e}")
    assert h.check_state() == gbr.GBR_OK
    h.close()
    assert e_rhs <= TOL and e_step <= TOL

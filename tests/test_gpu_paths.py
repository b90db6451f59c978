"""Parity cases for kernel paths that the small grids of the other parity
files do not reach, against the FP64 oracle through the C ABI (FP64 within a
max relative error of 1e-12 per evaluation, FP32-bulk within its stated
bounds):

- MIG4 on lines that span several IG4 line tiles (Eq. IG4_grads, Sec. 7): the
  IG4 gradient kernel cuts xi lines into 256-cell tiles and eta/zeta lines
  into 64-cell tiles, each with a 48-cell halo read from the neighbouring
  tiles; lines of 300 and 140 cells take two full tiles and a remainder;
- supersonic faces, where the curvilinear HLLC flux (Sec. 5.1.1) takes its
  one-sided branches (all waves to the right: the left flux; all waves to the
  left: the right flux), along every direction and in both signs.
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
FP32_RHS_TOL = 2e-4
FP32_STEP_TOL = 1e-5


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


# ---------------------------------------------------------------------------
# MIG4 across IG4 line tiles
# ---------------------------------------------------------------------------
MIG4_GRIDS = {
    # 300 = 256 + 44 along xi; 140 = 2 x 64 + 12 along eta and zeta
    "xi300_5x4": lambda: W.random3d((300, 5, 4), amp=0.2, seed=41),
    "eta140_5x4": lambda: W.random3d((5, 140, 4), amp=0.2, seed=42),
    "zeta140_5x4": lambda: W.random3d((5, 4, 140), amp=0.2, seed=43),
    "wavy2d_300x80": lambda: W.wavy2d((300, 80), L=10.0, amp=0.08, rand=0.2, seed=44),
    "jet_300x70x6": lambda: W.jet3d((300, 70, 6)),
}

MIG4_CASES = [
    ("xi300_ns_ducros_rough", "xi300_5x4",
     dict(viscous=True, limiter="ducros", theta_c=0.3, Re=300.0),
     lambda g: W.random_rough_state(g, seed=51, amp=0.2)),
    ("eta140_ns_mp_smooth", "eta140_5x4", dict(viscous=True, limiter="mp", Re=500.0),
     lambda g: W.random_smooth_state(g, seed=52)),
    ("zeta140_euler_ducros_rough", "zeta140_5x4", dict(viscous=False, limiter="ducros", theta_c=0.3),
     lambda g: W.random_rough_state(g, seed=53, amp=0.2)),
    ("wavy2d_300x80_euler_mp_vortex", "wavy2d_300x80", dict(viscous=False, limiter="mp"),
     lambda g: W.shu_vortex(g, xc=5.0, yc=5.0)),
    ("jet_300x70x6_ns_ducros", "jet_300x70x6", dict(viscous=True, limiter="ducros", Re=1.144e6),
     lambda g: W.jet_ic(g)),
]


@pytest.mark.parametrize("name", sorted(MIG4_GRIDS))
def test_mig4_multitile_metrics(gbr, name):
    g = MIG4_GRIDS[name]()
    say(f"[mig4 multitile metrics] {name} n={g['n']}")
    h = gbr.Grid(g, scheme="mig4")
    h.metrics(dev(g["xyz"]))
    torch.cuda.synchronize()
    m = oracle.metrics(g, scheme="mig4")
    worst = 0.0
    for d in range(3):
        for c in range(3):
            pairs = [(oracle.M_HAT(d, c), gbr.SLOT_CELL_HAT(d, c)),
                     (oracle.M_UNHAT(d, c), gbr.SLOT_CELL_UNHAT(d, c))]
            for o, s in pairs:
                ref = m[o]
                got = h.metric(s).cpu().numpy()
                scale = float(np.abs(ref).max())
                if scale > 1e-300:
                    worst = max(worst, float(np.abs(got - ref).max()) / scale)
    for f in range(g["ndim"]):
        ref = np.stack([m[oracle.M_FHAT(f, c)] for c in range(3)])
        got = np.stack([h.metric(gbr.SLOT_FACE_HAT(f, c)).cpu().numpy() for c in range(3)])
        worst = max(worst, float(np.abs(got - ref).max()) / float(np.abs(ref).max()))
        ref = np.stack([m[oracle.M_FUNHAT(f, e, c)] for e in range(3) for c in range(3)])
        got = np.stack([h.metric(gbr.SLOT_FACE_UNHAT(f, e, c)).cpu().numpy()
                        for e in range(3) for c in range(3)])
        worst = max(worst, float(np.abs(got - ref).max()) / float(np.abs(ref).max()))
    ref, got = m[oracle.M_J], h.metric(gbr.SLOT_CELL_J).cpu().numpy()
    worst = max(worst, float(np.abs(got - ref).max()) / float(np.abs(ref).max()))
    say(f"[mig4 multitile metrics] {name}: worst {worst:.3e}")
    h.close()
    assert worst <= TOL


@pytest.mark.parametrize("case", MIG4_CASES, ids=[c[0] for c in MIG4_CASES])
def test_mig4_multitile_rhs_and_steps(gbr, case):
    """One RHS, then two SSP-RK3 steps at a fixed dt (the last sweep of each
    stage applies the stage), on lines spanning several IG4 tiles."""
    name, gname, params, state = case
    g = MIG4_GRIDS[gname]()
    Q = state(g)
    params = dict(params, scheme="mig4")
    say(f"[mig4 multitile] {name} n={g['n']}")
    h = gbr.Grid(g, **params)
    h.metrics(dev(g["xyz"]))
    m = oracle.metrics(g, **params)
    Qd = dev(Q)
    res = torch.empty_like(Qd)
    h.rhs(Qd, res)
    torch.cuda.synchronize()
    assert h.check_state() == gbr.GBR_OK
    e_rhs = rel(res.cpu().numpy(), oracle.rhs(g, m, Q, **params))
    dt = 0.25 * oracle.cfl_min(g, m, Q, **params)
    for _ in range(2):
        h.step(Qd, dt, gbr.GBR_DT_FIXED)
        Q, _ = oracle.step(g, m, Q, dt, dt_mode=oracle.DT_FIXED, **params)
    torch.cuda.synchronize()
    e_step = rel(Qd.cpu().numpy(), Q)
    say(f"[mig4 multitile] {name}: rhs {e_rhs:.3e}, 2 steps {e_step:.3e}")
    assert h.check_state() == gbr.GBR_OK
    h.close()
    assert e_rhs <= TOL and e_step <= TOL


def test_mig4_multitile_fp32_bulk(gbr):
    g = MIG4_GRIDS["xi300_5x4"]()
    params = dict(viscous=True, limiter="ducros", theta_c=0.3, Re=300.0, scheme="mig4")
    Q = W.random_smooth_state(g, seed=54)
    h = gbr.Grid(g, precision="fp32_bulk", **params)
    h.metrics(dev(g["xyz"]))
    m = oracle.metrics(g, **params)
    res = torch.empty(Q.shape, dtype=torch.float32, device="cuda")
    Qd = dev(Q)
    h.rhs(Qd, res)
    torch.cuda.synchronize()
    e_rhs = rel(res.double().cpu().numpy(), oracle.rhs(g, m, Q, **params))
    dt = 0.25 * oracle.cfl_min(g, m, Q, **params)
    for _ in range(2):
        h.step(Qd, dt, gbr.GBR_DT_FIXED)
        Q, _ = oracle.step(g, m, Q, dt, dt_mode=oracle.DT_FIXED, **params)
    torch.cuda.synchronize()
    e_step = rel(Qd.cpu().numpy(), Q)
    say(f"[mig4 multitile fp32] rhs {e_rhs:.3e}, 2 steps {e_step:.3e}")
    h.close()
    assert e_rhs <= FP32_RHS_TOL and e_step <= FP32_STEP_TOL


# ---------------------------------------------------------------------------
# Supersonic faces: HLLC's one-sided branches
# ---------------------------------------------------------------------------
SUP_GRIDS = {
    "random3d_21x13x9": lambda: W.random3d((21, 13, 9), amp=0.2, seed=61),
    "wavy2d_37x23": lambda: W.wavy2d((37, 23), L=4.0, amp=0.08, rand=0.2, seed=62),
    "jet3d_40x18x18": lambda: W.jet3d((40, 18, 18)),
}

SUP_CASES = [
    ("3d_euler_none", "random3d_21x13x9", dict(limiter="none")),
    ("3d_euler_mp", "random3d_21x13x9", dict(limiter="mp")),
    ("3d_ns_ducros", "random3d_21x13x9", dict(viscous=True, limiter="ducros", theta_c=0.3, Re=300.0)),
    ("2d_euler_mp", "wavy2d_37x23", dict(limiter="mp")),
    ("2d_ns_none", "wavy2d_37x23", dict(viscous=True, limiter="none", Re=200.0)),
    ("jet_ns_ducros", "jet3d_40x18x18", dict(viscous=True, limiter="ducros", Re=1.144e6)),
    ("3d_ns_mp_mig4", "random3d_21x13x9", dict(viscous=True, limiter="mp", Re=300.0, scheme="mig4")),
]


@pytest.mark.parametrize("case", SUP_CASES, ids=[c[0] for c in SUP_CASES])
def test_supersonic_rhs_and_steps(gbr, case):
    """Mach-3 streams in both directions along every family of faces."""
    name, gname, params = case
    g = SUP_GRIDS[gname]()
    Q = W.supersonic_rough_state(g, seed=sum(map(ord, name)) % 97)
    say(f"[supersonic] {name} n={g['n']}")
    h = gbr.Grid(g, **params)
    h.metrics(dev(g["xyz"]))
    m = oracle.metrics(g, **params)
    Qd = dev(Q)
    res = torch.empty_like(Qd)
    h.rhs(Qd, res)
    torch.cuda.synchronize()
    assert h.check_state() == gbr.GBR_OK
    e_rhs = rel(res.cpu().numpy(), oracle.rhs(g, m, Q, **params))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    e_step = 0.0
    for s in range(2):
        h.step(Qd, 0.2, gbr.GBR_DT_CFL, dt_out=dt)
        Q, dt_ref = oracle.step(g, m, Q, 0.2, **params)
        torch.cuda.synchronize()
        e_step = max(e_step, rel(Qd.cpu().numpy(), Q))
        assert abs(dt.item() - dt_ref) <= TOL * dt_ref
    say(f"[supersonic] {name}: rhs {e_rhs:.3e}, 2 steps {e_step:.3e}")
    assert h.check_state() == gbr.GBR_OK
    h.close()
    assert e_rhs <= TOL and e_step <= TOL


@pytest.mark.parametrize("gname", ["random3d_21x13x9", "wavy2d_37x23"])
def test_supersonic_fp32_bulk(gbr, gname):
    g = SUP_GRIDS[gname]()
    params = dict(viscous=True, limiter="ducros", theta_c=0.3, Re=300.0)
    Q = W.supersonic_rough_state(g, seed=5)
    h = gbr.Grid(g, precision="fp32_bulk", **params)
    h.metrics(dev(g["xyz"]))
    m = oracle.metrics(g, **params)
    Qd = dev(Q)
    res = torch.empty(Q.shape, dtype=torch.float32, device="cuda")
    h.rhs(Qd, res)
    torch.cuda.synchronize()
    e_rhs = rel(res.double().cpu().numpy(), oracle.rhs(g, m, Q, **params))
    dt = 0.2 * oracle.cfl_min(g, m, Q, **params)
    for _ in range(2):
        h.step(Qd, dt, gbr.GBR_DT_FIXED)
        Q, _ = oracle.step(g, m, Q, dt, dt_mode=oracle.DT_FIXED, **params)
    torch.cuda.synchronize()
    e_step = rel(Qd.cpu().numpy(), Q)
    say(f"[supersonic fp32] {gname}: rhs {e_rhs:.3e}, 2 steps {e_step:.3e}")
    h.close()
    assert e_rhs <= FP32_RHS_TOL and e_step <= FP32_STEP_TOL


@pytest.mark.parametrize("tile", [0, 1, 2])
def test_supersonic_batch(gbr, tile):
    """The batched tile kernel has its own HLLC: Mach-3 streams through its
    xi and eta interfaces, two steps per tile shape against the oracle."""
    params = dict(viscous=False, limiter="mp")
    cs = []
    for n, seed in [((40, 24), 71), ((19, 33), 72)]:
        g = W.wavy2d(n, L=4.0, amp=0.05, rand=0.1, seed=seed)
        cs.append((g, W.supersonic_rough_state(g, seed=seed)))
    grids, Qs = [], []
    for g, Q in cs:
        h = gbr.Grid(g, **params)
        h.metrics(dev(g["xyz"]))
        grids.append(h)
        Qs.append(dev(Q))
    b = gbr.Batch(grids, Qs, tile=tile)
    refs = [(oracle.metrics(g, **params), Q) for g, Q in cs]
    for step in range(2):
        b.run(1, 0.4, gbr.GBR_DT_CFL, graph=False)
        _, dts, _ = b.query()
        for q, (g, _) in enumerate(cs):
            m, Qr = refs[q]
            Qr, dt_ref = oracle.step(g, m, Qr, 0.4, **params)
            refs[q] = (m, Qr)
            e = rel(Qs[q].cpu().numpy(), Qr)
            say(f"[supersonic batch tile {tile}] grid {q} step {step}: {e:.3e}")
            assert e <= TOL and abs(dts[q] - dt_ref) <= TOL * dt_ref
    for h in grids:
        assert h.check_state() == gbr.GBR_OK
    b.close()
    for h in grids:
        h.close()

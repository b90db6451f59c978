"""MIG4 scheme (IG4 gradients, IG4-based metrics) on the GPU against the
FP64 oracle, through the C ABI. Same bar as MEG6: max relative error 1e-12
per evaluation (metrics per slot family); FP32-bulk within 2e-4 per RHS."""
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


def families(G):
    fam = {
        "cell_hat": [(oracle.M_HAT(d, c), G.SLOT_CELL_HAT(d, c)) for d in range(3) for c in range(3)],
        "cell_unhat": [(oracle.M_UNHAT(d, c), G.SLOT_CELL_UNHAT(d, c)) for d in range(3) for c in range(3)],
        "j": [(oracle.M_J, G.SLOT_CELL_J)],
        "invjt": [(oracle.M_INVJT, G.SLOT_CELL_INVJT)],
    }
    for f in range(3):
        fam[f"face{f}_hat"] = [(oracle.M_FHAT(f, c), G.SLOT_FACE_HAT(f, c)) for c in range(3)]
        fam[f"face{f}_t"] = [(oracle.M_FHATT(f), G.SLOT_FACE_HATT(f))]
        fam[f"face{f}_unhat"] = [(oracle.M_FUNHAT(f, e, c), G.SLOT_FACE_UNHAT(f, e, c))
                                 for e in range(3) for c in range(3)]
    return fam


GRIDS = {
    "random3d_9x8x7": lambda: W.random3d((9, 8, 7), seed=3),
    "sinusoidal3d_10x9x8": lambda: W.sinusoidal3d((10, 9, 8)),
    "wavy2d_random_24x20": lambda: W.wavy2d((24, 20), rand=0.2, seed=2),
    "tiny_4x3x2": lambda: W.random3d((4, 3, 2), seed=1),
    "deforming_12x10x9": lambda: W.Deforming3D((12, 10, 9), A=0.75, nmode=2, rand=0.2, seed=4).at(0.17),
    "jet_40x18x18": lambda: W.jet3d((40, 18, 18)),
}


@pytest.mark.parametrize("name", sorted(GRIDS))
def test_mig4_metrics(gbr, name):
    g = GRIDS[name]()
    h = gbr.Grid(g, scheme="mig4")
    xt = g.get("xyz_t")
    h.metrics(dev(g["xyz"]), dev(xt) if xt is not None else None)
    torch.cuda.synchronize()
    m = oracle.metrics(g, scheme="mig4")
    worst = {}
    for fam, pairs in families(gbr).items():
        if g["ndim"] == 2 and fam.startswith("face2"):
            continue
        ref = np.stack([m[o] for o, _ in pairs])
        got = np.stack([h.metric(s).cpu().numpy() for _, s in pairs])
        scale = float(np.abs(ref).max())
        worst[fam] = float(np.abs(got - ref).max()) / scale if scale > 1e-300 else float(np.abs(got - ref).max())
    say(f"[mig4 metrics] {name}: worst {max(worst.values()):.3e} ({max(worst, key=worst.get)})")
    h.close()
    assert max(worst.values()) <= TOL, worst


RHS_CASES = [
    ("euler_mp_random", "random3d_9x8x7", dict(viscous=False, limiter="mp"),
     lambda g: W.random_smooth_state(g, seed=4)),
    ("ns_ducros_rough", "random3d_9x8x7", dict(viscous=True, limiter="ducros", theta_c=0.3, Re=300.0),
     lambda g: W.random_rough_state(g, seed=5, amp=0.2)),
    ("ns_mp_sinusoidal", "sinusoidal3d_10x9x8", dict(viscous=True, limiter="mp", Re=500.0),
     lambda g: W.random_smooth_state(g, seed=6)),
    ("euler_none_vortex2d", "wavy2d_random_24x20", dict(viscous=False, limiter="none"),
     lambda g: W.shu_vortex(g, xc=5.0, yc=5.0)),
    ("ns_ducros_2d", "wavy2d_random_24x20", dict(viscous=True, limiter="ducros", theta_c=0.2, Re=200.0),
     lambda g: W.random_rough_state(g, seed=7, amp=0.2)),
    ("ns_mp_tiny", "tiny_4x3x2", dict(viscous=True, limiter="mp", Re=100.0),
     lambda g: W.random_smooth_state(g, seed=8)),
    ("ns_mp_moving", "deforming_12x10x9", dict(viscous=True, limiter="mp", Re=1e3, Mref=0.5),
     lambda g: W.random_smooth_state(g, seed=9)),
    ("ns_ducros_jet", "jet_40x18x18", dict(viscous=True, limiter="ducros", Re=1.144e6),
     lambda g: W.jet_ic(g)),
]


@pytest.mark.parametrize("case", RHS_CASES, ids=[c[0] for c in RHS_CASES])
def test_mig4_rhs(gbr, case):
    name, gname, params, state = case
    g = GRIDS[gname]()
    Q = state(g)
    h = gbr.Grid(g, scheme="mig4", **params)
    xt = g.get("xyz_t")
    h.metrics(dev(g["xyz"]), dev(xt) if xt is not None else None)
    Qd = dev(Q)
    res = torch.empty_like(Qd)
    h.rhs(Qd, res)
    torch.cuda.synchronize()
    assert h.check_state() == gbr.GBR_OK
    m = oracle.metrics(g, scheme="mig4", **params)
    ref = oracle.rhs(g, m, Q, scheme="mig4", **params)
    e = rel(res.cpu().numpy(), ref)
    say(f"[mig4 rhs] {name}: max rel err {e:.3e}")
    h.close()
    assert e <= TOL


def test_mig4_steps_2d_vortex(gbr):
    """Config-1-like 2-D vortex with MIG4: five SSP-RK3 steps at CFL 0.4."""
    g = W.wavy2d((32, 32), L=10.0, amp=0.1)
    params = dict(viscous=False, limiter="mp", scheme="mig4")
    Q = W.shu_vortex(g)
    h = gbr.Grid(g, **params)
    h.metrics(dev(g["xyz"]))
    m = oracle.metrics(g, **params)
    Qd = dev(Q)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    for s in range(5):
        h.step(Qd, 0.4, gbr.GBR_DT_CFL, dt_out=dt)
        Q, dt_ref = oracle.step(g, m, Q, 0.4, **params)
        torch.cuda.synchronize()
        e = rel(Qd.cpu().numpy(), Q)
        say(f"[mig4 step 2d] step {s}: {e:.3e}")
        assert e <= TOL and abs(dt.item() - dt_ref) <= TOL * dt_ref
    h.close()


def test_mig4_step_3d_ns(gbr):
    g = W.random3d((12, 10, 9), seed=11)
    params = dict(viscous=True, limiter="ducros", theta_c=0.3, Re=500.0, scheme="mig4")
    Q = W.random_smooth_state(g, seed=12)
    h = gbr.Grid(g, **params)
    h.metrics(dev(g["xyz"]))
    m = oracle.metrics(g, **params)
    Qd = dev(Q)
    for s in range(2):
        h.step(Qd, 0.2, gbr.GBR_DT_CFL)
        Q, _ = oracle.step(g, m, Q, 0.2, **params)
    torch.cuda.synchronize()
    e = rel(Qd.cpu().numpy(), Q)
    say(f"[mig4 step 3d ns] {e:.3e}")
    h.close()
    assert e <= TOL


def test_mig4_fp32_bulk_rhs(gbr):
    g = GRIDS["random3d_9x8x7"]()
    params = dict(viscous=True, limiter="mp", Re=500.0)
    Q = W.random_smooth_state(g, seed=13)
    h = gbr.Grid(g, scheme="mig4", precision="fp32_bulk", **params)
    h.metrics(dev(g["xyz"]))
    res = torch.empty(Q.shape, dtype=torch.float32, device="cuda")
    h.rhs(dev(Q), res)
    torch.cuda.synchronize()
    m = oracle.metrics(g, scheme="mig4", **params)
    ref = oracle.rhs(g, m, Q, scheme="mig4", **params)
    e = rel(res.double().cpu().numpy(), ref)
    say(f"[mig4 fp32 rhs] {e:.3e}")
    h.close()
    assert e <= 2e-4


def test_mig4_freestream_moving_on_gpu(gbr):
    """Uniform flow on the deforming grid with metrics recomputed every step:
    v and w stay at round-off with MIG4 too."""
    mv = W.Deforming3D((16, 14, 12), A=0.75, nmode=2, rand=0.2, seed=5)
    params = dict(viscous=True, limiter="mp", Re=1e3, Mref=0.5, scheme="mig4")
    g0 = mv.at(0.0)
    Q = W.uniform_flow(g0, 1.0, 1.0, 0.0, 0.0, 1.0 / (1.4 * 0.25))
    h = gbr.Grid(g0, **params)
    Qd = dev(Q)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    t = 0.0
    for s in range(10):
        gt = mv.at(t)
        h.step(Qd, 0.2, gbr.GBR_DT_CFL, xyz=dev(gt["xyz"]), xyz_t=dev(gt["xyz_t"]), dt_out=dt)
        t += dt.item()
    torch.cuda.synchronize()
    rho, u, v, w, p = oracle.prim_from_Q(Qd.cpu().numpy())
    vmax = max(np.abs(v).max(), np.abs(w).max())
    say(f"[mig4 freestream] 10 moving steps: max |v|,|w| {vmax:.3e}")
    h.close()
    assert vmax <= 1e-12

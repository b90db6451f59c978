"""Double periodic shear layer on a deforming mesh (Sec. 8.2; Re = 1e4,
M = 0.1, gamma = 5/3, unit square, mesh oscillating through one cycle to
t = 1).

The paper's reference curves are images, so what is checked is the property
the case demonstrates: the mesh motion does not change the flow. Kinetic
energy and enstrophy (Eq. KE-Ens, from gbr_diagnostics) on the deforming grid
follow those on a static grid of the same resolution, and MEG6 and MIG4
agree. Parity with the FP64 oracle on the deforming grid comes first.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PARAMS = dict(viscous=True, limiter="mp", gamma=5.0 / 3.0, Re=1e4, Mref=0.1)


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
    return max(float(np.abs(gpu[v] - ref[v]).max() / np.abs(ref[v]).max()) for v in range(ref.shape[0]))


@pytest.mark.parametrize("scheme", ["meg6", "mig4"])
def test_dpsl_steps_match_oracle(gbr, scheme):
    mv = W.Deforming2D((48, 48))
    params = dict(PARAMS, scheme=scheme)
    g = mv.at(0.0)
    Q = W.dpsl_ic(g)
    h = gbr.Grid(g, **params)
    Qd = dev(Q)
    t, dt = 0.0, 4e-4
    for s in range(3):
        gt = mv.at(t)
        h.step(Qd, dt, gbr.GBR_DT_FIXED, xyz=dev(gt["xyz"]), xyz_t=dev(gt["xyz_t"]))
        m = oracle.metrics(gt, **params)
        Q, _ = oracle.step(gt, m, Q, dt, dt_mode=oracle.DT_FIXED, **params)
        t += dt
    torch.cuda.synchronize()
    e = rel(Qd.cpu().numpy(), Q)
    say(f"[dpsl parity] {scheme}: 3 deforming-grid steps, max rel err {e:.3e}")
    assert h.check_state() == gbr.GBR_OK
    h.close()
    assert e <= 1e-12


def run_history(gbr, n, scheme, moving, t_end=1.0, steps_per_unit=5000, marks=(0.25, 0.5, 0.75, 1.0)):
    """KE and enstrophy at the marks; the mesh is moved on the device."""
    params = dict(PARAMS, scheme=scheme)
    mv = W.Deforming2D((n, n))
    g = mv.at(0.0) if moving else W.uniform2d((n, n), L=(1.0, 1.0))
    Q = dev(W.dpsl_ic(g))
    h = gbr.Grid(g, **params)
    if not moving:
        h.metrics(dev(g["xyz"]))
    base, mode = dev(mv.base), dev(mv.mode)
    w = 2 * math.pi * mv.omega
    integ = torch.zeros(3, dtype=torch.float64, device="cuda")
    nsteps = int(round(t_end * steps_per_unit))
    dt = t_end / nsteps
    out, k = [], 0
    for s in range(nsteps):
        t = s * dt
        if moving:
            xyz = base + math.sin(w * t) * mode
            xyz_t = (w * math.cos(w * t)) * mode
            h.step(Q, dt, gbr.GBR_DT_FIXED, xyz=xyz, xyz_t=xyz_t)
        else:
            h.step(Q, dt, gbr.GBR_DT_FIXED)
        if k < len(marks) and abs((s + 1) * dt - marks[k]) < 0.5 * dt:
            if moving:  # metrics at the mark's time for the volume weights
                tm = (s + 1) * dt
                h.metrics(base + math.sin(w * tm) * mode, (w * math.cos(w * tm)) * mode)
            h.diagnostics(Q, integrals=integ)
            ke, ens, _ = integ.tolist()
            out.append((marks[k], ke, ens))
            k += 1
    assert h.check_state() == gbr.GBR_OK
    h.close()
    return out


def histories(gbr, n):
    spu = 40 * n  # CFL about 0.28 with |u| + c = 11
    static = run_history(gbr, n, "meg6", moving=False, steps_per_unit=spu)
    moving = run_history(gbr, n, "meg6", moving=True, steps_per_unit=spu)
    mig4 = run_history(gbr, n, "mig4", moving=True, steps_per_unit=spu)
    worst = {"ke_mesh": 0.0, "ens_mesh": 0.0, "ke_scheme": 0.0, "ens_scheme": 0.0}
    for (t, ke_s, en_s), (_, ke_m, en_m), (_, ke_4, en_4) in zip(static, moving, mig4):
        say(f"[dpsl {n}^2] t = {t:.2f}: KE static {ke_s:.6f} moving {ke_m:.6f} MIG4 {ke_4:.6f}; "
            f"enstrophy static {en_s:.3f} moving {en_m:.3f} MIG4 {en_4:.3f}")
        worst["ke_mesh"] = max(worst["ke_mesh"], abs(ke_m - ke_s) / ke_s)
        worst["ens_mesh"] = max(worst["ens_mesh"], abs(en_m - en_s) / en_s)
        worst["ke_scheme"] = max(worst["ke_scheme"], abs(ke_4 - ke_m) / ke_m)
        worst["ens_scheme"] = max(worst["ens_scheme"], abs(en_4 - en_m) / en_m)
    say(f"[dpsl {n}^2] worst relative differences: {worst}")
    return worst


def test_dpsl_mesh_motion_leaves_energy_and_enstrophy(gbr):
    """At 256^2 the deforming-grid histories follow the static ones to 2e-4
    (KE) and 2 % (enstrophy), and the mesh-motion difference in enstrophy
    falls at least fourfold from 128^2 (it is a discretisation effect that
    refinement removes). MEG6 and MIG4 agree to 1e-3 in KE; their enstrophy,
    which the under-resolved layers of the roll-up make scheme-dependent,
    within 15 %."""
    coarse = histories(gbr, 128)
    fine = histories(gbr, 256)
    assert fine["ke_mesh"] <= 2e-4 and fine["ens_mesh"] <= 2e-2
    assert fine["ens_mesh"] <= coarse["ens_mesh"] / 4
    assert fine["ke_scheme"] <= 1e-3 and coarse["ke_scheme"] <= 1e-3
    assert fine["ens_scheme"] <= 0.15 and coarse["ens_scheme"] <= 0.15

"""Pins of the oracle's non-periodic boundaries: the App. C line closures,
the metrics built on them, the ghost-cell states of Sec. 6 and the sponge.

What fixes each piece independently of the oracle's own formulas:
- App. C line operator: exact first/second derivatives and interface values
  for quadratics at every cell and face (the printed placement of the
  partially one-sided stencil and the printed sign of the third-cell second
  derivative both fail this), mirror symmetry, order of accuracy.
- Metrics: exactness on affine grids, discrete metric identities and
  freestream with the boundary faces included.
- Ghost cells: on a Cartesian grid a wall boundary reproduces the periodic
  residual of the mirror-extended flow, a Dirichlet boundary that of the flow
  continued into the ghost cells, a zero-gradient boundary that of a flow
  constant near the ends; interior residuals never see deeper ghosts.
- Sponge: uniform flow relaxes by the SSP-RK3 polynomial of -sigma dt.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

NG = oracle.NG


# --------------------------------------------------------------------------
# App. C line operator
# --------------------------------------------------------------------------
@pytest.mark.parametrize("m", [12, 13, 20, 37])
def test_bline_exact_for_quadratics(m):
    x = np.arange(m, dtype=float) + 0.3
    for a, b, c in [(1.0, -2.0, 0.5), (0.0, 3.0, 1.0), (-0.7, 0.2, 2.0)]:
        v = a * x * x + b * x + c
        p, h = oracle.bline_derivs(v)
        assert np.abs(p - (2 * a * x + b)).max() <= 1e-12
        assert np.abs(h - 2 * a).max() <= 1e-12
        F = oracle.bline_faces(v)
        xf = np.arange(m + 1) - 0.5 + 0.3
        # the interior rule (Eq. FP-interp) gives f(x_f) - f''/24 for a
        # quadratic; the boundary closures must agree with it
        assert np.abs(F - (a * xf * xf + b * xf + c - 2 * a / 24)).max() <= 1e-12
        assert np.abs(np.diff(F) - (2 * a * x + b)).max() <= 1e-12


def test_bline_mirror_symmetry():
    rng = np.random.default_rng(5)
    v = rng.normal(size=23)
    F = oracle.bline_faces(v)
    Fr = oracle.bline_faces(v[::-1])
    assert np.abs(Fr - F[::-1]).max() <= 1e-14
    p, h = oracle.bline_derivs(v)
    pr, hr = oracle.bline_derivs(v[::-1])
    assert np.abs(pr + p[::-1]).max() <= 1e-13 and np.abs(hr - h[::-1]).max() <= 1e-13


def test_bline_orders():
    """Composite derivative: at least second order at the boundary cells
    (App. C is second order one-sided there), fourth order inside (the
    order of the periodic composite operator)."""
    errs_b, errs_i = [], []
    for m in (40, 80, 160):
        h = 1.0 / m
        x = (np.arange(m) + 0.5) * h
        v = np.sin(3 * x + 0.2)
        D = np.diff(oracle.bline_faces(v)) / h
        e = np.abs(D - 3 * np.cos(3 * x + 0.2))
        errs_b.append(e[:5].max())
        errs_i.append(e[m // 2 - 2:m // 2 + 2].max())
    ob = [math.log2(errs_b[k] / errs_b[k + 1]) for k in range(2)]
    oi = [math.log2(errs_i[k] / errs_i[k + 1]) for k in range(2)]
    assert min(ob) >= 1.9, (errs_b, ob)
    assert min(oi) >= 3.9, (errs_i, oi)


def test_bline_rejects_short_lines():
    with pytest.raises(ValueError):
        oracle.bline_faces(np.zeros(11))


# --------------------------------------------------------------------------
# metrics on bounded grids
# --------------------------------------------------------------------------
BGRIDS = {
    "wavy2d_x": lambda: W.bounded(W.wavy2d((30, 16), amp=0.1, rand=0.1, seed=2),
                                  [("inflow", "outflow")]),
    "wavy2d_xy": lambda: W.bounded(W.wavy2d((28, 26), amp=0.1), [("inflow", "outflow"), ("wall", "wall")]),
    "random3d_x": lambda: W.bounded(W.random3d((26, 7, 6), seed=3), [("inflow", "outflow")]),
    "sinusoidal3d_yz": lambda: W.bounded(W.sinusoidal3d((9, 25, 24)),
                                         [("periodic", "periodic"), ("outflow", "outflow"), ("wall", "outflow")]),
    "jet3d_xyz": lambda: W.bounded(W.jet3d((30, 26, 24)), [("inflow", "outflow"), ("outflow", "outflow"),
                                                          ("outflow", "outflow")]),
}


def _identity_error(g, m):
    inner = oracle.interior(g)
    worst = 0.0
    for c in range(3):
        s = 0.0
        for f in range(g["ndim"]):
            F = m[oracle.M_FHAT(f, c)]
            s = s + F - np.roll(F, 1, axis=2 - f)
        scale = max(np.abs(m[oracle.M_FHAT(f, c)]).max() for f in range(3))
        worst = max(worst, float(np.abs(s[inner]).max()) / scale)
    return worst


@pytest.mark.parametrize("name", sorted(BGRIDS))
def test_bounded_metric_identities_and_freestream(name):
    g = BGRIDS[name]()
    m = oracle.metrics(g)
    assert _identity_error(g, m) <= 1e-13
    # freestream: uniform flow, Dirichlet ghosts holding it, zero-gradient
    # elsewhere; walls replaced by outflow (uniform flow is not tangent to them)
    g2 = dict(g, bc=[tuple("outflow" if t == "wall" else t for t in b) for b in g["bc"]])
    Q = W.uniform_flow(g2, 1.0, 0.5, 0.3, 0.2 if g["ndim"] == 3 else 0.0, 1 / 1.4)
    inner = oracle.interior(g2)
    for params in (dict(viscous=False, limiter="mp"), dict(viscous=True, limiter="ducros", Re=200.0)):
        r = oracle.rhs(g2, m, Q, **params)
        scale = float(np.abs(m[oracle.M_FHAT(0, 0)]).max()) * 3.0
        assert np.abs(r[(slice(None),) + inner]).max() <= 1e-13 * scale, (name, params)


def test_bounded_ghost_residual_is_zero():
    g = BGRIDS["wavy2d_xy"]()
    m = oracle.metrics(g)
    Q = W.random_smooth_state(g, seed=3)
    r = oracle.rhs(g, m, Q, viscous=True, limiter="mp", Re=300.0)
    mask = np.ones(r.shape[1:], bool)
    mask[oracle.interior(g)] = False
    assert np.all(r[:, mask] == 0.0)
    assert np.abs(r[(slice(None),) + oracle.interior(g)]).max() > 0.0


def test_bounded_metrics_exact_on_affine_grid():
    n = (24, 25, 5)
    A = np.array([[1.0, 0.2, 0.1], [0.05, 0.8, 0.3], [0.0, 0.15, 1.2]])
    k, j, i = np.meshgrid(np.arange(n[2]) + 0.5, np.arange(n[1]) + 0.5, np.arange(n[0]) + 0.5, indexing="ij")
    xyz = np.stack([A[c, 0] * i + A[c, 1] * j + A[c, 2] * k for c in range(3)])
    off = [[A[c, d] * n[d] for c in range(3)] for d in range(3)]
    g = W.bounded({"n": n, "ndim": 3, "xyz": xyz, "off": np.array(off), "xyz_t": None},
                  [("inflow", "outflow"), ("wall", "wall")])
    m = oracle.metrics(g)
    inv = np.linalg.inv(A)
    for d in range(3):
        for c in range(3):
            assert np.abs(m[oracle.M_UNHAT(d, c)] - inv[d, c]).max() <= 1e-13
            assert np.abs(m[oracle.M_FUNHAT(d, d, c)] - inv[d, c]).max() <= 1e-13
    assert np.abs(m[oracle.M_INVJ] - np.linalg.det(A)).max() <= 1e-13


def test_bounded_rejects_unsupported():
    g = BGRIDS["random3d_x"]()
    with pytest.raises(NotImplementedError):
        oracle.metrics(g, scheme="mig4")
    mv = W.Deforming3D((26, 8, 8), seed=1).at(0.1)
    with pytest.raises(NotImplementedError):
        oracle.metrics(W.bounded(mv, [("inflow", "outflow")]))
    with pytest.raises(ValueError):
        W.bounded(W.wavy2d((20, 16)), [("inflow", "periodic")])
    with pytest.raises(ValueError):
        W.bounded(W.wavy2d((20, 16)), [("periodic", "periodic"), ("wall", "wall")])


# --------------------------------------------------------------------------
# ghost cells against periodic residuals (Cartesian grids: exact metrics)
# --------------------------------------------------------------------------
def _cartesian2d(nx, ny, hx, hy, y0=0.0):
    j, i = np.meshgrid(np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    xyz = np.stack([i * hx, y0 + j * hy, np.zeros_like(i)])[:, None]  # [3][nk = 1][nj][ni]
    return {"n": (nx, ny, 1), "ndim": 2, "xyz": xyz,
            "off": np.array([[nx * hx, 0, 0], [0, ny * hy, 0], [0, 0, 1.0]]), "xyz_t": None}


def _cartesian3d(n, h):
    k, j, i = np.meshgrid(*(np.arange(n[d]) + 0.5 for d in (2, 1, 0)), indexing="ij")
    xyz = np.stack([i * h[0], j * h[1], k * h[2]])
    return {"n": tuple(n), "ndim": 3, "xyz": xyz, "off": np.diag([n[d] * h[d] for d in range(3)]),
            "xyz_t": None}


PARAMS = [dict(viscous=False, limiter="mp"), dict(viscous=True, limiter="ducros", theta_c=0.2, Re=150.0),
          dict(viscous=True, limiter="none", Re=400.0)]


def _mirror_flow(x, y, Lx, H):
    """Flow symmetric about y = 0 and y = H (period 2H): rho, u, p even in y,
    v odd."""
    cx, sx = np.cos(2 * np.pi * x / Lx), np.sin(2 * np.pi * x / Lx)
    cy, sy = np.cos(np.pi * y / H), np.sin(np.pi * y / H)
    rho = 1.0 + 0.2 * cx * cy + 0.05 * np.cos(2 * np.pi * y / H)
    u = 0.4 + 0.1 * sx * cy
    v = 0.15 * sy * (1.0 + 0.3 * cx)
    p = 1.0 / 1.4 + 0.1 * cx * np.cos(2 * np.pi * y / H)
    return rho, u, v, p


@pytest.mark.parametrize("params", PARAMS, ids=["euler_mp", "ns_ducros", "ns_none"])
def test_wall_equals_mirrored_periodic_flow(params):
    nx, my = 16, 14
    hx, hy = 0.37, 0.29
    Lx, H = nx * hx, my * hy
    # periodic reference: y in (-H, H), the flow and its mirror image
    gp = _cartesian2d(nx, 2 * my, hx, hy, y0=-H)
    rho, u, v, p = _mirror_flow(gp["xyz"][0], gp["xyz"][1], Lx, H)
    Qp = W.conserved(rho, u, v, 0 * u, p, ndim=2)
    rp = oracle.rhs(gp, oracle.metrics(gp), Qp, **params)
    # bounded: y in (0, H) with walls, NG ghost rows each side (left unset)
    gb = W.bounded(_cartesian2d(nx, my + 2 * NG, hx, hy, y0=-NG * hy), [("periodic", "periodic"), ("wall", "wall")])
    rho, u, v, p = _mirror_flow(gb["xyz"][0], gb["xyz"][1], Lx, H)
    Qb = W.conserved(rho, u, v, 0 * u, p, ndim=2)
    Qb[:, :, :NG] = 7.0  # ghost contents are overwritten by the wall rule
    Qb[:, :, -NG:] = 7.0
    rb = oracle.rhs(gb, oracle.metrics(gb), Qb, **params)
    got = rb[:, :, NG:-NG]
    want = rp[:, :, my:]
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("params", PARAMS, ids=["euler_mp", "ns_ducros", "ns_none"])
def test_dirichlet_equals_periodic_residual(params):
    """With the ghost cells holding the flow's own values, interior residuals
    equal the periodic ones: the scheme never reaches beyond NG ghost layers."""
    n, h = (26, 7, 25), (0.3, 0.41, 0.35)
    gp = _cartesian3d(n, h)
    Q = W.random_smooth_state(gp, seed=11, amp=0.08)
    rp = oracle.rhs(gp, oracle.metrics(gp), Q, **params)
    gb = W.bounded(gp, [("inflow", "inflow"), ("periodic", "periodic"), ("inflow", "inflow")])
    rb = oracle.rhs(gb, oracle.metrics(gb), Q, **params)
    inner = (slice(None),) + oracle.interior(gb)
    assert np.abs(rb[inner] - rp[inner]).max() <= 1e-13 * np.abs(rp).max()


def test_zero_gradient_equals_periodic_for_flat_ends():
    """A flow that is constant (to round-off) within the stencil reach of
    both ends: zero-gradient ghosts hold the values a periodic continuation
    would, so the residuals agree."""
    n, h = (50, 9), (0.25, 0.3)
    gp = _cartesian2d(n[0], n[1], h[0], h[1])
    x, y = gp["xyz"][0], gp["xyz"][1]
    i = x / h[0] - 0.5
    bump = np.exp(-((i - 24.5) / 1.5) ** 2)  # < 1e-27 in the 13 cells next to each end
    rho = 1.0 + 0.3 * bump * (1 + 0.2 * np.sin(2 * np.pi * y / (n[1] * h[1])))
    u = 0.6 + 0.2 * bump
    v = 0.1 * bump * np.cos(2 * np.pi * y / (n[1] * h[1]))
    p = 1.0 / 1.4 + 0.1 * bump
    Q = W.conserved(rho, u, v, 0 * u, p, ndim=2)
    for params in PARAMS:
        rp = oracle.rhs(gp, oracle.metrics(gp), Q, **params)
        gb = W.bounded(gp, [("outflow", "outflow")])
        Qg = Q.copy()
        Qg[..., :NG] = 3.0
        Qg[..., -NG:] = 3.0
        rb = oracle.rhs(gb, oracle.metrics(gb), Qg, **params)
        inner = (slice(None),) + oracle.interior(gb)
        assert np.abs(rb[inner] - rp[inner]).max() <= 1e-13 * np.abs(rp).max(), params


def test_curvilinear_deep_interior_unaffected():
    """Away from the boundary (beyond the App. C closures and the stencils
    that read them) the bounded residual equals the periodic one."""
    gp = W.wavy2d((44, 20), amp=0.1)
    Q = W.random_smooth_state(gp, seed=4)
    params = dict(viscous=True, limiter="mp", Re=300.0)
    rp = oracle.rhs(gp, oracle.metrics(gp), Q, **params)
    gb = W.bounded(gp, [("inflow", "inflow")])
    rb = oracle.rhs(gb, oracle.metrics(gb), Q, **params)
    deep = (Ellipsis, slice(NG + 12, 44 - NG - 12))
    assert np.abs(rb[deep] - rp[deep]).max() <= 1e-13 * np.abs(rp).max()
    near = (Ellipsis, slice(NG, NG + 3))
    assert np.abs(rb[near] - rp[near]).max() > 1e-8  # App. C metrics differ near the boundary


def test_apply_bc_corner_and_wall_rules():
    g = W.bounded(W.wavy2d((26, 24), amp=0.1), [("outflow", "inflow"), ("wall", "outflow")])
    m4 = oracle.metrics(g)
    Q = W.random_smooth_state(g, seed=6)
    Qb = oracle.apply_bc(g, m4, Q)[:, 0]
    Q, m = Q[:, 0], m4[:, 0]  # drop the unit zeta axis
    nx = g["n"][0]
    # inflow side untouched, outflow side copies the boundary column
    assert np.array_equal(Qb[:, NG:-NG, -NG:], Q[:, NG:-NG, -NG:])
    assert np.array_equal(Qb[:, NG:-NG, :NG], np.repeat(Q[:, NG:-NG, NG:NG + 1], NG, axis=2))
    # wall: density and energy mirrored, normal momentum reversed, |momentum| kept
    for depth in range(NG):
        gho, src = Qb[:, NG - 1 - depth, NG:nx - NG], Q[:, NG + depth, NG:nx - NG]
        assert np.array_equal(gho[0], src[0]) and np.array_equal(gho[3], src[3])
        assert np.allclose(gho[1] ** 2 + gho[2] ** 2, src[1] ** 2 + src[2] ** 2, rtol=1e-14, atol=0)
        nrm = np.stack([m[oracle.M_FHAT(1, 0)][NG - 1, NG:nx - NG], m[oracle.M_FHAT(1, 1)][NG - 1, NG:nx - NG]])
        nrm = nrm / np.sqrt((nrm ** 2).sum(0))
        assert np.abs((gho[1] * nrm[0] + gho[2] * nrm[1]) + (src[1] * nrm[0] + src[2] * nrm[1])).max() <= 1e-14
    # corner ghosts: the later (eta) rule applied to the xi-filled values
    assert np.array_equal(Qb[:, -NG:, :NG], np.repeat(Qb[:, -NG - 1:-NG, :NG], NG, axis=1))


# --------------------------------------------------------------------------
# sponge, time step and stepping
# --------------------------------------------------------------------------
def test_sponge_relaxes_uniform_flow_by_rk3_polynomial():
    # zero-gradient sides only: the state stays uniform, so the flux part of
    # Res vanishes (a Dirichlet ghost would keep the unrelaxed state)
    g = W.bounded(W.jet3d((30, 26, 24)), [("outflow", "outflow")] * 3)
    m = oracle.metrics(g)
    Q0 = W.uniform_flow(g, 1.2, 0.4, -0.1, 0.2, 0.9)
    ref = (1.0, 0.1, 0.0, 0.0, 1.0 / 1.4)
    Qref = W.uniform_flow(g, *ref)
    sigma = np.full(Q0.shape[1:], 3.0)
    dt = 0.05
    Q1, _ = oracle.step(g, m, Q0, dt, dt_mode=oracle.DT_FIXED, viscous=True, limiter="ducros", Re=500.0,
                        sigma=sigma, qref=ref)
    z = 3.0 * dt
    amp = 1 - z + z * z / 2 - z ** 3 / 6
    inner = (slice(None),) + oracle.interior(g)
    want = Qref + amp * (Q0 - Qref)
    assert np.abs(Q1[inner] - want[inner]).max() <= 1e-13


def test_sponge_profile_shape():
    g = BGRIDS["wavy2d_x"]()
    s = W.sponge_sigma(g, width=5, amp=2.0, power=2.0)
    row = s[0, 0]
    assert np.all(row[:NG] == 0) and np.all(row[-NG:] == 0)
    assert row[NG] == 2.0 and row[NG + 4] == pytest.approx(2.0 * (1 / 5) ** 2) and row[NG + 5] == 0.0
    assert row[-NG - 1] == 2.0


def test_cfl_and_rk_ignore_ghost_cells():
    g = BGRIDS["sinusoidal3d_yz"]()
    m = oracle.metrics(g)
    Q = W.random_smooth_state(g, seed=2)
    Qg = Q.copy()
    mask = np.ones(Q.shape[1:], bool)
    mask[oracle.interior(g)] = False
    Qg[1][mask] *= 40.0  # fast ghost states would set a much smaller step
    params = dict(viscous=True, limiter="mp", Re=200.0)
    assert oracle.cfl_min(g, m, Qg, **params) == oracle.cfl_min(g, m, Q, **params)
    res = np.ones_like(Q)
    out = oracle.rk_stage(g, m, 0, 0.1, Q, Qg, res, **params)
    assert np.array_equal(out[:, mask], Qg[:, mask])


def test_step_keeps_inflow_ghosts_and_refills_others():
    g = W.bounded(W.wavy2d((30, 26), amp=0.08), [("inflow", "outflow"), ("wall", "wall")])
    m = oracle.metrics(g)
    Q = W.shu_vortex(g, eps=2.0)
    params = dict(viscous=False, limiter="mp")
    Q1, dt = oracle.step(g, m, Q, 0.4, **params)
    assert dt > 0
    assert np.array_equal(Q1[:, NG:-NG, :NG], Q[:, NG:-NG, :NG])
    assert np.array_equal(Q1, oracle.apply_bc(g, m, Q1, **params))
    assert np.abs(Q1 - Q).max() > 1e-6


@pytest.mark.parametrize("params", [dict(viscous=False, limiter="mp"),
                                    dict(viscous=True, limiter="ducros", theta_c=0.2, Re=200.0)],
                         ids=["euler_mp", "ns_ducros"])
def test_wall_box_conserves_mass_energy_and_tangential_momentum(params):
    """Slip walls (mirror ghosts) on a Cartesian box, periodic along x: the
    HLLC contact speed of mirrored states is zero, and the viscous shear and
    heat flux of a mirrored flow vanish at the wall, so the interior sums of
    rho/J, E/J and the wall-tangential momentum stay constant over steps."""
    nx, ny = 16, 12 + 2 * NG
    g = W.bounded(_cartesian2d(nx, ny, 0.3, 0.25, y0=-NG * 0.25), [("periodic", "periodic"), ("wall", "wall")])
    x, y = g["xyz"][0], g["xyz"][1]
    Lx = nx * 0.3
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x / Lx) * np.cos(1.3 * y)
    u = 0.3 + 0.1 * np.cos(2 * np.pi * x / Lx)
    v = 0.2 * np.sin(2.1 * y) * np.cos(2 * np.pi * x / Lx)
    p = 1.0 / 1.4 + 0.05 * np.sin(2 * np.pi * x / Lx + 0.4)
    Q = W.conserved(rho, u, v, 0 * u, p, ndim=2)
    m = oracle.metrics(g)
    inner = (slice(None),) + oracle.interior(g)
    vol = m[oracle.M_INVJ][oracle.interior(g)]
    tot0 = [(Q[inner][q] * vol).sum() for q in range(4)]
    for _ in range(4):
        Q, _ = oracle.step(g, m, Q, 0.4, **params)
    tot = [(Q[inner][q] * vol).sum() for q in range(4)]
    for q in (0, 1, 3):  # mass, x-momentum (tangential to the walls), energy
        assert abs(tot[q] - tot0[q]) <= 1e-13 * abs(tot0[q]), (q, tot[q] - tot0[q])
    assert abs(tot[2] - tot0[2]) > 1e-8  # the walls push on the normal momentum

"""Accuracy, conservation and time-integration pins of the oracle (Sec. 5.1
Step-7, Sec. 5.2, App. B), plus the 1-D Riemann problem against an exact
solver written here from the textbook mathematics (Toro, ch. 4)."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

G = 1.4


def _order(errs, ns):
    return [math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / ns[i]) for i in range(len(ns) - 1)]


def _dQdt(g, m, Q, **kw):
    return m[oracle.M_J] * oracle.rhs(g, m, Q, **kw)


@pytest.mark.parametrize("lim,min_order", [("none", 3.7)])
def test_entropy_wave_rhs_order(lim, min_order):
    """Linear advection of a density wave on the wavy curvilinear grid: the
    inviscid RHS is fourth-order accurate (Sec. 5.1, Step-7)."""
    ns, errs = [16, 32, 64], []
    for n in ns:
        g = W.wavy2d((n, n), L=10.0, amp=0.05)
        m = oracle.metrics(g)
        Q = W.entropy_wave(g, amp=0.2)
        x, y = g["xyz"][0], g["xyz"][1]
        k = 2 * np.pi / 10.0
        drho = -(1.0 + 1.0) * 0.2 * k * np.cos(k * (x + y))  # -(u d/dx + v d/dy) rho
        exact = np.stack([drho, drho * 1.0, drho * 1.0, drho * 0.5 * (1.0 + 1.0)])
        errs.append(np.abs(_dQdt(g, m, Q, limiter=lim) - exact).max())
    assert min(_order(errs, ns)) >= min_order, errs


def _vortex_exact_dqdt(g, eps=5.0, c=10.0, h=1e-5):
    """d/dt of the translating isentropic vortex: -(u_inf d/dx + v_inf d/dy) Q,
    with the spatial derivative of the closed form by central differences."""
    def q_at(dx, dy):
        gg = dict(g)
        xyz = g["xyz"].copy()
        xyz[0] += dx
        xyz[1] += dy
        gg["xyz"] = xyz
        return W.shu_vortex(gg, eps=eps, xc=c, yc=c)
    dqdx = (q_at(h, 0) - q_at(-h, 0)) / (2 * h)
    dqdy = (q_at(0, h) - q_at(0, -h)) / (2 * h)
    return -(dqdx + dqdy)


def test_isentropic_vortex_rhs_order():
    """Nonlinear vortex: the scheme drops to second order for nonlinear
    problems (Sec. 10), gate at 1.8 with the paper's MP limiter on."""
    ns, errs = [32, 64, 128], []
    for n in ns:
        g = W.wavy2d((n, n), L=20.0, amp=0.05)
        m = oracle.metrics(g)
        Q = W.shu_vortex(g, eps=5.0, xc=10.0, yc=10.0)
        errs.append(np.abs(_dQdt(g, m, Q, limiter="mp") - _vortex_exact_dqdt(g)).max())
    assert min(_order(errs, ns)) >= 1.8, errs


def _viscous_part(grid, n, a=0.1, L=10.0, Re=100.0):
    """Viscous part of J*Res (NS minus Euler, identical inviscid part) for
    u = a sin(k y), v = a sin(k x) at rho = 1, p = 1/gamma (T = 1, so mu is
    constant), and its exact value."""
    k = 2 * np.pi / L
    g = W.uniform2d((n, n), (L, L)) if grid == "cart" else W.wavy2d((n, n), L=L, amp=0.05)
    m = oracle.metrics(g)
    x, y = g["xyz"][0], g["xyz"][1]
    u, v = a * np.sin(k * y), a * np.sin(k * x)
    one = np.ones_like(x)
    Q = W.conserved(one, u, v, 0 * one, one / G, G, 2)
    kw = dict(limiter="none", Re=Re, Mref=1.0)
    visc = _dQdt(g, m, Q, viscous=True, **kw) - _dQdt(g, m, Q, viscous=False, **kw)
    mu = 1.0 / Re  # Sutherland normalised to 1 at T = 1
    txy = mu * a * k * (np.cos(k * y) + np.cos(k * x))
    mom_x = -mu * a * k * k * np.sin(k * y)
    mom_y = -mu * a * k * k * np.sin(k * x)
    # energy: d/dx(v txy) + d/dy(u txy)
    en = (a * k * np.cos(k * x)) * txy + v * (-mu * a * k * k * np.sin(k * x)) \
        + (a * k * np.cos(k * y)) * txy + u * (-mu * a * k * k * np.sin(k * y))
    return visc, np.stack([0 * one, mom_x, mom_y, en])


def test_alpha_damping_gradient_is_fourth_order():
    """Eq. AD-eqn1 with alpha_D = 4, beta_D = 0 gives a fourth-order interface
    gradient (Sec. 5.2). Isolated on a Cartesian grid where u = u(y) and
    v = v(x), so every stress is a normal derivative at its interface."""
    ns, errs = [16, 32, 64], []
    for n in ns:
        visc, exact = _viscous_part("cart", n)
        errs.append(max(np.abs(visc[1] - exact[1]).max(), np.abs(visc[2] - exact[2]).max()))
    o = _order(errs, ns)
    assert o[0] >= 3.3 and o[1] >= 3.7, errs


def test_viscous_terms_second_order_where_averages_enter():
    """The interface velocity (average of the beta_D = 0 states) in the work
    terms and the averaged tangential derivatives on skewed grids are second
    order: the energy term on the Cartesian grid and all terms on the wavy
    grid converge at order ~2."""
    for grid, comps in (("cart", [3]), ("wavy", [1, 2, 3])):
        ns, errs = [16, 32, 64], []
        for n in ns:
            visc, exact = _viscous_part(grid, n)
            errs.append(max(np.abs(visc[c] - exact[c]).max() for c in comps))
        assert min(_order(errs, ns)) >= 1.6, (grid, errs)


def test_ssprk3_amplification_factor():
    """Three stages on dQ/dt = lambda Q give 1 + z + z^2/2 + z^3/6 (App. B)."""
    g = W.uniform3d((2, 2, 2))
    m = np.zeros((oracle.M_TOTAL, 2, 2, 2))
    m[oracle.M_J] = 1.0
    lam, dt = -0.7, 0.3
    Q0 = np.random.default_rng(1).uniform(1, 2, size=(5, 2, 2, 2))
    Q = Q0.copy()
    for s in range(3):
        Q = oracle.rk_stage(g, m, s, dt, Q0, Q, lam * Q)
    z = lam * dt
    assert np.allclose(Q, (1 + z + z * z / 2 + z ** 3 / 6) * Q0, rtol=1e-14)


def test_rk_stage_uses_jacobian_and_gcl_term():
    """dQ/dt = J (Res - (1/J)_t Q) (Eq. time-split): one first stage with
    known J, (1/J)_t."""
    g = W.uniform3d((2, 2, 2))
    m = np.zeros((oracle.M_TOTAL, 2, 2, 2))
    m[oracle.M_J] = 2.0
    m[oracle.M_INVJT] = 0.25
    Q = np.full((5, 2, 2, 2), 3.0)
    res = np.full_like(Q, 1.0)
    out = oracle.rk_stage(g, m, 0, 0.1, Q, Q, res)
    assert np.allclose(out, 3.0 + 0.1 * 2.0 * (1.0 - 0.25 * 3.0), rtol=1e-15)


@pytest.mark.parametrize("moving", [False, True])
def test_periodic_conservation(moving):
    """Telescoping flux differences: sum over cells of Res vanishes to
    round-off on a periodic domain for any state (Sec. 3)."""
    if moving:
        g = W.Deforming3D((12, 10, 8), A=0.6, nmode=2, rand=0.2, seed=3).at(0.3)
    else:
        g = W.random3d((12, 10, 8), amp=0.2, seed=3)
    m = oracle.metrics(g)
    Q = W.random_rough_state(g, seed=4)
    r = oracle.rhs(g, m, Q, viscous=True, limiter="mp", Re=50.0)
    for v in range(5):
        assert abs(r[v].sum()) <= 1e-12 * np.abs(r[v]).sum()


def test_static_grid_conserves_q_over_j():
    """On a static grid sum(Q/J) is constant over SSP-RK3 steps."""
    g = W.random3d((10, 10, 10), amp=0.2, seed=12)
    m = oracle.metrics(g)
    Q = W.random_smooth_state(g, seed=5, amp=0.1)
    tot0 = (Q * m[oracle.M_INVJ]).sum(axis=(1, 2, 3))
    for _ in range(3):
        Q, _ = oracle.step(g, m, Q, 0.3, viscous=True, limiter="mp", Re=100.0)
    tot = (Q * m[oracle.M_INVJ]).sum(axis=(1, 2, 3))
    assert np.allclose(tot, tot0, rtol=1e-13, atol=1e-13)


def test_cfl_time_step_closed_form():
    """On a uniform Cartesian grid with uniform flow the time step of App. B
    is CFL * min_d dx_d / (|u_d| + c), and with viscosity also
    min_d dx_d^2 / (alpha nu)."""
    g = W.uniform3d((8, 8, 8), (2.0, 1.0, 4.0))
    m = oracle.metrics(g)
    u = np.array([0.3, -1.2, 0.5])
    rho, p = 1.3, 0.9
    Q = W.uniform_flow(g, rho, *u, p)
    c = math.sqrt(G * p / rho)
    dx = np.array([2.0, 1.0, 4.0]) / 8
    inv = min(dx / (np.abs(u) + c))
    assert oracle.cfl_min(g, m, Q) == pytest.approx(inv, rel=1e-13)
    Re, Mref = 20.0, 1.0
    T = G * Mref * Mref * p / rho
    S = 110.4 / 293.0
    nu = T ** 1.5 * (1 + S) / (T + S) / Re / rho
    vis = min(dx ** 2) / (4.0 * nu)
    assert oracle.cfl_min(g, m, Q, viscous=True, Re=Re) == pytest.approx(min(inv, vis), rel=1e-13)


# ----------------------------------------------------------------------------
# exact Riemann solver (Toro, Riemann Solvers and Numerical Methods, ch. 4)
# ----------------------------------------------------------------------------
def exact_riemann(WL, WR, xi, gamma=G):
    rl, ul, pl = WL
    rr, ur, pr = WR
    cl, cr = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    g1 = (gamma - 1) / (2 * gamma)
    g2 = (gamma + 1) / (2 * gamma)

    def fK(p, rK, pK, cK):
        if p > pK:
            A = 2 / ((gamma + 1) * rK)
            B = (gamma - 1) / (gamma + 1) * pK
            f = (p - pK) * math.sqrt(A / (p + B))
            df = math.sqrt(A / (B + p)) * (1 - (p - pK) / (2 * (B + p)))
        else:
            f = 2 * cK / (gamma - 1) * ((p / pK) ** g1 - 1)
            df = 1 / (rK * cK) * (p / pK) ** (-g2)
        return f, df

    p = 0.5 * (pl + pr)
    for _ in range(100):
        f1, d1 = fK(p, rl, pl, cl)
        f2, d2 = fK(p, rr, pr, cr)
        dp = (f1 + f2 + ur - ul) / (d1 + d2)
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-15 * p:
            break
    f1, _ = fK(p, rl, pl, cl)
    f2, _ = fK(p, rr, pr, cr)
    us = 0.5 * (ul + ur) + 0.5 * (f2 - f1)

    out = np.zeros((3, len(xi)))
    for q, s in enumerate(xi):
        if s <= us:
            r0, u0, p0, c0 = rl, ul, pl, cl
            if p > pl:
                rs = rl * ((p / pl + (gamma - 1) / (gamma + 1)) / ((gamma - 1) / (gamma + 1) * p / pl + 1))
                S = ul - cl * math.sqrt(g2 * p / pl + g1)
                out[:, q] = (r0, u0, p0) if s <= S else (rs, us, p)
            else:
                rs = rl * (p / pl) ** (1 / gamma)
                csl = cl * (p / pl) ** g1
                if s <= ul - cl:
                    out[:, q] = (r0, u0, p0)
                elif s >= us - csl:
                    out[:, q] = (rs, us, p)
                else:
                    uu = 2 / (gamma + 1) * (cl + (gamma - 1) / 2 * ul + s)
                    cc = 2 / (gamma + 1) * (cl + (gamma - 1) / 2 * (ul - s))
                    rrr = rl * (cc / cl) ** (2 / (gamma - 1))
                    out[:, q] = (rrr, uu, pl * (cc / cl) ** (2 * gamma / (gamma - 1)))
        else:
            if p > pr:
                rs = rr * ((p / pr + (gamma - 1) / (gamma + 1)) / ((gamma - 1) / (gamma + 1) * p / pr + 1))
                S = ur + cr * math.sqrt(g2 * p / pr + g1)
                out[:, q] = (rr, ur, pr) if s >= S else (rs, us, p)
            else:
                rs = rr * (p / pr) ** (1 / gamma)
                csr = cr * (p / pr) ** g1
                if s >= ur + cr:
                    out[:, q] = (rr, ur, pr)
                elif s <= us + csr:
                    out[:, q] = (rs, us, p)
                else:
                    uu = 2 / (gamma + 1) * (-cr + (gamma - 1) / 2 * ur + s)
                    cc = 2 / (gamma + 1) * (cr - (gamma - 1) / 2 * (ur - s))
                    rrr = rr * (cc / cr) ** (2 / (gamma - 1))
                    out[:, q] = (rrr, uu, pr * (cc / cr) ** (2 * gamma / (gamma - 1)))
    return out


def test_exact_riemann_solver_self_check():
    """The test's exact solver reproduces Toro's tabulated Sod star state
    (p* = 0.30313, u* = 0.92745; Toro Table 4.3, test 1)."""
    s = exact_riemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), np.array([0.0]))
    assert s[2, 0] == pytest.approx(0.30313, abs=1e-5)
    assert s[1, 0] == pytest.approx(0.92745, abs=1e-5)


def _sod_run(n, rotate=0.0):
    """Sod along xi on a one-cell-thick 2-D strip of length 2 (interface at
    x = 1), optionally rotated; SSP-RK3, CFL 0.2, t = 0.2."""
    L, h = 2.0, 0.05
    c, s = math.cos(rotate), math.sin(rotate)
    i = (np.arange(n) + 0.5) * (L / n)
    xyz = np.zeros((3, 1, 1, n))
    xyz[0, 0, 0] = c * i - s * 0.5 * h
    xyz[1, 0, 0] = s * i + c * 0.5 * h
    off = np.array([[c * L, s * L, 0.0], [-s * h, c * h, 0.0], [0.0, 0.0, 1.0]])
    g = dict(n=(n, 1, 1), ndim=2, xyz=xyz, off=off, xyz_t=None)
    m = oracle.metrics(g)
    left = i < 1.0
    rho = np.where(left, 1.0, 0.125)[None, None, :]
    p = np.where(left, 1.0, 0.1)[None, None, :]
    z = np.zeros_like(rho)
    Q = W.conserved(rho, z, z, z, p, G, 2)
    t = 0.0
    while t < 0.2 - 1e-14:
        dt = min(0.2 * oracle.cfl_min(g, m, Q), 0.2 - t)
        Q, _ = oracle.step(g, m, Q, dt, dt_mode=oracle.DT_FIXED, limiter="mp")
        t += dt
    rho, u, v, w, p = oracle.prim_from_Q(Q)
    un = c * u + s * v
    return i, rho[0, 0], un[0, 0], p[0, 0]


@pytest.mark.slow
def test_sod_against_exact_riemann_solution():
    """L1 density error against the exact solution falls with refinement at
    order >= 0.6 (shock-capturing), no overshoot beyond 1 %, and a 30-degree
    rotated strip gives the same solution to round-off."""
    ns, errs = [100, 200, 400], []
    for n in ns:
        x, rho, un, p = _sod_run(n)
        win = (x > 0.55) & (x < 1.45)
        ex = exact_riemann((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), (x[win] - 1.0) / 0.2)
        errs.append(np.mean(np.abs(rho[win] - ex[0])) * 0.9)
        assert rho.max() <= 1.0 * 1.01 and rho.min() >= 0.125 * 0.99
    assert errs[0] > errs[1] > errs[2]
    assert min(_order(errs, ns)) >= 0.6, errs
    x, rho_r, un_r, p_r = _sod_run(200, rotate=math.pi / 6)
    x, rho_0, un_0, p_0 = _sod_run(200)
    assert np.abs(rho_r - rho_0).max() < 1e-11
    assert np.abs(p_r - p_0).max() < 1e-11

"""Pins of the oracle's eigenstructure (App. A), HLLC flux (Sec. 5.1.1),
MP limiter (App. E) and symmetries of the assembled right-hand side."""
import numpy as np
import pytest

import oracle
import workloads as W

G = 1.4
rng = np.random.default_rng(42)


def _unit(v):
    return v / np.linalg.norm(v)


def _B_primitive(rho, u, p, n):
    """Primitive-variable coefficient matrix of App. A for a unit normal n and
    zero grid speed (the printed B-bar with the 1/J factor dropped)."""
    U = n @ u
    B = np.zeros((5, 5))
    B[0, 0] = U
    B[0, 1:4] = rho * n
    for a in range(3):
        B[1 + a, 1 + a] = U
        B[1 + a, 4] = n[a] / rho
    B[4, 1:4] = G * p * n
    B[4, 4] = U
    return B


@pytest.mark.parametrize("trial", range(6))
def test_eigenvectors_diagonalise_primitive_jacobian(trial):
    n = _unit(rng.normal(size=3))
    rho, p = rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0)
    u = rng.normal(size=3)
    a = np.sqrt(G * p / rho)
    R, Ri = oracle.eigvec(n, rho, a)
    assert np.allclose(R @ Ri, np.eye(5), atol=1e-13)
    lam = Ri @ _B_primitive(rho, u, p, n) @ R
    U = n @ u
    assert np.allclose(lam, np.diag([U - a, U, U, U, U + a]), atol=1e-12)


def _toro_hllc(PL, PR, gamma=G):
    """Textbook Cartesian HLLC along x (Toro, Riemann Solvers, Sec. 10.4),
    written independently of the curvilinear form of the paper."""
    def cons(P):
        r, u, v, w, p = P
        return np.array([r, r * u, r * v, r * w, p / (gamma - 1) + 0.5 * r * (u * u + v * v + w * w)])

    def flux(P):
        r, u, v, w, p = P
        E = cons(P)[4]
        return np.array([r * u, r * u * u + p, r * u * v, r * u * w, u * (E + p)])

    rl, ul, vl, wl, pl = PL
    rr, ur, vr, wr, pr = PR
    cl, cr = np.sqrt(gamma * pl / rl), np.sqrt(gamma * pr / rr)
    sl = min(ul - cl, ur - cr)
    sr = max(ul + cl, ur + cr)
    ss = (pr - pl + rl * ul * (sl - ul) - rr * ur * (sr - ur)) / (rl * (sl - ul) - rr * (sr - ur))
    if sl >= 0:
        return flux(PL)
    if sr <= 0:
        return flux(PR)

    def star(P, s):
        r, u, v, w, p = P
        E = cons(P)[4]
        f = r * (s - u) / (s - ss)
        return f * np.array([1.0, ss, v, w, E / r + (ss - u) * (ss + p / (r * (s - u)))])

    if ss >= 0:
        return flux(PL) + sl * (star(PL, sl) - cons(PL))
    return flux(PR) + sr * (star(PR, sr) - cons(PR))


def _rand_state(uscale=0.6):
    return np.array([rng.uniform(0.3, 2), *rng.normal(scale=uscale, size=3), rng.uniform(0.3, 2)])


@pytest.mark.parametrize("trial", range(40))
def test_hllc_reduces_to_textbook_cartesian(trial):
    PL, PR = _rand_state(1.5), _rand_state(1.5)
    F = oracle.hllc(PL, PR, [0.0, 1.0, 0.0, 0.0])
    assert np.allclose(F, _toro_hllc(PL, PR), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("trial", range(10))
def test_hllc_consistency(trial):
    P = _rand_state()
    nt_n = np.array([rng.normal(), *rng.normal(size=3)])
    assert np.allclose(oracle.hllc(P, P, nt_n), oracle.euler_flux(P, nt_n), rtol=1e-12, atol=1e-12)


def _rot(axis, ang):
    axis = _unit(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


@pytest.mark.parametrize("trial", range(10))
def test_hllc_rotation_and_scaling_invariance(trial):
    PL, PR = _rand_state(1.2), _rand_state(1.2)
    n = _unit(rng.normal(size=3)) * rng.uniform(0.2, 3.0)
    F = oracle.hllc(PL, PR, [0.0, *n])
    Rm = _rot(rng.normal(size=3), rng.uniform(0, 2 * np.pi))
    rot = lambda P: np.array([P[0], *(Rm @ P[1:4]), P[4]])
    Fr = oracle.hllc(rot(PL), rot(PR), [0.0, *(Rm @ n)])
    assert np.allclose(Fr[[0, 4]], F[[0, 4]], rtol=1e-12, atol=1e-12)
    assert np.allclose(Fr[1:4], Rm @ F[1:4], rtol=1e-12, atol=1e-12)
    k = rng.uniform(0.1, 10.0)
    assert np.allclose(oracle.hllc(PL, PR, [0.0, *(k * n)]), k * F, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("trial", range(20))
def test_hllc_moving_face_is_galilean(trial):
    """A face moving with velocity vg has hat-xi_t = -n . vg. Its flux equals
    the static-face flux of the states seen from the face, transformed back:
    mass F0, momentum F0' + vg F0, energy F0'' + vg.F' + |vg|^2/2 F0. This pins
    the grid-speed terms of the curvilinear HLLC."""
    PL, PR = _rand_state(1.0), _rand_state(1.0)
    n = rng.normal(size=3)
    vg = rng.normal(scale=0.7, size=3)
    rel = lambda P: np.array([P[0], *(P[1:4] - vg), P[4]])
    F = oracle.hllc(PL, PR, [-(n @ vg), *n])
    Fs = oracle.hllc(rel(PL), rel(PR), [0.0, *n])
    expect = np.empty(5)
    expect[0] = Fs[0]
    expect[1:4] = Fs[1:4] + vg * Fs[0]
    expect[4] = Fs[4] + vg @ Fs[1:4] + 0.5 * (vg @ vg) * Fs[0]
    assert np.allclose(F, expect, rtol=1e-11, atol=1e-11)


def test_mp_limiter_keeps_smooth_and_linear_data():
    # linear data: curvatures zero, interface value between the cells -> kept
    for slope in (-1.3, 0.0, 2.0):
        w = slope * np.arange(-1, 3)
        wl = w[1] + 0.5 * slope
        assert oracle.mp_limit(w[0], w[1], w[2], 0, 0, 0, wl) == pytest.approx(wl, abs=1e-15)
    # constant data
    assert oracle.mp_limit(1.0, 1.0, 1.0, 0, 0, 0, 1.0) == 1.0


def test_mp_limiter_removes_overshoot_at_a_step():
    """At a discontinuity an overshooting interface value is pulled back into
    the monotonicity bounds (no new extrema)."""
    wm1, w0, wp1 = 0.0, 0.0, 1.0
    d = [0.0, 2.0, -2.0]
    out = oracle.mp_limit(wm1, w0, wp1, d[0], d[1], d[2], 1.7)
    assert 0.0 <= out <= 1.0
    out = oracle.mp_limit(wm1, w0, wp1, d[0], d[1], d[2], -0.4)
    assert 0.0 <= out <= 1.0


@pytest.mark.parametrize("trial", range(200))
def test_mp_limiter_preserves_monotonicity(trial):
    """Monotone cell data with zero curvature: whatever the unlimited interface
    value, the limited one lies between the two adjacent cell values (the
    monotonicity-preserving property the limiter exists for)."""
    steps = rng.uniform(0, 1, size=2) * rng.choice([-1.0, 1.0])
    w = np.cumsum(np.concatenate([[rng.normal()], steps]))  # monotone triple
    wf = w[1] + rng.normal() * 3
    out = oracle.mp_limit(w[0], w[1], w[2], 0.0, 0.0, 0.0, wf)
    lo, hi = min(w[1], w[2]), max(w[1], w[2])
    assert lo - 1e-12 <= out <= hi + 1e-12
    # the admissible interval also stops at the upper limit
    # w_UL = w0 + alpha (w0 - w-1) (alpha = 4): inside it the value is kept
    wul = w[1] + 4.0 * (w[1] - w[0])
    near = w[2] if abs(w[2] - w[1]) <= abs(wul - w[1]) else wul
    if min(w[1], near) <= wf <= max(w[1], near):
        assert out == pytest.approx(wf, abs=1e-15)
    else:
        assert out == pytest.approx(near if abs(wf - near) < abs(wf - w[1]) else w[1], abs=1e-12)


def _mirror_x(g, Q):
    """Reflect a 3-D grid and state through x = 0 with the xi index reversed
    (keeps a right-handed index frame). Returns the mirrored (grid, Q)."""
    xyz = g["xyz"][:, :, :, ::-1].copy()
    xyz[0] = -xyz[0]
    Qm = Q[:, :, :, ::-1].copy()
    Qm[1] = -Qm[1]
    g2 = dict(g)
    g2["xyz"] = xyz
    return g2, Qm


@pytest.mark.parametrize("visc", [False, True])
@pytest.mark.parametrize("lim", ["mp", "ducros"])
def test_rhs_mirror_symmetry(visc, lim):
    """Reversing xi with x -> -x, u -> -u mirrors Res (rho u component
    negated). Exercises the left/right symmetry of reconstruction and limiter.
    The grid is axis-aligned: there each characteristic variable of App. A
    maps to +-itself under the reflection. On oblique faces the three middle
    rows of R^-1 mix the entropy variable with components of n x u, so a
    component-wise limiter is not reflection-covariant there (a property of
    the printed eigenvectors, not of the implementation)."""
    g = W.uniform3d((10, 8, 6), (1.0, 0.9, 0.7))
    Q = W.random_rough_state(g, seed=3)
    m = oracle.metrics(g)
    r = oracle.rhs(g, m, Q, viscous=visc, limiter=lim, theta_c=0.3)
    # the limiter really changes the result here
    assert np.abs(r - oracle.rhs(g, m, Q, viscous=visc, limiter="none")).max() > 1e-3
    g2, Q2 = _mirror_x(g, Q)
    m2 = oracle.metrics(g2)
    r2 = oracle.rhs(g2, m2, Q2, viscous=visc, limiter=lim, theta_c=0.3)
    back = r2[:, :, :, ::-1].copy()
    back[1] = -back[1]
    assert np.abs(back - r).max() <= 1e-12 * np.abs(r).max()


def test_rhs_rotation_invariance_2d():
    """Rotating a 2-D grid and the velocity field by 30 degrees rotates the
    momentum residual and leaves the others unchanged (the unit normals of
    the characteristic projection and the HLLC rotate with the grid)."""
    g = W.wavy2d((16, 12), L=2.0, amp=0.05, rand=0.1, seed=2)
    Q = W.random_rough_state(g, seed=8)
    m = oracle.metrics(g)
    r = oracle.rhs(g, m, Q, limiter="mp")
    th = np.pi / 6
    c, s = np.cos(th), np.sin(th)
    g2 = dict(g)
    xyz = g["xyz"].copy()
    xyz[0], xyz[1] = c * g["xyz"][0] - s * g["xyz"][1], s * g["xyz"][0] + c * g["xyz"][1]
    off = g["off"].copy()
    for d in range(2):
        off[d, 0], off[d, 1] = c * g["off"][d, 0] - s * g["off"][d, 1], s * g["off"][d, 0] + c * g["off"][d, 1]
    g2["xyz"], g2["off"] = xyz, off
    Q2 = Q.copy()
    Q2[1], Q2[2] = c * Q[1] - s * Q[2], s * Q[1] + c * Q[2]
    m2 = oracle.metrics(g2)
    r2 = oracle.rhs(g2, m2, Q2, limiter="mp")
    expect = r.copy()
    expect[1], expect[2] = c * r[1] - s * r[2], s * r[1] + c * r[2]
    assert np.abs(r2 - expect).max() <= 1e-12 * np.abs(r).max()

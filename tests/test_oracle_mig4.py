"""Pins of the oracle's MIG4 scheme: IG4 gradients (Eq. IG4_grads, read as
differences like Eq. E6_grads, alpha = 5/14), the metrics built on them
(Sec. 7 with IG4 in Eq. FP-interp, as the paper directs for MIG4) and the
RHS with IG4 gradients in place of E6 (Sec. 5.1 Step-1).

The IG4 solver is checked against the Fourier symbol of the printed scheme,
a linear-plus-periodic line (the periodic-offset case the metrics need),
fourth-order convergence, and exactness of the metrics on affine grids; the
metrics against the discrete metric identities and freestream; the RHS
against fourth-order convergence on a linear wave.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

ALPHA = 5.0 / 14.0


def symbol(w):
    """i * k_eff(w) of the IG4 scheme for a mode exp(i w k): the printed
    left-hand side multiplies by 1 + 2 alpha cos w, the right-hand side by
    2 i (a sin w + b sin 2w), a = 2 (2 + alpha) / 6, b = (4 alpha - 1) / 12."""
    a = 2 * (2 + ALPHA) / 6
    b = (4 * ALPHA - 1) / 12
    return (2 * a * np.sin(w) + 2 * b * np.sin(2 * w)) / (1 + 2 * ALPHA * np.cos(w))


@pytest.mark.parametrize("n", [3, 4, 5, 8, 17, 32])
def test_ig4_matches_fourier_symbol(n):
    k = np.arange(n)
    for m in range(1, (n + 1) // 2):
        w = 2 * np.pi * m / n
        for f, df in ((np.sin(w * k), np.cos(w * k)), (np.cos(w * k), -np.sin(w * k))):
            got = oracle.line_ig4(f)
            assert np.abs(got - symbol(w) * df).max() <= 1e-13, (n, m)


def test_ig4_symbol_is_fourth_order():
    """k_eff(w) - w = O(w^5): the scheme is consistent at fourth order."""
    ws = np.array([0.2, 0.1, 0.05])
    err = np.abs(symbol(ws) - ws)
    orders = np.log(err[:-1] / err[1:]) / np.log(2.0)
    assert (orders > 4.9).all(), orders


def test_ig4_linear_plus_periodic_line():
    """A coordinate-like line v[i] = s i + periodic, extended by v[i+n] =
    v[i] + s n: the derivative is s plus that of the periodic part."""
    for n in (1, 2, 3, 7, 24):
        k = np.arange(n)
        per = np.sin(2 * np.pi * k / n) if n > 2 else np.zeros(n)
        v = 0.37 * k + per
        got = oracle.line_ig4(v, shift=0.37 * n)
        want = 0.37 + (symbol(2 * np.pi / n) * np.cos(2 * np.pi * k / n) if n > 2 else 0.0)
        assert np.abs(got - want).max() <= 1e-13, n


def test_ig4_converges_at_fourth_order():
    ns, errs = [32, 64, 128], []
    for n in ns:
        h = 2 * np.pi / n
        x = np.arange(n) * h
        f = np.exp(np.sin(x))
        errs.append(np.abs(oracle.line_ig4(f) - h * np.cos(x) * f).max())
    orders = [math.log(errs[i] / errs[i + 1], 2) for i in range(2)]
    assert min(orders) >= 3.9, (errs, orders)


def test_ig4_composite_derivative_and_faces_on_linear_lines():
    """Interface values of a linear line are its midpoints and their
    difference is its slope (Eq. FP-interp, FP-interp2 with IG4)."""
    for n in (1, 4, 9):
        k = np.arange(n)
        v = 1.5 + 0.25 * k
        assert np.abs(oracle.line_ig4_face(v, shift=0.25 * n) - (1.5 + 0.25 * (k + 0.5))).max() <= 1e-14
        assert np.abs(oracle.line_ig4_dcomp(v, shift=0.25 * n) - 0.25).max() <= 1e-14


def _identity_error(g, m):
    worst = 0.0
    for c in range(3):
        s = 0.0
        for f in range(g["ndim"]):
            F = m[oracle.M_FHAT(f, c)]
            s = s + F - np.roll(F, 1, axis=2 - f)
        scale = max(np.abs(m[oracle.M_FHAT(f, c)]).max() for f in range(3))
        worst = max(worst, float(np.abs(s).max()) / scale)
    return worst


GRIDS = {
    "random3d": lambda: W.random3d((8, 7, 6), seed=3),
    "sinusoidal3d": lambda: W.sinusoidal3d((9, 8, 7)),
    "wavy2d_random": lambda: W.wavy2d((12, 10), rand=0.2, seed=2),
    "tiny": lambda: W.random3d((4, 3, 2), seed=1),
    "deforming": lambda: W.Deforming3D((10, 9, 8), A=0.75, nmode=2, rand=0.2, seed=4).at(0.17),
}


@pytest.mark.parametrize("name", sorted(GRIDS))
def test_mig4_metric_identities_and_freestream(name):
    g = GRIDS[name]()
    m = oracle.metrics(g, scheme="mig4")
    assert _identity_error(g, m) <= 1e-13
    Q = W.uniform_flow(g, 1.0, 0.5, 0.3, 0.2 if g["ndim"] == 3 else 0.0, 1 / 1.4)
    for params in (dict(viscous=False, limiter="mp"), dict(viscous=True, limiter="ducros", Re=200.0)):
        r = oracle.rhs(g, m, Q, scheme="mig4", **params)
        if g.get("xyz_t") is not None:
            r = r - m[oracle.M_INVJT] * Q  # moving freestream: Res balances the GCL term
        scale = float(np.abs(m[oracle.M_FHAT(0, 0)]).max()) * 3.0
        assert np.abs(r).max() <= 1e-13 * scale, (name, params)


def test_mig4_metrics_exact_on_affine_grid():
    """Every central scheme is exact for linear coordinates."""
    n = (6, 5, 4)
    A = np.array([[1.0, 0.2, 0.1], [0.05, 0.8, 0.3], [0.0, 0.15, 1.2]])
    k, j, i = np.meshgrid(np.arange(n[2]) + 0.5, np.arange(n[1]) + 0.5, np.arange(n[0]) + 0.5, indexing="ij")
    xyz = np.stack([A[c, 0] * i + A[c, 1] * j + A[c, 2] * k for c in range(3)])
    off = [[A[c, d] * n[d] for c in range(3)] for d in range(3)]
    g = {"n": n, "ndim": 3, "xyz": xyz, "off": off, "xyz_t": None}
    m = oracle.metrics(g, scheme="mig4")
    inv = np.linalg.inv(A)  # d(xi, eta, zeta)/d(x, y, z)
    for d in range(3):
        for c in range(3):
            assert np.abs(m[oracle.M_UNHAT(d, c)] - inv[d, c]).max() <= 1e-13
    assert np.abs(m[oracle.M_INVJ] - np.linalg.det(A)).max() <= 1e-13


def test_mig4_entropy_wave_rhs_is_fourth_order():
    ns, errs = [16, 32, 64], []
    for n in ns:
        g = W.wavy2d((n, n), L=10.0, amp=0.05)
        m = oracle.metrics(g, scheme="mig4")
        Q = W.entropy_wave(g, amp=0.2)
        x, y = g["xyz"][0], g["xyz"][1]
        k = 2 * np.pi / 10.0
        drho = -2.0 * 0.2 * k * np.cos(k * (x + y))
        exact = np.stack([drho, drho, drho, drho])
        got = m[oracle.M_J] * oracle.rhs(g, m, Q, scheme="mig4", limiter="none")
        errs.append(np.abs(got - exact).max())
    orders = [math.log(errs[i] / errs[i + 1], 2) for i in range(2)]
    assert min(orders) >= 3.7, (errs, orders)


def test_mig4_differs_from_meg6_on_rough_data():
    g = W.random3d((8, 7, 6), seed=5)
    Q = W.random_rough_state(g, seed=2)
    r6 = oracle.rhs(g, oracle.metrics(g), Q)
    r4 = oracle.rhs(g, oracle.metrics(g, scheme="mig4"), Q, scheme="mig4")
    assert np.abs(r6 - r4).max() > 1e-3 * np.abs(r6).max()


def test_mig4_cell_gradients_are_ig4_of_each_field():
    """The MIG4 cell gradients (viscous tangential terms, sensor) in slot
    (d, s), s = u, v, w, T, equal the IG4 line derivative of that field along
    d (T = gamma Mref^2 p / rho, Sec. 2)."""
    g = W.random3d((7, 6, 5), seed=8)
    Q = W.random_rough_state(g, seed=3, amp=0.2)
    Mref = 0.7
    grad = oracle.gradients(g, Q, scheme="mig4", Mref=Mref)
    rho, u, v, w, p = oracle.prim_from_Q(Q)
    T = 1.4 * Mref * Mref * p / rho
    fields = [u, v, w, T]
    for d in range(3):
        axis = 2 - d
        for s, f in enumerate(fields):
            want = np.apply_along_axis(oracle.line_ig4, axis, f)
            assert np.abs(grad[d * 4 + s] - want).max() <= 1e-13 * max(1.0, np.abs(want).max()), (d, s)

"""Pins of the oracle's shared-gradient diagnostics (vorticity, Q-criterion,
density-gradient magnitude; kinetic-energy and enstrophy averages of
Eq. KE-Ens) against closed forms."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def shear_state(g, A=0.3, B=0.2, rho0=1.0, amp_rho=0.1, p=1.0, L=10.0):
    """u = A sin(k y), v = B sin(k x), w = 0, rho = rho0 + amp sin(k x), k = 2 pi / L."""
    k = 2 * np.pi / L
    x, y = g["xyz"][0], g["xyz"][1]
    u = A * np.sin(k * y)
    v = B * np.sin(k * x)
    rho = rho0 + amp_rho * np.sin(k * x)
    z = np.zeros_like(u)
    return W.conserved(rho, u, v, z, p + z, 1.4, g["ndim"]), k, x, y


@pytest.mark.parametrize("scheme", ["meg6", "mig4"])
def test_shear_flow_closed_forms(scheme):
    """omega_z = B k cos kx - A k cos ky, Q = -(A k cos ky)(B k cos kx),
    |grad rho| = amp k |cos kx|; with rho = 1 the averages are
    E_k = (A^2 + B^2) / 4 and enstrophy = k^2 (A^2 + B^2) / 4."""
    A, B = 0.3, 0.2
    errs = []
    for n in (32, 64):
        g = W.uniform2d((n, n), L=(10.0, 10.0))
        m = oracle.metrics(g, scheme=scheme)
        Q, k, x, y = shear_state(g, A, B)
        f, (ke, ens, vol) = oracle.diagnostics(g, m, Q, scheme=scheme)
        a, b = A * k * np.cos(k * y), B * k * np.cos(k * x)
        errs.append(max(np.abs(f[2] - (b - a)).max(), np.abs(f[3] + a * b).max(),
                        np.abs(f[4] - 0.1 * k * np.abs(np.cos(k * x))).max()))
        assert np.abs(f[0]).max() <= 1e-15 and np.abs(f[1]).max() <= 1e-15
        assert abs(vol - 100.0) <= 1e-11
        Q1, *_ = shear_state(g, A, B, amp_rho=0.0)
        _, (ke1, ens1, _) = oracle.diagnostics(g, m, Q1, scheme=scheme)
        assert abs(ke1 - (A * A + B * B) / 4) <= 1e-14
        assert abs(ens1 - k * k * (A * A + B * B) / 4) <= 1e-4 * ens1  # derivative error only
    order = math.log(errs[0] / errs[1], 2)
    assert order >= (5.5 if scheme == "meg6" else 3.9), (errs, order)


def test_uniform_state_on_affine_grid_is_exact():
    """Constant state on a skewed affine grid: zero vorticity and Q,
    E_k = rho |u|^2 / 2, volume = det(A) * cells."""
    n = (6, 5, 4)
    A = np.array([[1.0, 0.2, 0.1], [0.05, 0.8, 0.3], [0.0, 0.15, 1.2]])
    k, j, i = np.meshgrid(np.arange(n[2]) + 0.5, np.arange(n[1]) + 0.5, np.arange(n[0]) + 0.5, indexing="ij")
    xyz = np.stack([A[c, 0] * i + A[c, 1] * j + A[c, 2] * k for c in range(3)])
    off = [[A[c, d] * n[d] for c in range(3)] for d in range(3)]
    g = {"n": n, "ndim": 3, "xyz": xyz, "off": off, "xyz_t": None}
    m = oracle.metrics(g)
    Q = W.uniform_flow(g, 1.3, 0.4, -0.2, 0.1, 2.0)
    f, (ke, ens, vol) = oracle.diagnostics(g, m, Q)
    assert np.abs(f).max() <= 1e-13
    assert abs(ke - 0.5 * 1.3 * (0.16 + 0.04 + 0.01)) <= 1e-14
    assert abs(ens) <= 1e-25
    assert abs(vol - np.linalg.det(A) * 120) <= 1e-12


def test_curvilinear_grid_converges_to_closed_form():
    """The same shear flow on the wavy grid: vorticity converges."""
    A, B = 0.3, 0.2
    errs = []
    for n in (32, 64):
        g = W.wavy2d((n, n), L=10.0, amp=0.05)
        m = oracle.metrics(g)
        Q, k, x, y = shear_state(g, A, B)
        f, _ = oracle.diagnostics(g, m, Q)
        errs.append(np.abs(f[2] - (B * k * np.cos(k * x) - A * k * np.cos(k * y))).max())
    assert math.log(errs[0] / errs[1], 2) >= 3.5, errs

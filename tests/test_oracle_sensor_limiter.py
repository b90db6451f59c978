"""Pins of the oracle's shock sensor, of the curvature terms of the MP
limiter (App. E) and of the translation invariance of the metrics (Sec. 4.2).

Each test names the plausible mistake it is built to catch; the mutation was
applied to a copy of the oracle and the test failed under it.
"""
import numpy as np
import pytest

import oracle
import workloads as W


# ---------------------------------------------------------------------------
# Ducros sensor on an affine skewed grid with a linear velocity field
# ---------------------------------------------------------------------------
SKEW = np.array([[0.30, 0.07, -0.04],
                 [0.05, 0.26, 0.06],
                 [-0.03, 0.04, 0.22]])


def _affine_grid(n, M):
    """Cell centres x = M (i + 1/2, j + 1/2, k + 1/2), periodic with shifts n_d M[:, d]."""
    k, j, i = np.meshgrid(np.arange(n[2]) + 0.5, np.arange(n[1]) + 0.5,
                          np.arange(n[0]) + 0.5, indexing="ij")
    xyz = np.stack([M[c, 0] * i + M[c, 1] * j + M[c, 2] * k for c in range(3)])
    off = [[M[c, d] * n[d] for c in range(3)] for d in range(3)]
    return {"n": tuple(n), "ndim": 3, "xyz": np.ascontiguousarray(xyz), "off": off, "xyz_t": None}


def _linear_velocity_state(g, A):
    """rho = 1, p = 1, velocity u = A x (not periodic: only cells whose
    seven-point E6 windows stay inside the box see the linear field)."""
    x = g["xyz"].reshape(3, -1)
    u = (A @ x).reshape(g["xyz"].shape)
    one = np.ones(g["xyz"].shape[1:])
    return W.conserved(one, u[0], u[1], u[2], one)


def _inner(a, margin=3):
    return a[margin:-margin, margin:-margin, margin:-margin]


def _theta_exact(A):
    div = np.trace(A)
    w = np.array([A[2, 1] - A[1, 2], A[0, 2] - A[2, 0], A[1, 0] - A[0, 1]])
    return div * div / (div * div + w @ w + 1e-30)


@pytest.mark.parametrize("case", ["dilatation", "rotation", "general", "shear"])
def test_sensor_exact_for_linear_fields_on_skewed_grid(case):
    """For u = A x on an affine grid the E6 cell gradients and the
    conservative cell metrics are exact, so du_a/dx_b = A[a][b] and the
    sensor is theta = tr(A)^2 / (tr(A)^2 + |curl|^2 + 1e-30) at every cell
    whose stencil stays inside the box:
    - pure dilatation A = s I: theta = 1;
    - solid-body rotation (antisymmetric A): theta = 0;
    - a general A and a pure shear: the closed form.
    Catches: the chain rule with the metric index transposed
    (d_{x_b} replaced by b_{x_d}, wrong on a skewed grid), a vorticity
    component built from the wrong pair of derivatives, the divergence taken
    from the index-space gradients instead of the physical ones. (The sign of
    a single vorticity component does not enter theta.)"""
    A = {"dilatation": 0.7 * np.eye(3),
         "rotation": np.array([[0.0, -0.4, 0.3], [0.4, 0.0, -0.2], [-0.3, 0.2, 0.0]]),
         "general": np.array([[0.5, -0.3, 0.2], [0.1, -0.2, 0.4], [-0.6, 0.25, 0.35]]),
         "shear": np.array([[0.0, 0.8, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])}[case]
    g = _affine_grid((14, 13, 12), SKEW)
    m = oracle.metrics(g)
    Q = _linear_velocity_state(g, A)
    th = _inner(oracle.sensor(g, m, Q))
    expect = _theta_exact(A)
    assert np.abs(th - expect).max() <= 1e-12, (case, expect, th.min(), th.max())


def test_sensor_distinguishes_the_chain_rule_orientation():
    """The skewed grid makes the two orientations of the chain rule differ on
    the general field by far more than the tolerance above, so the pin is
    sensitive to the metric index order (a check of the test itself)."""
    A = np.array([[0.5, -0.3, 0.2], [0.1, -0.2, 0.4], [-0.6, 0.25, 0.35]])
    Minv = np.linalg.inv(SKEW)
    G_index = A @ SKEW                       # du_a / dxi_d
    G_wrong = G_index @ Minv.T               # sum_d Minv[b][d] du_a/dxi_d
    assert abs(_theta_exact(G_wrong) - _theta_exact(A)) > 1e-3


# ---------------------------------------------------------------------------
# MP limiter: App. E with non-zero curvatures, hand-evaluated
# ---------------------------------------------------------------------------
def test_mp_limiter_median_bound_is_wmd():
    """Local maximum W = (0, 2, 1) at i-1, i, i+1 with curvatures
    d = (-1, -4, -2) and an overshooting W^L = 3 (alpha = beta = 4):
      W^MP = 2 + minmod(-1, 8) = 2, and (3 - 2)(3 - 2) > 1e-20, so limit;
      d^M(i+1/2) = minmod(-4, -2) = -2,  d^M(i-1/2) = minmod(-1, -4) = -1;
      W^MD = (2 + 1)/2 - (-2)/2 = 2.5;  W^UL = 2 + 4 * 2 = 10;
      W^LC = (3 * 2 - 0)/2 + (4/3)(-1) = 5/3;
      W^min = max(min(2, 1, 2.5), min(2, 10, 5/3)) = 5/3;
      W^max = min(max(2, 1, 2.5), max(2, 10, 5/3)) = 2.5;
      limited = median(3, 5/3, 2.5) = 2.5 = W^MD.
    Catches: the sign of the curvature term in W^MD (+ gives 2), d^M at
    i+1/2 and i-1/2 swapped (gives 2)."""
    out = oracle.mp_limit(0.0, 2.0, 1.0, -1.0, -4.0, -2.0, 3.0)
    assert out == pytest.approx(2.5, abs=1e-15)
    # odd under negation of all data (the limiter is sign-symmetric)
    out = oracle.mp_limit(0.0, -2.0, -1.0, 1.0, 4.0, 2.0, -3.0)
    assert out == pytest.approx(-2.5, abs=1e-15)


def test_mp_limiter_median_bound_is_wlc():
    """Flat-then-rising data W = (1, 1, 4) with curvatures d = (0.75, 1.5, 3)
    and W^L = 3:
      W^MP = 1 + minmod(3, 0) = 1, and (3 - 1)(3 - 1) > 1e-20, so limit;
      d^M(i+1/2) = minmod(1.5, 3) = 1.5,  d^M(i-1/2) = minmod(0.75, 1.5) = 0.75;
      W^MD = 2.5 - 0.75 = 1.75;  W^UL = 1 + 4 * 0 = 1;
      W^LC = (3 - 1)/2 + (4/3)(0.75) = 2;
      W^min = max(min(1, 4, 1.75), min(1, 1, 2)) = 1;
      W^max = min(max(1, 4, 1.75), max(1, 1, 2)) = 2;
      limited = median(3, 1, 2) = 2 = W^LC.
    Catches: the 4/3 factor of W^LC mis-written (1/3 gives 1.25, 2/3 gives
    1.5), d^M at i+1/2 used in W^LC (gives 3), the 1/2 (3 W_i - W_{i-1})
    part mis-written as W_i + 1/2 (W_i + W_{i-1}) (gives 3)."""
    out = oracle.mp_limit(1.0, 1.0, 4.0, 0.75, 1.5, 3.0, 3.0)
    assert out == pytest.approx(2.0, abs=1e-15)


def test_mp_limiter_lower_bound_from_wlc():
    """Mirror image (negated data) of the previous case: the lower bound
    W^min = W^LC = -2 is the active one."""
    out = oracle.mp_limit(-1.0, -1.0, -4.0, -0.75, -1.5, -3.0, -3.0)
    assert out == pytest.approx(-2.0, abs=1e-15)


def test_mp_limiter_curvature_signs_disagree():
    """Curvatures of opposite sign give d^M = 0 at that interface:
    W = (0, 1, 3), d = (2, -1, 5), W^L = 4:
      W^MP = 1 + minmod(2, 4) = 3, and (4 - 1)(4 - 3) > 1e-20, so limit;
      d^M(i+1/2) = minmod(-1, 5) = 0, d^M(i-1/2) = minmod(2, -1) = 0;
      W^MD = 2;  W^UL = 5;  W^LC = 1.5;
      W^min = max(min(1, 3, 2), min(1, 5, 1.5)) = 1;
      W^max = min(max(1, 3, 2), max(1, 5, 1.5)) = 3;
      limited = median(4, 1, 3) = 3.
    A minmod that ignores the sign rule gives d^M = -1 at both interfaces
    here (W^MD = 2.5, W^LC = 1/6) and still 3; the next case separates it."""
    assert oracle.mp_limit(0.0, 1.0, 3.0, 2.0, -1.0, 5.0, 4.0) == pytest.approx(3.0, abs=1e-15)


def test_mp_limiter_minmod_sign_rule_in_wmd():
    """W = (0, 2, 1), d = (-1, 3, -2), W^L = 3:
      W^MP = 2, limit; d^M(i+1/2) = minmod(3, -2) = 0 -> W^MD = 1.5;
      d^M(i-1/2) = minmod(-1, 3) = 0 -> W^LC = 3; W^UL = 10;
      W^min = max(min(2, 1, 1.5), min(2, 10, 3)) = 2;
      W^max = min(max(2, 1, 1.5), max(2, 10, 3)) = 2;
      limited = 2.
    Catches a minmod that ignores the sign rule (d^M(i+1/2) = -2 would
    give W^MD = 2.5 and W^max = 2.5, limited 2.5)."""
    assert oracle.mp_limit(0.0, 2.0, 1.0, -1.0, 3.0, -2.0, 3.0) == pytest.approx(2.0, abs=1e-15)


# ---------------------------------------------------------------------------
# Metrics: translation invariance (Sec. 4.2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("scheme", ["meg6", "mig4"])
@pytest.mark.parametrize("maker", [
    lambda: W.random3d((14, 12, 10), amp=0.2, seed=4),
    lambda: W.jet3d((24, 16, 14)),
    lambda: W.Deforming3D((12, 12, 12), rand=0.2, seed=2).at(0.13),
])
def test_metrics_invariant_under_translation(maker, scheme):
    """Every metric slot depends on coordinate differences only, so moving the
    whole grid by (1e3, -2e3, 5e2) leaves all 66 slots unchanged up to the
    rounding of the translated coordinates: a relative change per slot family
    within 4 eps max|x| / h (h the smallest cell spacing; observed 0.2-1.0
    of eps max|x| / h).
    Catches: a cell origin subtracted in one of the two products of
    Eq. GCL_metrics but not in the other (the translation then no longer
    cancels between them). Raw coordinates in both products stay within the
    bound for MEG6: the cancellation they leave is of the same order as the
    rounding of the translated coordinates. For MIG4, whose derivatives come
    from whole-line IG4 systems, raw coordinates leave errors of O(eps
    max|x| / h) times the growth of the wide stencils, about 100 eps max|x|
    / h here, which this bound rejects."""
    g = maker()
    m0 = oracle.metrics(g, scheme=scheme)
    g2 = dict(g)
    shift = np.array([1e3, -2e3, 5e2]).reshape(3, 1, 1, 1)
    g2["xyz"] = np.ascontiguousarray(g["xyz"] + shift)
    m1 = oracle.metrics(g2, scheme=scheme)
    h = min(np.abs(np.diff(g["xyz"][c], axis=2 - c)).min() for c in range(3))
    tol = 4.0 * np.finfo(float).eps * np.abs(g2["xyz"]).max() / h
    families = [range(0, 9), range(9, 18), [18], [19], range(20, 23), range(23, 26), [26]]
    families += [range(27 + f * 13, 27 + (f + 1) * 13) for f in range(3)]
    for fam in families:
        fam = list(fam)
        scale = np.abs(m0[fam]).max()
        if scale == 0.0:
            assert np.abs(m1[fam]).max() == 0.0
            continue
        assert np.abs(m1[fam] - m0[fam]).max() <= tol * scale, (fam, tol)

"""Pins of the oracle's 1-D stencils and metric discretisation against what the
paper prints (Sec. 7) and against polynomial exactness."""
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows, den = [], None
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("denominator"):
                den = int(line.split()[1])
                continue
            rows.append([int(t) for t in line.split()])
    return den, rows


def test_composite_derivative_matches_printed_stencil():
    """D = Delta o I applied to a unit impulse gives the printed weights
    (2282, -546, 89, -3, -1)/2880 of Sec. 7 (this pins the E6 difference form,
    the Hermite second derivative and the 1/12 van Leer coefficient)."""
    den, rows = _read_golden("composite_derivative.txt")
    n = 16
    v = np.zeros(n)
    v[0] = 1.0
    d = oracle.line_dcomp(v)
    # d[i] = sum_m c_m (v[i+m] - v[i-m]) -> at i = -m the impulse enters with +c_m
    for m, cm in rows:
        assert d[(-m) % n] * den == pytest.approx(cm, abs=1e-9)
        assert d[m % n] * den == pytest.approx(-cm, abs=1e-9)
    assert d[0] == 0.0
    assert np.count_nonzero(np.abs(d) > 1e-15) == 10


def _poly_line(deg, n=64, h=1.0):
    x = (np.arange(n) - n / 2) * h
    return x, x ** deg


@pytest.mark.parametrize("deg", range(0, 7))
def test_e6_exact_to_degree_six(deg):
    x, f = _poly_line(deg)
    out = oracle.line_e6(f)
    exact = deg * x ** (deg - 1) if deg else 0 * x
    sl = slice(8, -8)
    assert np.allclose(out[sl], exact[sl], rtol=1e-10, atol=1e-8)


def test_e6_not_exact_at_degree_seven():
    x, f = _poly_line(7)
    out = oracle.line_e6(f)
    assert np.max(np.abs(out[8:-8] - 7 * x[8:-8] ** 6)) > 1.0


@pytest.mark.parametrize("deg", range(0, 6))
def test_hermite_second_derivative_exact_to_degree_five(deg):
    x, f = _poly_line(deg)
    out = oracle.line_hermite(f)
    exact = deg * (deg - 1) * x ** (deg - 2) if deg >= 2 else 0 * x
    sl = slice(8, -8)
    assert np.allclose(out[sl], exact[sl], rtol=1e-9, atol=1e-7)


@pytest.mark.parametrize("deg", range(0, 5))
def test_composite_derivative_exact_to_degree_four(deg):
    """Fourth-order claim of Sec. 5.1 Step-7 for the linear metric derivative."""
    x, f = _poly_line(deg)
    out = oracle.line_dcomp(f)
    exact = deg * x ** (deg - 1) if deg else 0 * x
    sl = slice(8, -8)
    assert np.allclose(out[sl], exact[sl], rtol=1e-9, atol=1e-7)


def test_periodic_shift_gives_exact_linear_derivative():
    """A periodic line with a coordinate shift (x[i+n] = x[i] + L) is
    differentiated as its periodic extension: D of i*h is h everywhere."""
    n, h = 12, 0.3
    v = np.arange(n) * h
    assert np.allclose(oracle.line_dcomp(v, shift=n * h), h, atol=1e-15)
    assert np.allclose(oracle.line_e6(v, shift=n * h), h, atol=1e-15)
    assert np.allclose(oracle.line_face(v, shift=n * h), (np.arange(n) + 0.5) * h, atol=1e-14)


def test_face_interpolation_is_symmetric_and_consistent():
    """Central interface value: weights sum to one and are mirror symmetric."""
    n = 16
    w = np.zeros(n)
    for q in range(n):
        v = np.zeros(n)
        v[q] = 1.0
        w[q] = oracle.line_face(v)[0]
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    # face 0 sits between cells 0 and 1: weight of cell q equals that of 1-q
    for q in range(-4, 6):
        assert w[q % n] == pytest.approx(w[(1 - q) % n], abs=1e-16)


def _identity_term(y_off, z_off, amp=1.0):
    """Mixed second difference in (delta_y, delta_z) of Delta_xi(I_xi hat(xi)_x)
    at the centre cell (8, 8, 8) of a 16^3 uniform unit grid whose y and z
    coordinates carry impulses of size delta at the given offsets. The
    quantity is bilinear in (y, z), so the mixed difference is its exact
    coefficient for the pair of impulses."""
    n = 16
    c = np.array([8, 8, 8])

    def f(dy, dz):
        g = W.uniform3d((n, n, n), (n, n, n))
        xyz = g["xyz"].copy()
        ya = c + np.array(y_off)
        za = c + np.array(z_off)
        xyz[1, ya[2], ya[1], ya[0]] += dy
        xyz[2, za[2], za[1], za[0]] += dz
        g["xyz"] = xyz
        m = oracle.metrics(g)
        face = m[oracle.M_FHAT(0, 0)]
        return face[c[2], c[1], c[0]] - face[c[2], c[1], c[0] - 1]

    return (f(amp, amp) - f(amp, -amp) - f(-amp, amp) + f(-amp, -amp)) / (4 * amp * amp)


def test_metric_identity_expansion_coefficients():
    """The printed coefficients of the expansion of d/dxi(hat xi_x) (Sec. 7):
    -1, -3, +3, +1 over 23887872000 for the listed (y, z) index pairs."""
    den, rows = _read_golden("metric_identity_coefficients.txt")
    assert den == 2880 ** 3
    for num, ydi, ydj, ydk, zdi, zdj, zdk in rows:
        coef = _identity_term((ydi, ydj, ydk), (zdi, zdj, zdk), amp=0.25)
        assert coef * den == pytest.approx(num, abs=2e-3), (num, coef * den)

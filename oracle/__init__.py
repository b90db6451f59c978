"""Python access to the FP64 CPU oracle (``gbr_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg. The HIP product package never imports this
module, and this module imports nothing from the product package.

Arrays are numpy float64 in the [var][nk][nj][ni] layout of ``workloads``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import _build

LIM = {"none": 0, "mp": 1, "ducros": 2}
DT_CFL, DT_FIXED = 0, 1

# metric-slot helpers (mirror the macros of gbr_oracle.h)
M_TOTAL = 66


def M_HAT(d, c):
    return d * 3 + c


def M_UNHAT(d, c):
    return 9 + d * 3 + c


M_INVJ, M_J, M_INVJT = 18, 19, 26


def M_HATT(d):
    return 20 + d


def M_UNHATT(d):
    return 23 + d


def M_FHAT(f, c):
    return 27 + f * 13 + c


def M_FHATT(f):
    return 27 + f * 13 + 3


def M_FUNHAT(f, e, c):
    return 27 + f * 13 + 4 + e * 3 + c


class _Cfg(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3),
        ("ndim", C.c_int),
        ("viscous", C.c_int),
        ("limiter", C.c_int),
        ("moving", C.c_int),
        ("scheme", C.c_int),
        ("off", C.c_double * 9),
        ("gamma", C.c_double),
        ("Pr", C.c_double),
        ("Re", C.c_double),
        ("Mref", C.c_double),
        ("suth", C.c_double),
        ("theta_c", C.c_double),
        ("alpha_mp", C.c_double),
        ("beta_mp", C.c_double),
        ("alpha_d", C.c_double),
        ("bc", C.c_int * 6),
        ("sigma", C.POINTER(C.c_double)),
        ("qref", C.c_double * 5),
    ]


DEFAULTS = dict(gamma=1.4, Pr=0.71, Re=1e4, Mref=1.0, suth=110.4 / 293.0,
                viscous=False, limiter="mp", theta_c=0.5, alpha_mp=4.0, beta_mp=4.0,
                alpha_d=4.0, scheme="meg6")
SCHEMES = {"meg6": 0, "mig4": 1}
BC = {"periodic": 0, "inflow": 1, "outflow": 2, "wall": 3}
NG = 6  # ghost layers on each non-periodic side (REF_NG)

_lib = None
_P = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        path = _build.library_path()
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        cfgp = C.POINTER(_Cfg)
        L.ref_metrics.argtypes = [cfgp, _P, _P, _P]
        L.ref_metrics.restype = C.c_int
        L.ref_metrics_nonfp.argtypes = [cfgp, _P, _P]
        L.ref_metrics_nonfp.restype = C.c_int
        L.ref_gradients.argtypes = [cfgp, _P, _P]
        L.ref_sensor.argtypes = [cfgp, _P, _P, _P]
        L.ref_rhs.argtypes = [cfgp, _P, _P, _P]
        L.ref_rhs.restype = C.c_int
        L.ref_cfl_min.argtypes = [cfgp, _P, _P]
        L.ref_cfl_min.restype = C.c_double
        L.ref_rk_stage.argtypes = [cfgp, _P, C.c_int, C.c_double, _P, _P, _P]
        L.ref_step.argtypes = [cfgp, _P, _P, _P, _P, C.c_double, C.c_int, _P]
        L.ref_step.restype = C.c_int
        for nm in ("ref_line_e6", "ref_line_hermite", "ref_line_face", "ref_line_dcomp"):
            getattr(L, nm).argtypes = [_P, C.c_int, C.c_double, _P]
        for nm in ("ref_line_ig4", "ref_line_ig4_face", "ref_line_ig4_dcomp"):
            getattr(L, nm).argtypes = [_P, C.c_int, C.c_double, _P]
            getattr(L, nm).restype = C.c_int
        L.ref_eigvec.argtypes = [_P, C.c_double, C.c_double, _P, _P]
        L.ref_diagnostics.argtypes = [cfgp, _P, _P, _P, _P]
        L.ref_diagnostics.restype = C.c_int
        L.ref_mp_limit.argtypes = [C.c_double] * 9
        L.ref_mp_limit.restype = C.c_double
        L.ref_bline_derivs.argtypes = [_P, C.c_int, _P, _P]
        L.ref_bline_derivs.restype = C.c_int
        L.ref_bline_faces.argtypes = [_P, C.c_int, _P]
        L.ref_bline_faces.restype = C.c_int
        L.ref_apply_bc.argtypes = [cfgp, _P, _P]
        L.ref_hllc.argtypes = [_P, _P, _P, C.c_double, _P]
        L.ref_euler_flux.argtypes = [_P, _P, C.c_double, _P]
        _lib = L
    return _lib


def set_num_threads(n):
    """Number of OpenMP threads the oracle's parallel loops use from now on
    (the library's OpenMP runtime, loaded with it). Returns the previous
    maximum."""
    lib()
    omp = C.CDLL("libgomp.so.1")
    omp.omp_get_max_threads.restype = C.c_int
    prev = int(omp.omp_get_max_threads())
    omp.omp_set_num_threads(C.c_int(int(n)))
    return prev


def _ptr(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_P)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_cfg(grid, **params):
    p = dict(DEFAULTS)
    p.update(params)
    c = _Cfg()
    for d in range(3):
        c.n[d] = int(grid["n"][d])
    c.ndim = int(grid["ndim"])
    c.viscous = int(bool(p["viscous"]))
    c.limiter = LIM[p["limiter"]] if isinstance(p["limiter"], str) else int(p["limiter"])
    c.moving = int(grid.get("xyz_t") is not None)
    c.scheme = SCHEMES[p["scheme"]] if isinstance(p["scheme"], str) else int(p["scheme"])
    off = np.asarray(grid["off"], dtype=np.float64).reshape(9)
    for q in range(9):
        c.off[q] = float(off[q])
    for k in ("gamma", "Pr", "Re", "Mref", "suth", "theta_c", "alpha_mp", "beta_mp", "alpha_d"):
        setattr(c, k, float(p[k]))
    bc = grid.get("bc")
    for d in range(3):
        for side in range(2):
            t = bc[d][side] if bc is not None and d < len(bc) else "periodic"
            c.bc[d * 2 + side] = BC[t] if isinstance(t, str) else int(t)
    sigma = p.get("sigma")
    if sigma is not None:
        keep = _f64(sigma).reshape(-1)
        assert keep.size == _ncell(grid)
        c.sigma = keep.ctypes.data_as(_P)
        c._keep = keep  # the array must outlive the call
        for q, v in enumerate(p.get("qref", (1.0, 0.0, 0.0, 0.0, 1.0 / 1.4))):
            c.qref[q] = float(v)
    return c


def _ncell(grid):
    n = grid["n"]
    return n[0] * n[1] * n[2]


def _shape(grid):
    n = grid["n"]
    return (n[2], n[1], n[0])


def metrics(grid, nonfp=False, **params):
    """All metric slots as an array [66][nk][nj][ni]; raises on 1/J <= 0."""
    cfg = make_cfg(grid, **params)
    xyz = _f64(grid["xyz"])
    m = np.zeros((M_TOTAL,) + _shape(grid))
    if nonfp:
        rc = lib().ref_metrics_nonfp(C.byref(cfg), _ptr(xyz), _ptr(m))
    else:
        xt = grid.get("xyz_t")
        keep = _f64(xt) if xt is not None else None
        rc = lib().ref_metrics(C.byref(cfg), _ptr(xyz), _ptr(keep) if keep is not None else None,
                               _ptr(m))
    if rc == -2:
        raise NotImplementedError("oracle metrics: unsupported combination (rc=-2)")
    if rc != 0:
        raise ValueError("oracle metrics: non-positive Jacobian (rc=%d)" % rc)
    return m


def gradients(grid, Q, **params):
    cfg = make_cfg(grid, **params)
    Q = _f64(Q)
    g = np.zeros((12,) + _shape(grid))
    lib().ref_gradients(C.byref(cfg), _ptr(Q), _ptr(g))
    return g


def sensor(grid, m, Q, **params):
    cfg = make_cfg(grid, **params)
    g = gradients(grid, Q, **params)
    th = np.zeros(_shape(grid))
    lib().ref_sensor(C.byref(cfg), _ptr(_f64(m)), _ptr(g), _ptr(th))
    return th


def rhs(grid, m, Q, **params):
    cfg = make_cfg(grid, **params)
    Q = _f64(Q)
    res = np.zeros_like(Q)
    rc = lib().ref_rhs(C.byref(cfg), _ptr(_f64(m)), _ptr(Q), _ptr(res))
    if rc != 0:
        raise FloatingPointError("oracle rhs: non-physical state (rc=%d)" % rc)
    return res


def cfl_min(grid, m, Q, **params):
    cfg = make_cfg(grid, **params)
    return lib().ref_cfl_min(C.byref(cfg), _ptr(_f64(m)), _ptr(_f64(Q)))


def rk_stage(grid, m, stage, dt, Qn, Q, res, **params):
    """Returns the updated Q (the input is not modified)."""
    cfg = make_cfg(grid, **params)
    out = _f64(Q).copy()
    lib().ref_rk_stage(C.byref(cfg), _ptr(_f64(m)), int(stage), float(dt), _ptr(_f64(Qn)),
                       _ptr(out), _ptr(_f64(res)))
    return out


def step(grid, m, Q, cfl_or_dt, dt_mode=DT_CFL, **params):
    """One SSP-RK3 step. For moving grids ``grid`` holds xyz, xyz_t at t^n and
    ``m`` is overwritten with the metrics at t^n. Returns (Q_new, dt)."""
    cfg = make_cfg(grid, **params)
    Qw = _f64(Q).copy()
    dt = C.c_double(0.0)
    xyz = _f64(grid["xyz"])
    xt = grid.get("xyz_t")
    xt = _f64(xt) if xt is not None else None
    rc = lib().ref_step(C.byref(cfg), _ptr(m), _ptr(xyz), _ptr(xt) if xt is not None else None,
                        _ptr(Qw), float(cfl_or_dt), int(dt_mode), C.byref(dt))
    if rc != 0:
        raise FloatingPointError("oracle step failed (rc=%d)" % rc)
    return Qw, dt.value


# --- pointwise / line pieces ------------------------------------------------
def _line(fn, v, shift):
    v = _f64(v)
    out = np.zeros_like(v)
    getattr(lib(), fn)(_ptr(v), len(v), float(shift), _ptr(out))
    return out


def line_e6(v, shift=0.0):
    return _line("ref_line_e6", v, shift)


def line_hermite(v, shift=0.0):
    return _line("ref_line_hermite", v, shift)


def line_face(v, shift=0.0):
    return _line("ref_line_face", v, shift)


def line_dcomp(v, shift=0.0):
    return _line("ref_line_dcomp", v, shift)


def _line_checked(fn, v, shift):
    v = _f64(v)
    out = np.zeros_like(v)
    if getattr(lib(), fn)(_ptr(v), len(v), float(shift), _ptr(out)) != 0:
        raise FloatingPointError(f"{fn}: singular line system")
    return out


def line_ig4(v, shift=0.0):
    """IG4 derivative (MIG4, Eq. IG4_grads) of a periodic line, v[i+n] = v[i] + shift."""
    return _line_checked("ref_line_ig4", v, shift)


def line_ig4_face(v, shift=0.0):
    """Interface values at i + 1/2 built on IG4 gradients (Eq. FP-interp)."""
    return _line_checked("ref_line_ig4_face", v, shift)


def line_ig4_dcomp(v, shift=0.0):
    """Difference of the IG4 interface values (Eq. FP-interp2)."""
    return _line_checked("ref_line_ig4_dcomp", v, shift)


def bline_derivs(v):
    """App. C first and second derivatives on a non-periodic line (m >= 12)."""
    v = _f64(v)
    p, h = np.zeros_like(v), np.zeros_like(v)
    if lib().ref_bline_derivs(_ptr(v), len(v), _ptr(p), _ptr(h)) != 0:
        raise ValueError("line too short")
    return p, h


def bline_faces(v):
    """App. C interface values F[0..m] of a non-periodic line (m >= 12)."""
    v = _f64(v)
    F = np.zeros(len(v) + 1)
    if lib().ref_bline_faces(_ptr(v), len(v), _ptr(F)) != 0:
        raise ValueError("line too short")
    return F


def apply_bc(grid, m, Q, **params):
    """Q with its ghost cells set from the grid's boundary types (a copy)."""
    cfg = make_cfg(grid, **params)
    out = _f64(Q).copy()
    lib().ref_apply_bc(C.byref(cfg), _ptr(_f64(m)), _ptr(out))
    return out


def interior(grid):
    """Index tuple (slices over [nk][nj][ni]) of the interior cells."""
    bc = grid.get("bc")
    sl = []
    for d in (2, 1, 0):
        bounded = bc is not None and d < len(bc) and bc[d][0] != "periodic"
        sl.append(slice(NG, grid["n"][d] - NG) if bounded else slice(None))
    return tuple(sl)


def eigvec(nrm, rho, a):
    R = np.zeros(25)
    Ri = np.zeros(25)
    lib().ref_eigvec(_ptr(_f64(nrm)), float(rho), float(a), _ptr(R), _ptr(Ri))
    return R.reshape(5, 5), Ri.reshape(5, 5)


def mp_limit(wm1, w0, wp1, dm1, d0, dp1, wface, alpha=4.0, beta=4.0):
    return lib().ref_mp_limit(wm1, w0, wp1, dm1, d0, dp1, wface, alpha, beta)


def hllc(PL, PR, nt_n, gamma=1.4):
    F = np.zeros(5)
    lib().ref_hllc(_ptr(_f64(PL)), _ptr(_f64(PR)), _ptr(_f64(nt_n)), float(gamma), _ptr(F))
    return F


def euler_flux(P, nt_n, gamma=1.4):
    F = np.zeros(5)
    lib().ref_euler_flux(_ptr(_f64(P)), _ptr(_f64(nt_n)), float(gamma), _ptr(F))
    return F


def diagnostics(grid, m, Q, **params):
    """(fields[5] = vorticity x, y, z, Q-criterion, |grad rho|; (KE, enstrophy, volume))."""
    cfg = make_cfg(grid, **params)
    Q = _f64(Q)
    f = np.zeros((5,) + _shape(grid))
    it = np.zeros(3)
    if lib().ref_diagnostics(C.byref(cfg), _ptr(_f64(m)), _ptr(Q), _ptr(f), _ptr(it)) != 0:
        raise MemoryError("oracle diagnostics")
    return f, tuple(it)


def prim_from_Q(Q, gamma=1.4):
    """(rho, u, v, w, p) from conserved Q (w = 0 for 2-D)."""
    rho = Q[0]
    u = Q[1] / rho
    v = Q[2] / rho
    if Q.shape[0] == 5:
        w = Q[3] / rho
    else:
        w = np.zeros_like(u)
    p = (gamma - 1.0) * (Q[-1] - 0.5 * rho * (u * u + v * v + w * w))
    return rho, u, v, w, p

"""Thin ctypes binding of libgbr (include/gbr.h).

Functions keep the C names and only marshal arguments: torch tensors are
passed as device pointers, the stream is the current torch stream. Every step
of the computation runs in the library's HIP kernels; there is no fallback.
If the library is missing, loading raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(os.path.dirname(HERE), "include", "gbr.h")

GBR_OK, GBR_E_ARG, GBR_E_JACOBIAN, GBR_E_STATE, GBR_E_NOMEM, GBR_E_DEVICE, GBR_E_UNSUPPORTED = range(7)
STATUS_NAMES = {0: "GBR_OK", 1: "GBR_E_ARG", 2: "GBR_E_JACOBIAN", 3: "GBR_E_STATE",
                4: "GBR_E_NOMEM", 5: "GBR_E_DEVICE", 6: "GBR_E_UNSUPPORTED"}
LIM = {"none": 0, "mp": 1, "ducros": 2}
GBR_FP64, GBR_FP32_BULK = 0, 1
PRECISION = {"fp64": GBR_FP64, "fp32_bulk": GBR_FP32_BULK}
GBR_SCHEME_MEG6, GBR_SCHEME_MIG4 = 0, 1
SCHEME = {"meg6": GBR_SCHEME_MEG6, "mig4": GBR_SCHEME_MIG4}
GBR_DT_CFL, GBR_DT_FIXED = 0, 1
GBR_BC_PERIODIC, GBR_BC_INFLOW, GBR_BC_OUTFLOW, GBR_BC_WALL = 0, 1, 2, 3
BC = {"periodic": GBR_BC_PERIODIC, "inflow": GBR_BC_INFLOW, "outflow": GBR_BC_OUTFLOW, "wall": GBR_BC_WALL}
GBR_NG = 6
GBR_TILE_AUTO, GBR_TILE_16X16, GBR_TILE_32X8, GBR_TILE_8X32 = -1, 0, 1, 2
TILE_NAMES = {0: "16x16", 1: "32x8", 2: "8x32"}


def SLOT_FACE_HAT(f, c):
    return f * 13 + c


def SLOT_FACE_HATT(f):
    return f * 13 + 3


def SLOT_FACE_UNHAT(f, e, c):
    return f * 13 + 4 + e * 3 + c


def SLOT_CELL_UNHAT(e, c):
    return 39 + e * 3 + c


SLOT_CELL_J, SLOT_CELL_INVJ, SLOT_CELL_INVJT = 48, 49, 50


def SLOT_CELL_UNHATT(e):
    return 51 + e


def SLOT_CELL_HAT(e, c):
    return 54 + e * 3 + c


def SLOT_CELL_HATT(e):
    return 63 + e


SLOT_COUNT = 66


class GbrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class gbr_config(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32),
        ("n", C.c_int32 * 3),
        ("viscous", C.c_int32),
        ("limiter", C.c_int32),
        ("moving", C.c_int32),
        ("precision", C.c_int32),
        ("scheme", C.c_int32),
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
        ("bc", C.c_int32 * 6),
    ]


_lib = None
_VP = C.c_void_p
_PP = C.POINTER(C.c_void_p)


def library_path():
    return os.path.join(HERE, "libgbr.so")


def lib():
    """Load libgbr.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    L = C.CDLL(path)
    L.gbr_grid_create.argtypes = [C.POINTER(gbr_config), _VP, C.POINTER(_VP)]
    L.gbr_grid_destroy.argtypes = [_VP]
    L.gbr_grid_bytes.argtypes = [C.POINTER(gbr_config)]
    L.gbr_grid_bytes.restype = C.c_size_t
    L.gbr_set_stream.argtypes = [_VP, _VP]
    L.gbr_metrics.argtypes = [_PP, C.c_int, _PP, _PP]
    L.gbr_rhs.argtypes = [_PP, C.c_int, _PP, _PP]
    L.gbr_rk_stage.argtypes = [_PP, C.c_int, C.c_int, _PP, _PP, _PP, _PP]
    L.gbr_cfl.argtypes = [_PP, C.c_int, _PP, C.c_double, _PP]
    L.gbr_step.argtypes = [_PP, C.c_int, _PP, _PP, _PP, C.c_double, C.c_int, _PP, _PP]
    L.gbr_check_state.argtypes = [_VP]
    L.gbr_metric_ptr.argtypes = [_VP, C.c_int]
    L.gbr_metric_ptr.restype = _VP
    L.gbr_timing_enable.argtypes = [_VP, C.c_int]
    L.gbr_timing_collect.argtypes = [_VP, C.POINTER(C.c_double), C.POINTER(C.c_long)]
    L.gbr_last_error.argtypes = [_VP]
    L.gbr_last_error.restype = C.c_char_p
    L.gbr_metrics_nonfp.argtypes = [_PP, C.c_int, _PP]
    L.gbr_set_sponge.argtypes = [_VP, _VP, C.POINTER(C.c_double)]
    L.gbr_metrics_nonfp.restype = C.c_int
    L.gbr_diagnostics.argtypes = [_PP, C.c_int, _PP, _PP, _PP]
    L.gbr_diagnostics.restype = C.c_int
    L.gbr_batch_create.argtypes = [_PP, C.c_int, _PP, C.c_int, C.POINTER(_VP)]
    L.gbr_batch_run.argtypes = [_VP, C.c_int, C.c_double, C.c_int, C.c_int]
    L.gbr_batch_query.argtypes = [_VP, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.gbr_batch_destroy.argtypes = [_VP]
    L.gbr_cfl_noalloc.argtypes = [_PP, C.c_int, _PP, C.c_double, _PP]
    L.gbr_cfl_noalloc.restype = C.c_int
    L.gbr_probe_triad.argtypes = [_VP, _VP, _VP, C.c_double, C.c_long, _VP]
    L.gbr_probe_triad.restype = C.c_int
    for nm in ("gbr_grid_create", "gbr_grid_destroy", "gbr_set_stream", "gbr_metrics", "gbr_rhs",
               "gbr_rk_stage", "gbr_cfl", "gbr_step", "gbr_check_state", "gbr_timing_enable",
               "gbr_timing_collect", "gbr_batch_create", "gbr_batch_run", "gbr_batch_query",
               "gbr_batch_destroy"):
        getattr(L, nm).restype = C.c_int
    _lib = L
    return L


def header_functions():
    """Names of the functions declared in include/gbr.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gbr_[a-z_]+)\s*\(", text)))


# ---------------------------------------------------------------------------
# marshalling helpers
# ---------------------------------------------------------------------------
def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _arr(items):
    return (C.c_void_p * max(1, len(items)))(*[_ptr(x) for x in items])


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _check(status, handle=None):
    if status != GBR_OK:
        msg = lib().gbr_last_error(handle).decode() if handle is not None else ""
        raise GbrError(status, msg)


def make_config(n, ndim, off, viscous=False, limiter="mp", moving=False, gamma=1.4, Pr=0.71,
                Re=1e4, Mref=1.0, suth=110.4 / 293.0, theta_c=0.5, alpha_mp=4.0, beta_mp=4.0,
                alpha_d=4.0, precision="fp64", scheme="meg6", bc=None):
    c = gbr_config()
    c.ndim = int(ndim)
    for d in range(3):
        c.n[d] = int(n[d])
    c.viscous = int(bool(viscous))
    c.limiter = LIM[limiter] if isinstance(limiter, str) else int(limiter)
    c.moving = int(bool(moving))
    c.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    c.scheme = SCHEME[scheme] if isinstance(scheme, str) else int(scheme)
    flat = [float(v) for row in off for v in row]
    for q in range(9):
        c.off[q] = flat[q]
    c.gamma, c.Pr, c.Re, c.Mref, c.suth = gamma, Pr, Re, Mref, suth
    c.theta_c, c.alpha_mp, c.beta_mp, c.alpha_d = theta_c, alpha_mp, beta_mp, alpha_d
    for d in range(3):
        for side in range(2):
            t = bc[d][side] if bc is not None and d < len(bc) else "periodic"
            c.bc[d * 2 + side] = BC[t] if isinstance(t, str) else int(t)
    return c


# ---------------------------------------------------------------------------
# C-ABI calls under their own names
# ---------------------------------------------------------------------------
def gbr_grid_bytes(cfg):
    return int(lib().gbr_grid_bytes(C.byref(cfg)))


def gbr_grid_create(cfg, stream=None):
    h = C.c_void_p()
    st = _stream() if stream is None else stream
    _check(lib().gbr_grid_create(C.byref(cfg), C.c_void_p(st), C.byref(h)))
    return h.value


def gbr_grid_destroy(h):
    _check(lib().gbr_grid_destroy(h))


def gbr_set_stream(h, stream=None):
    st = _stream() if stream is None else stream
    _check(lib().gbr_set_stream(h, C.c_void_p(st)), h)


def gbr_metrics(handles, xyz, xyz_t=None):
    n = len(handles)
    xt = _arr(xyz_t) if xyz_t is not None else None
    _check(lib().gbr_metrics(_arr(handles), n, _arr(xyz), xt), handles[0] if n else None)


def gbr_metrics_nonfp(handles, xyz):
    n = len(handles)
    _check(lib().gbr_metrics_nonfp(_arr(handles), n, _arr(xyz)), handles[0] if n else None)


def gbr_set_sponge(h, sigma, ref=None):
    """sigma: device pointer (int) to ncell doubles, or None to remove the
    sponge; ref: reference primitive state (rho, u, v, w, p)."""
    if sigma is None:
        _check(lib().gbr_set_sponge(h, None, None), h)
        return
    r = (C.c_double * 5)(*[float(v) for v in ref])
    _check(lib().gbr_set_sponge(h, C.c_void_p(sigma), r), h)


def gbr_rhs(handles, Q, res):
    n = len(handles)
    _check(lib().gbr_rhs(_arr(handles), n, _arr(Q), _arr(res)), handles[0] if n else None)


def gbr_rk_stage(handles, stage, dt, Qn, Q, res):
    n = len(handles)
    _check(lib().gbr_rk_stage(_arr(handles), n, int(stage), _arr(dt), _arr(Qn), _arr(Q), _arr(res)),
           handles[0] if n else None)


def gbr_cfl(handles, Q, cfl, dt):
    n = len(handles)
    _check(lib().gbr_cfl(_arr(handles), n, _arr(Q), float(cfl), _arr(dt)), handles[0] if n else None)


def gbr_cfl_noalloc(handles, Q, cfl, dt):
    n = len(handles)
    _check(lib().gbr_cfl_noalloc(_arr(handles), n, _arr(Q), float(cfl), _arr(dt)), handles[0] if n else None)


def gbr_step(handles, Q, cfl_or_dt, dt_mode=GBR_DT_CFL, xyz=None, xyz_t=None, dt_out=None, t=None):
    n = len(handles)
    _check(lib().gbr_step(_arr(handles), n, _arr(Q), _arr(xyz) if xyz is not None else None,
                          _arr(xyz_t) if xyz_t is not None else None, float(cfl_or_dt), int(dt_mode),
                          _arr(dt_out) if dt_out is not None else None,
                          _arr(t) if t is not None else None), handles[0] if n else None)


def gbr_check_state(h):
    return int(lib().gbr_check_state(h))


def gbr_metric_ptr(h, slot):
    return lib().gbr_metric_ptr(h, int(slot))


KERNEL_CLASSES = ["metrics", "cell_grad", "sweep_xi", "sweep_eta", "sweep_zeta", "rk_stage", "cfl", "copy",
                  "prims", "diagnostics"]


def gbr_diagnostics(handles, Q, fields=None, integrals=None):
    n = len(handles)
    _check(lib().gbr_diagnostics(_arr(handles), n, _arr(Q), _arr(fields) if fields is not None else None,
                                 _arr(integrals) if integrals is not None else None),
           handles[0] if n else None)


def gbr_timing_enable(h, on=True):
    _check(lib().gbr_timing_enable(h, int(bool(on))), h)


def gbr_timing_collect(h):
    """{class: (total ms, launches)} since the last collect."""
    n = len(KERNEL_CLASSES)
    ms = (C.c_double * n)()
    cnt = (C.c_long * n)()
    _check(lib().gbr_timing_collect(h, ms, cnt), h)
    return {KERNEL_CLASSES[q]: (ms[q], cnt[q]) for q in range(n)}


def gbr_last_error(h):
    return lib().gbr_last_error(h).decode()


def gbr_probe_triad(a, b, c, s, stream=None):
    """a = b + s c over three device tensors of equal length (measurement probe)."""
    n = a.numel()
    if b.numel() != n or c.numel() != n:
        raise ValueError("triad operands differ in length")
    st = _stream() if stream is None else stream
    _check(lib().gbr_probe_triad(_ptr(a), _ptr(b), _ptr(c), float(s), n, C.c_void_p(st)))


def gbr_batch_create(handles, Q, tile=GBR_TILE_AUTO):
    n = len(handles)
    b = C.c_void_p()
    _check(lib().gbr_batch_create(_arr(handles), n, _arr(Q), int(tile), C.byref(b)),
           handles[0] if n else None)
    return b


def gbr_batch_run(b, steps, cfl_or_dt, dt_mode=GBR_DT_CFL, use_graph=True, err_handle=None):
    _check(lib().gbr_batch_run(b, int(steps), float(cfl_or_dt), int(dt_mode), int(bool(use_graph))),
           err_handle)


def gbr_batch_query(b, n, err_handle=None):
    """(t, dt, tile): per-grid accumulated time and last dt (host lists)."""
    t = (C.c_double * n)()
    dt = (C.c_double * n)()
    tile = C.c_int()
    _check(lib().gbr_batch_query(b, t, dt, C.byref(tile)), err_handle)
    return list(t), list(dt), tile.value


def gbr_batch_destroy(b):
    _check(lib().gbr_batch_destroy(b))


# ---------------------------------------------------------------------------
# convenience wrapper over one grid
# ---------------------------------------------------------------------------
class Grid:
    """One grid handle bound to the current torch stream. ``grid`` is a dict
    with n, ndim, off (and optionally xyz_t) as produced by ``workloads``."""

    def __init__(self, grid, **params):
        import torch
        self.n = tuple(grid["n"])
        self.ndim = int(grid["ndim"])
        self.nvar = self.ndim + 2
        self.moving = grid.get("xyz_t") is not None or params.pop("moving", False)
        self.bc = grid.get("bc")
        self.cfg = make_config(self.n, self.ndim, grid["off"], moving=self.moving, bc=self.bc, **params)
        self.precision = self.cfg.precision
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.h = gbr_grid_create(self.cfg)

    def close(self):
        if self.h:
            gbr_grid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    def metrics(self, xyz, xyz_t=None):
        gbr_metrics([self.h], [xyz], [xyz_t] if xyz_t is not None else None)

    def metrics_nonfp(self, xyz):
        gbr_metrics_nonfp([self.h], [xyz])

    def set_sponge(self, sigma, ref=None):
        """sigma: device tensor of ncell doubles (copied), or None."""
        gbr_set_sponge(self.h, _ptr(sigma) if sigma is not None else None, ref)

    def rhs(self, Q, res):
        gbr_rhs([self.h], [Q], [res])

    def rk_stage(self, stage, dt, Qn, Q, res):
        gbr_rk_stage([self.h], stage, [dt], [Qn], [Q], [res])

    def cfl(self, Q, cfl, dt):
        gbr_cfl([self.h], [Q], cfl, [dt])

    def step(self, Q, cfl_or_dt, dt_mode=GBR_DT_CFL, xyz=None, xyz_t=None, dt_out=None, t=None):
        """t: device tensor of one double, advanced by the step's dt."""
        gbr_step([self.h], [Q], cfl_or_dt, dt_mode, [xyz] if xyz is not None else None,
                 [xyz_t] if xyz_t is not None else None, [dt_out] if dt_out is not None else None,
                 [t] if t is not None else None)

    def diagnostics(self, Q, fields=None, integrals=None):
        """fields: device tensor [5][...] or None; integrals: device tensor of
        3 doubles or None."""
        gbr_diagnostics([self.h], [Q], [fields] if fields is not None else None,
                        [integrals] if integrals is not None else None)

    def res_dtype(self):
        import torch
        return torch.float32 if self.precision == GBR_FP32_BULK else torch.float64

    def check_state(self):
        return gbr_check_state(self.h)

    def metric(self, slot):
        """Copy of one metric slot as a torch tensor [nk][nj][ni] on the device."""
        import torch
        ptr = gbr_metric_ptr(self.h, slot)
        if not ptr:
            raise GbrError(GBR_E_ARG, "bad metric slot")
        out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        nbytes = out.numel() * 8
        torch.cuda.current_stream().synchronize()
        _memcpy_d2d(out.data_ptr(), ptr, nbytes)
        return out


def _memcpy_d2d(dst, src, nbytes):
    """Device-to-device copy through the HIP runtime torch already loaded."""
    global _hip
    try:
        _hip
    except NameError:
        _hip = None
    if _hip is None:
        for name in ("libamdhip64.so", "libamdhip64.so.7", "libamdhip64.so.6"):
            try:
                _hip = C.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            raise ImportError("libamdhip64 not found")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    rc = _hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(src), C.c_size_t(nbytes), 3)  # device to device
    if rc != 0:
        raise GbrError(GBR_E_DEVICE, f"hipMemcpy failed ({rc})")


class Batch:
    """Batched stepping of several 2-D Euler ``Grid`` objects whose metrics
    are computed; ``Q`` are their device states (advanced in place)."""

    def __init__(self, grids, Q, tile=GBR_TILE_AUTO):
        self.grids = list(grids)
        self.Q = list(Q)
        self.n = len(self.grids)
        self.h0 = self.grids[0].h if self.grids else None
        self.b = gbr_batch_create([g.h for g in self.grids], self.Q, tile)

    def run(self, steps, cfl_or_dt, dt_mode=GBR_DT_CFL, graph=True):
        gbr_batch_run(self.b, steps, cfl_or_dt, dt_mode, graph, self.h0)

    def query(self):
        return gbr_batch_query(self.b, self.n, self.h0)

    def close(self):
        if self.b:
            gbr_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

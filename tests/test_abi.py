"""The C-ABI library loads on the CPU and exports every symbol the header
declares; configuration sizing and validation need no GPU."""
import ctypes as C
import os
import subprocess

import pytest

from paper_2303_10785_amd import gbr


def test_library_exports_every_declared_function():
    names = gbr.header_functions()
    assert {"gbr_metrics", "gbr_rhs", "gbr_rk_stage", "gbr_step", "gbr_grid_create",
            "gbr_grid_destroy", "gbr_last_error"} <= set(names)
    L = gbr.lib()
    for nm in names:
        assert hasattr(L, nm), nm


def test_config_struct_matches_header_layout(tmp_path):
    """sizeof and field offsets of gbr_config as the C compiler sees the
    header agree with the ctypes mirror of the binding."""
    fields = [f[0] for f in gbr.gbr_config._fields_]
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"gbr.h\"\nint main(void){\n"
                   + 'printf("%zu\\n", sizeof(gbr_config));\n'
                   + "".join(f'printf("%zu\\n", offsetof(gbr_config, {f}));\n' for f in fields)
                   + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(gbr.HEADER), str(src), "-o", str(exe)], check=True)
    out = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert out[0] == C.sizeof(gbr.gbr_config)
    for f, off in zip(fields, out[1:]):
        assert getattr(gbr.gbr_config, f).offset == off, f


def test_grid_bytes_and_validation():
    cfg = gbr.make_config((8, 6, 4), 3, [[1, 0, 0], [0, 1, 0], [0, 0, 1]])
    n = 8 * 6 * 4
    assert gbr.gbr_grid_bytes(cfg) >= n * 8 * (gbr.SLOT_COUNT + 12)
    bad = [dict(ndim=4), dict(n=(0, 4, 4)), dict(ndim=2, n=(4, 4, 2)), dict(limiter=7),
           dict(gamma=1.0), dict(Re=0.0)]
    for b in bad:
        kw = dict(n=(8, 6, 4), ndim=3, off=[[1, 0, 0], [0, 1, 0], [0, 0, 1]])
        kw.update(b)
        assert gbr.gbr_grid_bytes(gbr.make_config(**kw)) == 0, b


def test_boundary_config_validation():
    """Boundary types: both sides of a direction periodic or neither, at
    least 2 GBR_NG + 12 cells along a bounded direction, only d < ndim."""
    off = [[1, 0, 0], [0, 1, 0], [0, 0, 1]]
    ok = gbr.make_config((24, 30, 8), 3, off, bc=[("inflow", "outflow"), ("wall", "wall")])
    assert gbr.gbr_grid_bytes(ok) > 0
    for bc, n, nd in [([("inflow", "periodic")], (24, 30, 8), 3),
                      ([("periodic", "wall")], (24, 30, 8), 3),
                      ([("inflow", "outflow")], (23, 30, 8), 3),
                      ([("periodic", "periodic"), ("periodic", "periodic"), ("wall", "wall")], (24, 24, 1), 2),
                      ([(7, 0)], (24, 30, 8), 3)]:
        assert gbr.gbr_grid_bytes(gbr.make_config(n, nd, off, bc=bc)) == 0, bc
    assert gbr.lib().gbr_set_sponge(None, None, None) == gbr.GBR_E_ARG


def test_null_arguments_rejected_without_device_work():
    L = gbr.lib()
    assert L.gbr_grid_create(None, None, None) == gbr.GBR_E_ARG
    out = C.c_void_p()
    cfg = gbr.make_config((4, 4, 4), 5, [[1, 0, 0], [0, 1, 0], [0, 0, 1]])
    assert L.gbr_grid_create(C.byref(cfg), None, C.byref(out)) == gbr.GBR_E_ARG
    assert out.value is None
    # empty batches are no-ops
    assert L.gbr_rhs(None, 0, None, None) == gbr.GBR_OK
    assert L.gbr_metrics(None, 0, None, None) == gbr.GBR_OK
    assert L.gbr_step(None, 0, None, None, None, 0.1, 0, None, None) == gbr.GBR_OK
    assert L.gbr_rhs(None, -1, None, None) == gbr.GBR_E_ARG
    assert L.gbr_check_state(None) == gbr.GBR_E_ARG
    assert L.gbr_last_error(None) == b"null grid handle"
    assert L.gbr_metric_ptr(None, 0) is None
    # batched stepping
    b = C.c_void_p()
    assert L.gbr_batch_create(None, 1, None, -1, C.byref(b)) == gbr.GBR_E_ARG
    assert L.gbr_batch_create(None, 0, None, -1, C.byref(b)) == gbr.GBR_E_ARG
    assert L.gbr_batch_create(None, 1, None, -1, None) == gbr.GBR_E_ARG
    assert b.value is None
    assert L.gbr_batch_run(None, 1, 0.4, 0, 1) == gbr.GBR_E_ARG
    assert L.gbr_batch_query(None, None, None, None) == gbr.GBR_E_ARG
    assert L.gbr_batch_destroy(None) == gbr.GBR_OK
    assert L.gbr_diagnostics(None, 0, None, None, None) == gbr.GBR_OK
    assert L.gbr_diagnostics(None, 1, None, None, None) == gbr.GBR_E_ARG


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(gbr, "_lib", None)
    monkeypatch.setattr(gbr, "HERE", str(tmp_path))
    with pytest.raises(ImportError):
        gbr.lib()

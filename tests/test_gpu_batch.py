"""Batched stepping of many 2-D Euler grids (gbr_batch_*) against the FP64
oracle, plus the properties serving relies on: a grid's result does not
depend on which other grids share the batch, graph replay equals eager
launches, per-grid time steps and per-grid state flags.

Tolerances: FP64 as for single grids (max relative error 1e-12 per step,
per variable); FP32-bulk against the FP64 oracle on smooth data as for the
single-grid FP32-bulk path (1e-5 per step).
"""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
FP32_STEP_TOL = 1e-5
CFL = 0.4
PARAMS = dict(viscous=False, limiter="mp")


@pytest.fixture(scope="module")
def gbr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_10785_amd import gbr as G
    G.lib()
    return G


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def say(*a):
    print(*a, flush=True)


def rel(gpu, ref):
    worst = 0.0
    for v in range(ref.shape[0]):
        s = float(np.abs(ref[v]).max())
        d = float(np.abs(gpu[v] - ref[v]).max())
        worst = max(worst, d / s if s > 0 else d)
    return worst


def cases():
    """Grids of several tile counts, a ragged tail in both directions, one
    smaller than a tile, and both initial conditions of the batch workload."""
    out = []
    g = W.wavy2d((37, 29), amp=0.08, rand=0.1, seed=21)
    out.append(("37x29 vortex", g, W.shu_vortex(g)))
    g = W.wavy2d((70, 64), amp=0.05)
    out.append(("70x64 sod+vortex", g, W.vortex_sod(g)))
    g = W.wavy2d((5, 3), amp=0.02)
    out.append(("5x3 vortex", g, W.shu_vortex(g)))
    g = W.wavy2d((16, 16), amp=0.1)
    out.append(("16x16 vortex", g, W.shu_vortex(g, eps=3.0)))
    g = W.wavy2d((33, 17), amp=0.06)
    out.append(("33x17 sod+vortex", g, W.vortex_sod(g)))
    return out


def make(gbr, cs, precision="fp64", limiter="mp"):
    grids, Qs = [], []
    for _, g, Q in cs:
        h = gbr.Grid(g, precision=precision, viscous=False, limiter=limiter)
        h.metrics(dev(g["xyz"]))
        grids.append(h)
        Qs.append(dev(Q))
    return grids, Qs


@pytest.mark.parametrize("tile", [0, 1, 2])
def test_batch_fp64_matches_oracle(gbr, tile):
    cs = cases()
    grids, Qs = make(gbr, cs)
    b = gbr.Batch(grids, Qs, tile=tile)
    refs = [(g, oracle.metrics(g, **PARAMS), Q) for _, g, Q in cs]
    for step in range(2):
        b.run(1, CFL, gbr.GBR_DT_CFL, graph=True)
        _, dts, used = b.query()
        assert used == tile
        for q, (name, g, _) in enumerate(cs):
            gg, m, Qr = refs[q]
            Qr, dt_ref = oracle.step(gg, m, Qr, CFL, **PARAMS)
            refs[q] = (gg, m, Qr)
            e = rel(Qs[q].cpu().numpy(), Qr)
            say(f"[batch fp64 tile {gbr.TILE_NAMES[tile]}] {name} step {step}: max rel err {e:.3e}")
            assert e <= TOL, (name, step, e)
            assert abs(dts[q] - dt_ref) <= TOL * dt_ref, (name, dts[q], dt_ref)
    for h in grids:
        assert h.check_state() == gbr.GBR_OK
    b.close()
    for h in grids:
        h.close()


def test_batch_fixed_dt_and_no_limiter(gbr):
    """GBR_DT_FIXED and limiter NONE (the direct van Leer states) on the
    smooth cases (without a limiter the Sod jumps go non-physical)."""
    cs = [c for c in cases() if "sod" not in c[0]]
    params = dict(viscous=False, limiter="none")
    grids, Qs = make(gbr, cs, limiter="none")
    b = gbr.Batch(grids, Qs, tile=gbr.GBR_TILE_AUTO)
    b.run(2, 1e-3, gbr.GBR_DT_FIXED, graph=False)
    t, dts, tile = b.query()
    assert tile in (0, 1, 2)
    assert all(abs(x - 2e-3) <= 1e-18 for x in t) and all(x == 1e-3 for x in dts)
    for q, (name, g, Q) in enumerate(cs):
        m = oracle.metrics(g, **params)
        for _ in range(2):
            Q, _ = oracle.step(g, m, Q, 1e-3, dt_mode=oracle.DT_FIXED, **params)
        e = rel(Qs[q].cpu().numpy(), Q)
        say(f"[batch fp64 none fixed dt] {name}: max rel err {e:.3e}")
        assert e <= TOL, (name, e)
    b.close()


def test_batch_fp32_bulk_against_fp64_oracle(gbr):
    """FP32-bulk batch on smooth vortex data against the FP64 oracle."""
    cs = [c for c in cases() if "vortex" in c[0] and "sod" not in c[0]]
    grids, Qs = make(gbr, cs, precision="fp32_bulk")
    b = gbr.Batch(grids, Qs, tile=0)
    refs = [(oracle.metrics(g, **PARAMS), Q) for _, g, Q in cs]
    for step in range(2):
        b.run(1, CFL, gbr.GBR_DT_CFL, graph=True)
        for q, (name, g, _) in enumerate(cs):
            m, Qr = refs[q]
            Qr, _ = oracle.step(g, m, Qr, CFL, **PARAMS)
            refs[q] = (m, Qr)
            e = rel(Qs[q].cpu().numpy(), Qr)
            say(f"[batch fp32] {name} step {step}: max rel err vs FP64 oracle {e:.3e}")
            assert e <= FP32_STEP_TOL, (name, e)
    b.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_alone_equals_mix(gbr, precision):
    """A grid stepped alone and inside a batch of other grids gives bitwise
    the same state and time (same tile shape)."""
    cs = cases()
    grids, Qs = make(gbr, cs, precision=precision)
    mix = gbr.Batch(grids, Qs, tile=1)
    mix.run(3, CFL, gbr.GBR_DT_CFL, graph=True)
    t_mix, _, _ = mix.query()
    mix.close()
    for q, (name, g, Q) in enumerate(cs):
        h, = make(gbr, [cs[q]], precision=precision)[0]
        Qa = dev(Q)
        alone = gbr.Batch([h], [Qa], tile=1)
        alone.run(3, CFL, gbr.GBR_DT_CFL, graph=True)
        t_alone, _, _ = alone.query()
        same = torch.equal(Qa, Qs[q])
        say(f"[alone vs mix {precision}] {name}: bitwise equal {same}")
        assert same, name
        assert t_alone[0] == t_mix[q]
        alone.close()
        h.close()


def test_graph_replay_equals_eager(gbr):
    """Replays of the captured step, with eager torch work and host
    synchronisation between them, equal eager launches bitwise."""
    cs = cases()
    ga, Qa = make(gbr, cs)
    ge, Qe = make(gbr, cs)
    A = gbr.Batch(ga, Qa, tile=0)
    E = gbr.Batch(ge, Qe, tile=0)
    for step in range(4):
        A.run(1, CFL, gbr.GBR_DT_CFL, graph=True)
        E.run(1, CFL, gbr.GBR_DT_CFL, graph=False)
        junk = sum(float(x.abs().sum()) for x in Qa)  # eager library work between replays
        torch.cuda.synchronize()
        assert np.isfinite(junk)
        for q in range(len(cs)):
            assert torch.equal(Qa[q], Qe[q]), (step, cs[q][0])
    ta, _, _ = A.query()
    te, _, _ = E.query()
    assert ta == te
    A.close()
    E.close()


def test_batch_flags_only_the_bad_grid(gbr):
    cs = cases()[:3]
    bad = cs[1][2].copy()
    bad[-1, 0, 10] = -1.0  # negative energy: non-physical cell in grid 1
    cs[1] = (cs[1][0], cs[1][1], bad)
    grids, Qs = make(gbr, cs)
    b = gbr.Batch(grids, Qs, tile=0)
    b.run(1, CFL, gbr.GBR_DT_CFL, graph=False)
    b.query()
    assert grids[0].check_state() == gbr.GBR_OK
    assert grids[1].check_state() == gbr.GBR_E_STATE
    assert grids[2].check_state() == gbr.GBR_OK
    b.close()


def test_batch_rejects_unsupported_grids(gbr):
    g2 = W.wavy2d((16, 16))
    g3 = W.random3d((8, 8, 8))
    h2 = gbr.Grid(g2, viscous=False, limiter="mp")
    h2b = gbr.Grid(g2, viscous=False, limiter="mp", precision="fp32_bulk")
    hv = gbr.Grid(g2, viscous=True, limiter="mp")
    hd = gbr.Grid(g2, viscous=False, limiter="ducros")
    h3 = gbr.Grid(g3, viscous=False, limiter="mp")
    Q2 = dev(W.shu_vortex(g2))
    Q3 = dev(W.uniform_flow(g3))
    for hs, Qs, status in [([h3], [Q3], gbr.GBR_E_UNSUPPORTED), ([hv], [Q2], gbr.GBR_E_UNSUPPORTED),
                           ([hd], [Q2], gbr.GBR_E_UNSUPPORTED), ([h2, h2b], [Q2, Q2], gbr.GBR_E_ARG),
                           ([h2, h2], [Q2, Q2], gbr.GBR_E_ARG)]:
        with pytest.raises(gbr.GbrError) as ei:
            gbr.Batch(hs, Qs)
        assert ei.value.status == status
    with pytest.raises(gbr.GbrError) as ei:
        gbr.Batch([h2], [Q2], tile=7)
    assert ei.value.status == gbr.GBR_E_ARG
    b = gbr.Batch([h2], [Q2], tile=0)
    for args in [(-1, 0.4, 0), (1, 0.0, 0), (1, 0.4, 5)]:
        with pytest.raises(gbr.GbrError):
            b.run(*args)
    b.close()
    for h in (h2, h2b, hv, hd, h3):
        h.close()

"""gbr_cfl_noalloc (the time step for callers that cannot allocate) against
gbr_cfl through the C ABI: bitwise the same dt, on two calls in a row, the
second with fewer and smaller grids, and the bound on grids per call."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gbr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_10785_amd import gbr as G
    G.lib()
    return G


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def setup(gbr, cases):
    hs, Qs = [], []
    for g, params, Q in cases:
        h = gbr.Grid(g, **params)
        h.metrics(dev(g["xyz"]))
        hs.append(h)
        Qs.append(dev(Q))
    return hs, Qs


def dts_of(gbr, fn, hs, Qs, cfl):
    dts = [torch.full((1,), -1.0, dtype=torch.float64, device="cuda") for _ in hs]
    fn([h.h for h in hs], Qs, cfl, dts)
    torch.cuda.synchronize()
    return [float(d.item()) for d in dts]


def test_noalloc_cfl_equals_cfl_twice(gbr):
    big3 = W.random3d((128, 96, 96), amp=0.2, seed=81)      # more cells than 4096 blocks of 256 cover
    mid2 = W.wavy2d((37, 23), L=4.0, amp=0.08, rand=0.2, seed=82)
    small3 = W.random3d((9, 8, 7), amp=0.2, seed=83)
    cases = [(big3, dict(viscous=True, limiter="ducros", Re=300.0), W.random_smooth_state(big3, seed=1)),
             (mid2, dict(limiter="mp"), W.shu_vortex(mid2, xc=2.0, yc=2.0)),
             (small3, dict(viscous=True, limiter="mp", Re=50.0), W.random_rough_state(small3, seed=2))]
    hs, Qs = setup(gbr, cases)
    ref = dts_of(gbr, gbr.gbr_cfl, hs, Qs, 0.3)
    got = dts_of(gbr, gbr.gbr_cfl_noalloc, hs, Qs, 0.3)
    print(f"[noalloc] 3 grids: gbr_cfl {ref}, gbr_cfl_noalloc {got}", flush=True)
    assert got == ref
    for (g, params, Q), d in zip(cases, got):
        d_ref = 0.3 * oracle.cfl_min(g, oracle.metrics(g, **params), Q, **params)
        assert abs(d - d_ref) <= 1e-12 * d_ref
    # second call: one smaller grid, after the scratch holds the first call's partials
    ref2 = dts_of(gbr, gbr.gbr_cfl, hs[2:], Qs[2:], 0.25)
    got2 = dts_of(gbr, gbr.gbr_cfl_noalloc, hs[2:], Qs[2:], 0.25)
    print(f"[noalloc] 1 small grid: gbr_cfl {ref2}, gbr_cfl_noalloc {got2}", flush=True)
    assert got2 == ref2
    for h in hs:
        h.close()


def test_noalloc_cfl_rejects_too_many_grids(gbr):
    g = W.random3d((6, 5, 4), amp=0.1, seed=84)
    h = gbr.Grid(g, limiter="mp")
    h.metrics(dev(g["xyz"]))
    Q = dev(W.random_smooth_state(g, seed=3))
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(gbr.GbrError) as ei:
        gbr.gbr_cfl_noalloc([h.h] * 33, [Q] * 33, 0.3, [dt] * 33)
    assert ei.value.status == gbr.GBR_E_ARG and "at most 32" in str(ei.value)
    ok = dts_of(gbr, gbr.gbr_cfl_noalloc, [h] * 32, [Q] * 32, 0.3)
    assert len(set(ok)) == 1 and ok[0] > 0
    h.close()

"""Serving loop on the GPU: every request of a small mixed trace finishes
with a physical state; a request served alone and inside the mix ends in
bitwise the same state (FP64 and FP32-bulk, 2-D batched and 3-D); and a
served FP64 request matches the oracle stepped the same number of times."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def serve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_10785_amd import gbr, serve as S
    gbr.lib()
    return S


def small_trace(S):
    return S.make_trace(10, rate=400.0, seed=9, n2d=(12, 48), n3d=(8, 14), steps=(4, 30))


def test_mixed_trace_and_alone_equals_mix(serve):
    tr = small_trace(serve)
    ex = serve.GpuExecutor(keep_results=True)
    out = serve.run(tr, ex, budget_bytes=8 << 30, tick_steps=7)
    print(f"[serve] {out}", flush=True)
    assert out["requests"] == len(tr) and out["all_states_ok"]
    mixed = dict(ex.results)
    ex.close()
    kinds = set()
    for r in tr:
        key = (r.ndim, r.precision)
        if key in kinds:
            continue
        kinds.add(key)
        solo = serve.GpuExecutor(keep_results=True)
        alone = serve.Request(r.rid, 0.0, r.ndim, r.n, r.steps, r.precision, r.ic, r.seed)
        o = serve.run([alone], solo, budget_bytes=8 << 30, tick_steps=5)
        assert o["all_states_ok"]
        same = np.array_equal(solo.results[r.rid], mixed[r.rid])
        print(f"[serve] request {r.rid} ({r.ndim}-D {r.precision} n={r.n} steps={r.steps}): "
              f"alone == mix bitwise: {same}", flush=True)
        assert same
        solo.close()
    assert len(kinds) >= 3


def test_served_request_matches_oracle(serve):
    req = serve.Request(0, 0.0, 2, 20, 6, "fp64", "sod", 11)
    ex = serve.GpuExecutor(keep_results=True)
    serve.run([req], ex, budget_bytes=1 << 30, tick_steps=4)
    got = ex.results[0]
    ex.close()
    grid, xyz, Q = serve.request_inputs(req, torch.device("cuda"))
    g = dict(grid, xyz=xyz.cpu().numpy())
    params = dict(viscous=False, limiter="mp")
    m = oracle.metrics(g, **params)
    Qr = Q.cpu().numpy()
    for _ in range(req.steps):
        Qr, _ = oracle.step(g, m, Qr, serve.CFL_2D, **params)
    err = max(float(np.abs(got[v] - Qr[v]).max() / np.abs(Qr[v]).max()) for v in range(4))
    print(f"[serve] served 2-D FP64 request vs oracle after {req.steps} steps: {err:.3e}", flush=True)
    assert err <= TOL

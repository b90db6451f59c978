"""Diagnostics (vorticity, Q-criterion, |grad rho|, Eq. KE-Ens averages) on
the GPU against the FP64 oracle: fields within 1e-12 of the largest value
of each field, integrals within 1e-12 relative; FP32-bulk within 1e-4."""
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


CASES = [
    ("random3d_meg6", lambda: W.random3d((11, 9, 8), seed=3), "meg6", lambda g: W.random_smooth_state(g, seed=2)),
    ("random3d_mig4", lambda: W.random3d((11, 9, 8), seed=3), "mig4", lambda g: W.random_rough_state(g, seed=4, amp=0.1)),
    ("wavy2d_meg6", lambda: W.wavy2d((33, 29), rand=0.1, seed=5), "meg6", lambda g: W.shu_vortex(g)),
    ("wavy2d_mig4", lambda: W.wavy2d((33, 29), rand=0.1, seed=5), "mig4", lambda g: W.shu_vortex(g)),
    ("tiny_meg6", lambda: W.random3d((4, 3, 2), seed=1), "meg6", lambda g: W.random_smooth_state(g, seed=6)),
    ("jet_meg6", lambda: W.jet3d((48, 20, 20)), "meg6", lambda g: W.jet_ic(g)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_diagnostics_match_oracle(gbr, case, precision):
    name, grid, scheme, state = case
    g = grid()
    Q = state(g)
    h = gbr.Grid(g, scheme=scheme, precision=precision)
    h.metrics(dev(g["xyz"]))
    f = torch.zeros((5,) + h.shape, dtype=torch.float64, device="cuda")
    it = torch.zeros(3, dtype=torch.float64, device="cuda")
    h.diagnostics(dev(Q), f, it)
    f2 = torch.zeros_like(f)
    it2 = torch.zeros_like(it)
    h.diagnostics(dev(Q), f2, it2)  # repeatable bit for bit
    torch.cuda.synchronize()
    assert torch.equal(f, f2) and torch.equal(it, it2)
    h.close()
    m = oracle.metrics(g, scheme=scheme)
    fr, itr = oracle.diagnostics(g, m, Q, scheme=scheme)
    tol = 1e-12 if precision == "fp64" else 1e-4
    got = f.cpu().numpy()
    for q in range(5):
        s = float(np.abs(fr[q]).max())
        err = float(np.abs(got[q] - fr[q]).max())
        assert err <= tol * max(s, 1e-300) or (s == 0 and err <= 1e-15), (name, q, err, s)
    for q, (a, b) in enumerate(zip(it.cpu().numpy(), itr)):
        assert abs(a - b) <= tol * abs(b) + 1e-300, (name, q, a, b)
    print(f"[diag] {name} {precision}: integrals {it.cpu().numpy()} vs {itr}", flush=True)

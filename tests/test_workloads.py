"""Properties of the seeded inputs that parity cases rely on (CPU only)."""
import numpy as np

import oracle
import workloads as W


def _face_branch_fractions(g, Q, gamma=1.4):
    """Per face family, the fraction of interfaces whose two cell states give
    HLLC wave-speed estimates (Sec. 5.1.1: S_L = min(U_L - c_L|n|, U_R - c_R|n|),
    S_R = max(U_L + c_L|n|, U_R + c_R|n|)) with S_L > 0, and with S_R < 0, each
    by a margin of half a sound speed so that the reconstructed states, which
    differ from the cell states by the reconstruction corrections, fall on the
    same side."""
    m = oracle.metrics(g)
    rho, u, v, w, p = oracle.prim_from_Q(Q, gamma)
    c = np.sqrt(gamma * p / rho)
    out = []
    axis_of = {0: 2, 1: 1, 2: 0}  # array axes are [k][j][i]
    for f in range(g["ndim"]):
        nx, ny, nz = (m[oracle.M_FHAT(f, e)] for e in range(3))
        sn = np.sqrt(nx * nx + ny * ny + nz * nz)
        ax = axis_of[f]
        nxt = lambda a: np.roll(a, -1, axis=ax)  # noqa: E731  (cell i+1 of face i+1/2)
        UL = nx * u + ny * v + nz * w
        UR = nx * nxt(u) + ny * nxt(v) + nz * nxt(w)
        SL = np.minimum(UL - c * sn, UR - nxt(c) * sn)
        SR = np.maximum(UL + c * sn, UR + nxt(c) * sn)
        margin = 0.5 * np.minimum(c, nxt(c)) * sn
        out.append((float(np.mean(SL > margin)), float(np.mean(SR < -margin))))
    return out


def test_supersonic_state_reaches_one_sided_hllc_branches():
    """The supersonic parity state puts a fifth or more of every face family
    on each one-sided HLLC branch, with margin."""
    for g in [W.random3d((21, 13, 9), amp=0.2, seed=61),
              W.wavy2d((37, 23), L=4.0, amp=0.08, rand=0.2, seed=62),
              W.jet3d((40, 18, 18)),
              W.wavy2d((40, 24), L=4.0, amp=0.05, rand=0.1, seed=71)]:
        Q = W.supersonic_rough_state(g, seed=3)
        for f, (fl, fr) in enumerate(_face_branch_fractions(g, Q)):
            assert fl >= 0.2 and fr >= 0.2, (g["n"], f, fl, fr)


def test_rough_state_stays_subsonic():
    """The ordinary rough state never reaches the one-sided branches by this
    estimate: the supersonic state above is what covers them."""
    g = W.random3d((21, 13, 9), amp=0.2, seed=61)
    Q = W.random_rough_state(g, seed=3)
    for fl, fr in _face_branch_fractions(g, Q):
        assert fl == 0.0 and fr == 0.0

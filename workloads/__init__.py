"""Seeded synthetic inputs: grids (cell-centre coordinates and grid velocities)
and initial conditions.

This module serves both the HIP path and the CPU oracle. It holds none of the
method's arithmetic (no derivatives, metrics, fluxes or time stepping): only
analytic node positions, their vertex centroids and closed-form initial states.

Conventions
-----------
* A grid is a dict with
    ``n``    : (ni, nj, nk) cell counts along xi, eta, zeta (nk = 1 in 2-D),
    ``ndim`` : 2 or 3,
    ``xyz``  : float64 array [3][nk][nj][ni] of cell-centre coordinates,
    ``off``  : float64 [3][3]; ``off[d]`` is the (x, y, z) shift of the
               coordinates when the index along direction d wraps by n[d]
               (all grids here are periodic in every direction),
    ``xyz_t``: float64 [3][nk][nj][ni] grid velocity at the cell centres, or
               None for a static grid.
  In 2-D the z coordinate is zero and ``off[2] = (0, 0, 1)``.
    ``bc``   : optional, per direction a pair (low, high) of "periodic",
               "inflow", "outflow" or "wall" (see ``bounded``).
* Cell centres are the centroids of the cell's vertices (Sec. 3 of the paper:
  the solution lives at the vertex centroid of each hexahedral cell).
* Q is float64 [nvar][nk][nj][ni], nvar = ndim + 2, variable order
  (rho, rho u, rho v, [rho w], E).
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 2303_10785


# ----------------------------------------------------------------------------
# node -> cell-centre helpers
# ----------------------------------------------------------------------------
def _centroids3(X, Y, Z):
    """Vertex centroids of the cells of a (nk+1, nj+1, ni+1) node lattice."""
    def c(A):
        return 0.125 * (A[:-1, :-1, :-1] + A[:-1, :-1, 1:] + A[:-1, 1:, :-1]
                        + A[:-1, 1:, 1:] + A[1:, :-1, :-1] + A[1:, :-1, 1:]
                        + A[1:, 1:, :-1] + A[1:, 1:, 1:])
    return np.stack([c(X), c(Y), c(Z)])


def _centroids2(X, Y):
    """Vertex centroids of a (nj+1, ni+1) node lattice, returned as [3][1][nj][ni]."""
    def c(A):
        return 0.25 * (A[:-1, :-1] + A[:-1, 1:] + A[1:, :-1] + A[1:, 1:])
    cx, cy = c(X), c(Y)
    return np.stack([cx, cy, np.zeros_like(cx)])[:, None, :, :].copy()


def _grid(n, ndim, xyz, off, xyz_t=None, **extra):
    g = dict(n=tuple(int(v) for v in n), ndim=int(ndim),
             xyz=np.ascontiguousarray(xyz, dtype=np.float64),
             off=np.asarray(off, dtype=np.float64).reshape(3, 3).copy(),
             xyz_t=None if xyz_t is None else np.ascontiguousarray(xyz_t, dtype=np.float64))
    g.update(extra)
    return g


def _periodic_noise(rng, shape_nodes, amp):
    """Uniform U[-amp, amp] node noise that is periodic (last node = first)."""
    base = rng.uniform(-amp, amp, size=tuple(s - 1 for s in shape_nodes))
    pad = [(0, 1)] * len(shape_nodes)
    return np.pad(base, pad, mode="wrap")


# ----------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------
def uniform3d(n, L=(1.0, 1.0, 1.0)):
    ni, nj, nk = n
    i = np.arange(ni + 1) * (L[0] / ni)
    j = np.arange(nj + 1) * (L[1] / nj)
    k = np.arange(nk + 1) * (L[2] / nk)
    Z, Y, X = np.meshgrid(k, j, i, indexing="ij")
    return _grid(n, 3, _centroids3(X, Y, Z), np.diag(L))


def uniform2d(n, L=(1.0, 1.0)):
    ni, nj = n
    i = np.arange(ni + 1) * (L[0] / ni)
    j = np.arange(nj + 1) * (L[1] / nj)
    Y, X = np.meshgrid(j, i, indexing="ij")
    return _grid((ni, nj, 1), 2, _centroids2(X, Y),
                 [[L[0], 0, 0], [0, L[1], 0], [0, 0, 1.0]])


def wavy2d(n, L=10.0, amp=0.1, rand=0.0, seed=0):
    """x = L[xi + amp sin(2 pi eta) sin(2 pi xi)], y = L[eta + amp sin(2 pi xi) sin(2 pi eta)],
    xi = i/ni, eta = j/nj, periodic with period L; optional seeded uniform node
    noise of +-rand cell widths."""
    ni, nj = n
    xi = np.arange(ni + 1) / ni
    et = np.arange(nj + 1) / nj
    ET, XI = np.meshgrid(et, xi, indexing="ij")
    s = np.sin(2 * np.pi * ET) * np.sin(2 * np.pi * XI)
    X = L * (XI + amp * s)
    Y = L * (ET + amp * s)
    if rand:
        rng = np.random.default_rng(SEED_BASE + seed)
        X = X + _periodic_noise(rng, X.shape, rand * L / ni)
        Y = Y + _periodic_noise(rng, Y.shape, rand * L / nj)
    return _grid((ni, nj, 1), 2, _centroids2(X, Y),
                 [[L, 0, 0], [0, L, 0], [0, 0, 1.0]])


def sinusoidal3d(n, L=4.0):
    """Static sinusoidal grid of the 3-D uniform-flow test (Sec. 8.1.1):
    x = xmin + dx[(i-1) + sin(pi (j-1) dy) sin(pi (k-1) dz)] and cyclic."""
    ni, nj, nk = n
    dx, dy, dz = L / ni, L / nj, L / nk
    i = np.arange(ni + 1)
    j = np.arange(nj + 1)
    k = np.arange(nk + 1)
    K, J, I = np.meshgrid(k, j, i, indexing="ij")
    X = -L / 2 + dx * (I + np.sin(np.pi * J * dy) * np.sin(np.pi * K * dz))
    Y = -L / 2 + dy * (J + np.sin(np.pi * K * dz) * np.sin(np.pi * I * dx))
    Z = -L / 2 + dz * (K + np.sin(np.pi * I * dx) * np.sin(np.pi * J * dy))
    # periodic only when L * pi * ... returns to zero at the last node: L = 4
    # with unit-period sines (pi * n * L / n = pi L) gives sin(4 pi) = 0.
    return _grid(n, 3, _centroids3(X, Y, Z), np.diag([L, L, L]))


def random3d(n, L=4.0, amp=0.2, seed=0):
    """Uniform grid whose nodes move by seeded U[-amp, amp] cell widths in
    each coordinate (the randomized grid of Sec. 8.1.1), periodic."""
    ni, nj, nk = n
    g = uniform3d(n, (L, L, L))
    i = np.arange(ni + 1) * (L / ni)
    j = np.arange(nj + 1) * (L / nj)
    k = np.arange(nk + 1) * (L / nk)
    Z, Y, X = np.meshgrid(k, j, i, indexing="ij")
    rng = np.random.default_rng(SEED_BASE + seed)
    X = X + _periodic_noise(rng, X.shape, amp * L / ni)
    Y = Y + _periodic_noise(rng, Y.shape, amp * L / nj)
    Z = Z + _periodic_noise(rng, Z.shape, amp * L / nk)
    g["xyz"] = _centroids3(X, Y, Z)
    return g


class Deforming3D:
    """Deforming sinusoidal grid (Sec. 8.2.1) with an optional static seeded
    node perturbation:

        x(t) = xmin + dx [i + A sin(2 pi w t) sin(n pi j dy / L) sin(n pi k dz / L)] + noise

    and cyclic for y, z. The grid velocity is the analytic time derivative.
    Both are linear in sin / cos of (2 pi w t), so cell centres are
    ``base + sin(2 pi w t) * mode`` and velocities ``2 pi w cos(2 pi w t) * mode``.
    """

    def __init__(self, n, L=12.0, A=1.5, nmode=4, omega=1.0, rand=0.0, seed=0):
        ni, nj, nk = n
        self.n, self.L, self.A, self.nmode, self.omega = tuple(n), L, A, nmode, omega
        dx, dy, dz = L / ni, L / nj, L / nk
        i = np.arange(ni + 1)
        j = np.arange(nj + 1)
        k = np.arange(nk + 1)
        K, J, I = np.meshgrid(k, j, i, indexing="ij")
        X0 = -L / 2 + dx * I
        Y0 = -L / 2 + dy * J
        Z0 = -L / 2 + dz * K
        if rand:
            rng = np.random.default_rng(SEED_BASE + seed)
            X0 = X0 + _periodic_noise(rng, X0.shape, rand * dx)
            Y0 = Y0 + _periodic_noise(rng, Y0.shape, rand * dy)
            Z0 = Z0 + _periodic_noise(rng, Z0.shape, rand * dz)
        s = lambda a, d: np.sin(nmode * np.pi * a * d / L)
        MX = dx * A * s(J, dy) * s(K, dz)
        MY = dy * A * s(I, dx) * s(K, dz)
        MZ = dz * A * s(I, dx) * s(J, dy)
        self.base = _centroids3(X0, Y0, Z0)
        self.mode = _centroids3(MX, MY, MZ)
        self.off = np.diag([L, L, L])

    def at(self, t):
        w = 2 * np.pi * self.omega
        xyz = self.base + math.sin(w * t) * self.mode
        xyz_t = (w * math.cos(w * t)) * self.mode
        return _grid(self.n, 3, xyz, self.off, xyz_t)


class Deforming2D:
    """Deforming 2-D grid of the double periodic shear layer (Sec. 8.2,
    Eq. DPSL-eqn1 / DPSL-eqn2):

        x(t) = xmin + dx [i + A sin(2 pi w t) sin(n pi j dy / L)]
        y(t) = ymin + dy [j + A sin(2 pi w t) sin(n pi i dx / L)]

    with i, j the node indices from 0. The printed phase terms i phi / (IL - 1)
    are taken as zero (any other value breaks the periodicity of the grid);
    A and n, which the paper takes from its reference, default to the values
    of its 3-D deforming case (1.5 cells, 4). Cell centres are
    ``base + sin(2 pi w t) * mode``, velocities ``2 pi w cos(2 pi w t) * mode``.
    """

    def __init__(self, n, L=1.0, A=1.5, nmode=4, omega=1.0):
        ni, nj = n
        self.n, self.L, self.A, self.nmode, self.omega = (ni, nj, 1), L, A, nmode, omega
        dx, dy = L / ni, L / nj
        J, I = np.meshgrid(np.arange(nj + 1), np.arange(ni + 1), indexing="ij")
        X0, Y0 = dx * I, dy * J
        MX = dx * A * np.sin(nmode * np.pi * J * dy / L)
        MY = dy * A * np.sin(nmode * np.pi * I * dx / L)
        self.base = _centroids2(X0, Y0)
        self.mode = _centroids2(MX, MY)
        self.off = [[L, 0, 0], [0, L, 0], [0, 0, 1.0]]

    def at(self, t):
        w = 2 * np.pi * self.omega
        xyz = self.base + math.sin(w * t) * self.mode
        xyz_t = (w * math.cos(w * t)) * self.mode
        return _grid(self.n, 2, xyz, self.off, xyz_t)


def dpsl_ic(grid, gamma=5.0 / 3.0, M=0.1):
    """Double periodic shear layer (Sec. 8.2): rho = 1 / (gamma M^2),
    u = tanh(80 (y - 1/4)) for y <= 1/2 and tanh(80 (3/4 - y)) above,
    v = 0.05 sin(2 pi (x + 1/4)), T = 1 (so p = rho T / (gamma M^2)) on the
    unit square."""
    x, y = grid["xyz"][0], grid["xyz"][1]
    g = gamma * M * M
    rho = np.full_like(x, 1.0 / g)
    u = np.where(y <= 0.5, np.tanh(80.0 * (y - 0.25)), np.tanh(80.0 * (0.75 - y)))
    v = 0.05 * np.sin(2 * np.pi * (x + 0.25))
    p = rho * 1.0 / g
    return conserved(rho, u, v, 0 * u, p, gamma, 2)


def jet3d(n=(400, 180, 180), a_x=0.86, b_yz=0.325, skew=0.02):
    """Jet-shaped stretched periodic grid (synthetic stand-in for the paper's
    13 M-cell jet mesh of Sec. 8.3; the real mesh is not published).

    Axial: x = Lx [xi - a/(2 pi) sin(2 pi xi)], spacing ratio (1+a)/(1-a) ~ 13
    (0.0075 D -> 0.1 D). Cross-stream: y = Ly [(eta - 1/2) - b/(4 pi) sin(4 pi (eta - 1/4))],
    clustered at |y| = 0.5 D (the nozzle lip line) with Ly = 2 D; z alike.
    A ``skew`` (fraction of the domain length) sinusoidal shear makes all nine
    metric terms non-zero.
    """
    ni, nj, nk = n
    Lx = ni * 0.0075 / (1.0 - a_x)
    Ly = Lz = 2.0
    xi = np.arange(ni + 1) / ni
    et = np.arange(nj + 1) / nj
    ze = np.arange(nk + 1) / nk
    x1 = Lx * (xi - a_x / (2 * np.pi) * np.sin(2 * np.pi * xi))
    y1 = Ly * ((et - 0.5) - b_yz / (4 * np.pi) * np.sin(4 * np.pi * (et - 0.25)))
    z1 = Lz * ((ze - 0.5) - b_yz / (4 * np.pi) * np.sin(4 * np.pi * (ze - 0.25)))
    # vertex centroids of a tensor grid with additive skew: centroid of
    # x1[i] + skew*Lx*s(eta)s(zeta) over the 8 vertices separates per axis.
    def cavg(v):
        return 0.5 * (v[:-1] + v[1:])
    def savg(w):
        s = np.sin(2 * np.pi * w)
        return 0.5 * (s[:-1] + s[1:])
    cx, cy, cz = cavg(x1), cavg(y1), cavg(z1)
    sx, sy, sz = savg(xi), savg(et), savg(ze)
    X = cx[None, None, :] + skew * Lx * (sy[None, :, None] * sz[:, None, None])
    Y = cy[None, :, None] + skew * Ly * (sz[:, None, None] * sx[None, None, :])
    Z = cz[:, None, None] + skew * Lz * (sx[None, None, :] * sy[None, :, None])
    xyz = np.empty((3, nk, nj, ni), dtype=np.float64)
    xyz[0] = X
    xyz[1] = Y
    xyz[2] = Z
    return _grid(n, 3, xyz, np.diag([Lx, Ly, Lz]))


# ----------------------------------------------------------------------------
# initial conditions (return conserved Q)
# ----------------------------------------------------------------------------
def conserved(rho, u, v, w, p, gamma=1.4, ndim=3):
    E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + (w * w if ndim == 3 else 0.0))
    if ndim == 2:
        return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, E]))
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, rho * w, E]))


def uniform_flow(grid, rho=1.0, u=1.0, v=0.0, w=0.0, p=1.0, gamma=1.4):
    shp = grid["xyz"].shape[1:]
    one = np.ones(shp)
    return conserved(rho * one, u * one, v * one, w * one, p * one, gamma, grid["ndim"])


def shu_vortex(grid, eps=5.0, xc=5.0, yc=5.0, uinf=1.0, vinf=1.0, gamma=1.4,
               rho_inf=1.0, p_inf=1.0):
    """Isentropic vortex of Shu (ICASE 97-65): du = eps/(2 pi) e^{(1-r^2)/2}(-dy),
    dv = eps/(2 pi) e^{(1-r^2)/2} dx, dT = -(gamma-1) eps^2/(8 gamma pi^2) e^{1-r^2},
    rho = T^{1/(gamma-1)}, p = rho^gamma (T = p/rho, freestream T = 1)."""
    x, y = grid["xyz"][0], grid["xyz"][1]
    dx, dy = x - xc, y - yc
    r2 = dx * dx + dy * dy
    f = np.exp(0.5 * (1.0 - r2))
    u = uinf - eps / (2 * np.pi) * f * dy
    v = vinf + eps / (2 * np.pi) * f * dx
    T = 1.0 - (gamma - 1.0) * eps * eps / (8 * gamma * np.pi ** 2) * f * f
    rho = rho_inf * T ** (1.0 / (gamma - 1.0))
    p = p_inf * T ** (gamma / (gamma - 1.0))
    w = np.zeros_like(u)
    return conserved(rho, u, v, w, p, gamma, grid["ndim"])


def jet_exit_state(Mj=1.35, Tn_over_Tinf=1.0, gamma=1.4):
    """Nozzle-exit state of a choked under-expanded jet (Eq. ini-cons of the
    paper), non-dimensionalised by ambient density and sound speed."""
    pe = (1.0 / gamma) * ((2.0 + (gamma - 1.0) * Mj * Mj) / (gamma + 1.0)) ** (gamma / (gamma - 1.0))
    rhoe = gamma * (gamma + 1.0) * pe / (2.0 * Tn_over_Tinf)
    ue = math.sqrt(2.0 * Tn_over_Tinf / (gamma + 1.0))
    return rhoe, ue, pe


def jet_ic(grid, noise=0.01, seed=3, gamma=1.4, Mj=1.35, radius=0.5, width=0.1):
    """Tanh-profile jet column along x with ambient (1, 0, 0, 0, 1/gamma) and
    seeded uniform velocity noise of +-noise*u_e."""
    rhoe, ue, pe = jet_exit_state(Mj, 1.0, gamma)
    y, z = grid["xyz"][1], grid["xyz"][2]
    r = np.sqrt(y * y + z * z)
    s = 0.5 * (1.0 + np.tanh((radius - r) / width))
    rho = 1.0 + (rhoe - 1.0) * s
    p = 1.0 / gamma + (pe - 1.0 / gamma) * s
    u = ue * s
    rng = np.random.default_rng(SEED_BASE + seed)
    shp = u.shape
    u = u + noise * ue * rng.uniform(-1, 1, shp)
    v = noise * ue * rng.uniform(-1, 1, shp)
    w = noise * ue * rng.uniform(-1, 1, shp)
    return conserved(rho, u, v, w, p, gamma, 3)


def sod_x(grid, gamma=1.4, x0=None):
    """Sod shock tube along x: (1, 0, 1) left of x0, (0.125, 0, 0.1) right."""
    x = grid["xyz"][0]
    if x0 is None:
        x0 = 0.5 * grid["off"][0][0]
    left = x < x0
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    z = np.zeros_like(x)
    return conserved(rho, z, z, z, p, gamma, grid["ndim"])


def entropy_wave(grid, amp=0.2, u=1.0, v=1.0, p=1.0, gamma=1.4):
    """rho = 1 + amp sin(2 pi (x + y)/L) with constant u, v, p (2-D)."""
    L = grid["off"][0][0]
    x, y = grid["xyz"][0], grid["xyz"][1]
    rho = 1.0 + amp * np.sin(2 * np.pi * (x + y) / L)
    one = np.ones_like(x)
    return conserved(rho, u * one, v * one, 0 * one, p * one, gamma, grid["ndim"])


def random_smooth_state(grid, seed=0, amp=0.05, gamma=1.4, modes=3):
    """Smooth seeded perturbation of a uniform state (a few random Fourier
    modes of each primitive), for parity tests."""
    rng = np.random.default_rng(SEED_BASE + 100 + seed)
    nk, nj, ni = grid["xyz"].shape[1:]
    k, j, i = np.meshgrid(np.arange(nk) / nk, np.arange(nj) / nj, np.arange(ni) / ni,
                          indexing="ij")
    base = [1.0, 0.6, -0.3, 0.2, 1.0 / gamma]
    prims = []
    for b in base:
        f = np.full(i.shape, b)
        for _ in range(modes):
            a = rng.uniform(-amp, amp)
            ki, kj, kk = rng.integers(0, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            f = f + a * np.sin(2 * np.pi * (ki * i + kj * j + kk * k) + ph)
        prims.append(f)
    rho, u, v, w, p = prims
    if grid["ndim"] == 2:
        w = np.zeros_like(u)
    return conserved(rho, u, v, w, p, gamma, grid["ndim"])


def random_rough_state(grid, seed=0, amp=0.3, gamma=1.4):
    """Cell-to-cell random (non-smooth) state, so that the limiter and both
    HLLC branches are exercised; positive density and pressure."""
    rng = np.random.default_rng(SEED_BASE + 200 + seed)
    shp = grid["xyz"].shape[1:]
    rho = 1.0 + amp * rng.uniform(-1, 1, shp)
    u = 0.5 + amp * rng.uniform(-1, 1, shp)
    v = -0.2 + amp * rng.uniform(-1, 1, shp)
    w = 0.1 + amp * rng.uniform(-1, 1, shp) if grid["ndim"] == 3 else np.zeros(shp)
    p = 1.0 + amp * rng.uniform(-1, 1, shp)
    return conserved(rho, u, v, w, p, gamma, grid["ndim"])


def supersonic_rough_state(grid, seed=0, mach=3.0, amp=0.1, gamma=1.4):
    """Streams that cross each cell face family at up to `mach` times the sound
    speed, in both directions, with cell-to-cell noise on top.

    u depends on the (j, k) index of its xi line, v on (i, k), w on (i, j), as
    a cosine of the line index: every xi line carries one sign of u, and lines
    with |cos| > 1/mach (plus the noise) are supersonic through all of their
    xi faces. Across the lines both signs occur, so both one-sided flux
    branches of HLLC (all waves moving right, all moving left) and the star
    branches near the sign changes are taken along every direction."""
    rng = np.random.default_rng(SEED_BASE + 250 + seed)
    shp = grid["xyz"].shape[1:]
    nk, nj, ni = shp
    k, j, i = np.meshgrid(np.arange(nk), np.arange(nj), np.arange(ni), indexing="ij")
    rho = 1.0 + amp * rng.uniform(-1, 1, shp)
    p = 1.0 / gamma + (amp / gamma) * rng.uniform(-1, 1, shp)
    c = np.sqrt(gamma * p / rho)
    # phases chosen so that no line sits exactly on a sign change
    u = mach * c * np.cos(2 * np.pi * (j + 0.31) / nj + 2 * np.pi * (k + 0.17) / max(nk, 2))
    v = mach * c * np.cos(2 * np.pi * (i + 0.23) / ni + 2 * np.pi * (k + 0.41) / max(nk, 2))
    w = mach * c * np.cos(2 * np.pi * (i + 0.37) / ni + 2 * np.pi * (j + 0.11) / nj)
    u = u + amp * c * rng.uniform(-1, 1, shp)
    v = v + amp * c * rng.uniform(-1, 1, shp)
    w = (w + amp * c * rng.uniform(-1, 1, shp)) if grid["ndim"] == 3 else np.zeros(shp)
    return conserved(rho, u, v, w, p, gamma, grid["ndim"])


def vortex_sod(grid, eps=2.0, xc=None, yc=None, gamma=1.4):
    """Sod-type (rho, p) = (1, 1) | (0.125, 0.1) split at x = L/2 (periodic, so
    a second jump sits at the seam), with an isentropic vortex of strength eps
    superposed: vortex velocities and the vortex's isentropic density and
    pressure factors on top of the Sod state. Cells whose centre lies on the
    split (within 1e-9 L; odd N puts a whole column there) take the right
    state, so round-off in the coordinates cannot make that column zigzag."""
    L = grid["off"][0][0]
    xc = 0.5 * L if xc is None else xc
    yc = 0.5 * grid["off"][1][1] if yc is None else yc
    x, y = grid["xyz"][0], grid["xyz"][1]
    dx, dy = x - xc, y - yc
    f = np.exp(0.5 * (1.0 - (dx * dx + dy * dy)))
    u = -eps / (2 * np.pi) * f * dy
    v = eps / (2 * np.pi) * f * dx
    T = 1.0 - (gamma - 1.0) * eps * eps / (8 * gamma * np.pi ** 2) * f * f
    left = x < 0.5 * L - 1e-9 * L
    rho = np.where(left, 1.0, 0.125) * T ** (1.0 / (gamma - 1.0))
    p = np.where(left, 1.0, 0.1) * T ** (gamma / (gamma - 1.0))
    return conserved(rho, u, v, np.zeros_like(u), p, gamma, grid["ndim"])


def batch2d(count=256, seed=4, log2_min=5.0, log2_max=9.0, L=10.0):
    """Many-small-grids workload: ``count`` square periodic wavy grids with
    N = round(2^U(log2_min, log2_max)) cells per side and mapping amplitude
    U(0.02, 0.1) (fraction of L); even-numbered draws carry a Shu vortex
    (eps 5 at the centre, freestream (1, 1, 1, 1)), odd ones the Sod-type
    state with an eps = 2 vortex. Returns a list of (grid, Q, kind)."""
    rng = np.random.default_rng(SEED_BASE + seed)
    out = []
    for b in range(count):
        n = int(round(2.0 ** rng.uniform(log2_min, log2_max)))
        amp = float(rng.uniform(0.02, 0.1))
        vortex = rng.uniform() < 0.5
        g = wavy2d((n, n), L=L, amp=amp)
        if vortex:
            Q = shu_vortex(g, eps=5.0, xc=0.5 * L, yc=0.5 * L)
        else:
            Q = vortex_sod(g)
        out.append((g, Q, "vortex" if vortex else "sod"))
    return out


# ----------------------------------------------------------------------------
# non-periodic boundaries
# ----------------------------------------------------------------------------
NG = 6  # ghost layers on each non-periodic side


def bounded(grid, bc):
    """A copy of ``grid`` with boundary types ``bc`` (per direction a pair
    (low, high); both "periodic" or both non-periodic). Along a non-periodic
    direction the first and last NG cells are ghost cells: their
    coordinates are ignored and their states are set from the boundary type
    (an "inflow" ghost keeps the state stored in it)."""
    g = dict(grid)
    bc = [tuple(b) for b in bc] + [("periodic", "periodic")] * (3 - len(bc))
    for d, (lo, hi) in enumerate(bc):
        if (lo == "periodic") != (hi == "periodic"):
            raise ValueError("a direction is periodic on both sides or on neither")
        if lo != "periodic" and (d >= grid["ndim"] or grid["n"][d] - 2 * NG < 12):
            raise ValueError("a non-periodic direction needs at least 12 interior cells")
    g["bc"] = bc
    return g


def sponge_sigma(grid, width=10, amp=2.0, power=2.0, sides=None):
    """Sponge strength per cell [nk][nj][ni]: amp * (s / width) ** power in
    the ``width`` interior cells next to each listed non-periodic side (s =
    1 .. width, counted from the innermost cell of the layer), zero elsewhere
    and in ghost cells (the profile shape follows Bodony's layers; only its
    values enter the solver). ``sides``: (direction, side) pairs, default
    every non-periodic side."""
    nk, nj, ni = grid["xyz"].shape[1:]
    bc = grid.get("bc") or []
    if sides is None:
        sides = [(d, s) for d in range(len(bc)) for s in range(2) if bc[d][0] != "periodic"]
    sig = np.zeros((nk, nj, ni))
    idx = np.meshgrid(np.arange(nk), np.arange(nj), np.arange(ni), indexing="ij")
    for d, side in sides:
        pos = idx[2 - d]
        n = grid["n"][d]
        depth = (pos - NG) if side == 0 else (n - NG - 1 - pos)  # 0 at the boundary cell
        s = width - depth
        prof = np.where((depth >= 0) & (s > 0), amp * (np.clip(s, 0, None) / width) ** power, 0.0)
        sig = np.maximum(sig, prof)
    return sig

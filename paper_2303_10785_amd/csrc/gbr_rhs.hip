// Right-hand-side kernels (Sec. 3, Sec. 5.1 Steps 1-7, Sec. 5.2 Steps 1-5),
// SSP-RK3 stage (App. B) and time step (App. B).
//
// One RHS evaluation is 1 + ndim launches:
//   k_cell_grad   : per cell, primitives of the 3 x 6 stencil neighbours, E6
//                   gradients of (u, v, w, T) along xi, eta, zeta (stored for
//                   the tangential viscous terms) and the Ducros sensor.
//   k_sweep<D>    : per direction D, a tile of interfaces along D: primitive
//                   pencils staged in LDS with a 6-cell halo, E6 first and
//                   Hermite second derivatives computed once per cell in LDS,
//                   then one thread per interface forms the characteristic
//                   (or direct) L/R states, the MP limiter, HLLC and the
//                   alpha-damping viscous flux; the interface fluxes go back
//                   to LDS and each cell accumulates -(Phi(+1/2) - Phi(-1/2))
//                   into Res (written by the xi sweep, updated by the others).
// Tiles along D overlap by one interface, so no cell needs a flux computed by
// another workgroup.
#include "gbr_device.hpp"
#include "gbr_internal.hpp"

namespace gbr {
namespace {

constexpr int kBlock = 256;

struct RhsArgs {
    Dims dm;
    Phys ph;
    const double *Q;
    double *res;
    double *grad;          // 12 * ncell: (d * 4 + s), s = u, v, w, T
    double *theta;         // ncell
    const double *m;       // metrics
    int *flags;
};

__device__ __forceinline__ long pack(const Dims &dm, int i, int j, int k)
{
    return i + (long)dm.n[0] * (j + (long)dm.n[1] * k);
}

// ----------------------------------------------------------------------------
// cell gradients and sensor
// ----------------------------------------------------------------------------
template <int NDIM>
__device__ __forceinline__ void load_prim(const RhsArgs &a, long c, double &r, double &u, double &v,
                                          double &w, double &p)
{
    const long N = a.dm.ncell;
    r = a.Q[c];
    double ir = 1.0 / r;
    u = a.Q[N + c] * ir;
    v = a.Q[2 * N + c] * ir;
    w = (NDIM == 3) ? a.Q[3 * N + c] * ir : 0.0;
    double E = a.Q[(NDIM + 1) * N + c];
    p = a.ph.gm1 * (E - 0.5 * r * (u * u + v * v + w * w));
}

template <int NDIM, bool SENSOR>
__global__ void __launch_bounds__(kBlock) k_cell_grad(RhsArgs a)
{
    long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx >= a.dm.ncell) return;
    const long N = a.dm.ncell;
    int ijk[3];
    ijk[0] = int(idx % a.dm.n[0]);
    ijk[1] = int((idx / a.dm.n[0]) % a.dm.n[1]);
    ijk[2] = int(idx / ((long)a.dm.n[0] * a.dm.n[1]));
    {
        double r, u, v, w, p;
        load_prim<NDIM>(a, idx, r, u, v, w, p);
        if (!(r > 0.0 && p > 0.0 && isfinite(r) && isfinite(p) && isfinite(u) && isfinite(v) &&
              isfinite(w)))
            atomicOr(a.flags, 1);
    }
    double gd[3][4];
    for (int d = 0; d < 3; ++d) {
        if (d >= NDIM) {
            for (int s = 0; s < 4; ++s) gd[d][s] = 0.0;
            continue;
        }
        double su[7], sv[7], sw[7], sT[7];
        for (int q = -3; q <= 3; ++q) {
            int t[3] = {ijk[0], ijk[1], ijk[2]};
            t[d] = wrap_index(t[d] + q, a.dm.n[d]);
            double r, u, v, w, p;
            load_prim<NDIM>(a, pack(a.dm, t[0], t[1], t[2]), r, u, v, w, p);
            su[q + 3] = u;
            sv[q + 3] = v;
            sw[q + 3] = w;
            sT[q + 3] = a.ph.gM2 * p / r;
        }
        gd[d][0] = e6(su[0], su[1], su[2], su[4], su[5], su[6]);
        gd[d][1] = e6(sv[0], sv[1], sv[2], sv[4], sv[5], sv[6]);
        gd[d][2] = e6(sw[0], sw[1], sw[2], sw[4], sw[5], sw[6]);
        gd[d][3] = e6(sT[0], sT[1], sT[2], sT[4], sT[5], sT[6]);
    }
    for (int d = 0; d < 3; ++d)
        for (int s = 0; s < 4; ++s) a.grad[(d * 4 + s) * N + idx] = gd[d][s];
    if (SENSOR) {
        // physical velocity gradient G[a][b] = sum_d (d_{x_b}) du_a/dd
        double G[3][3];
        for (int aa = 0; aa < 3; ++aa)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int d = 0; d < 3; ++d) s += a.m[GBR_SLOT_CELL_UNHAT(d, b) * N + idx] * gd[d][aa];
                G[aa][b] = s;
            }
        double div = G[0][0] + G[1][1] + G[2][2];
        double wx = G[2][1] - G[1][2], wy = G[0][2] - G[2][0], wz = G[1][0] - G[0][1];
        double d2 = div * div;
        a.theta[idx] = d2 / (d2 + (wx * wx + wy * wy + wz * wz) + 1e-30);
    }
}

// ----------------------------------------------------------------------------
// per-direction interface sweep
// ----------------------------------------------------------------------------
template <int D>
struct Tile {
    // faces per tile along D, lanes across, and index roles:
    // s = sweep direction D, c = cross direction, o = outer direction.
    static constexpr int TS = (D == 0) ? 64 : 16;
    static constexpr int TC = kBlock / TS;
    static constexpr int SD = D;
    static constexpr int CD = (D == 0) ? 1 : 0;
    static constexpr int OD = (D == 2) ? 1 : 2;
    static constexpr int NP = TS + 11;  // primitive cells s0-6 .. s0+TS+4
    static constexpr int N1 = TS + 5;   // first derivatives s0-3 .. s0+TS+1
    static constexpr int N2 = TS + 3;   // second derivatives s0-2 .. s0+TS
    // LDS offset of (s, c) in an array with ns entries along s: s fastest for
    // the xi sweep (lanes run along s), c fastest otherwise (lanes run along c).
    __device__ static constexpr int at(int s, int c, int ns) { return D == 0 ? c * ns + s : s * TC + c; }
};

__device__ __forceinline__ long cell_of(const Dims &dm, int sd, int cd, int s, int c, int o)
{
    int t[3];
    t[sd] = s;
    t[cd] = c;
    t[3 - sd - cd] = o;
    return pack(dm, t[0], t[1], t[2]);
}

// Interface flux Phi = F - F^v for the interface between cells a and a+1
// along D. p* point to the LDS values of the primitives (offsets -1..2 about
// a), first derivatives (0, 1) and second derivatives (-1..2); st is the LDS
// stride between consecutive cells along D.
template <int D, int NDIM, bool VISC>
__device__ __forceinline__ bool interface_flux(const RhsArgs &a, const double *sP, const double *s1,
                                               const double *s2, int vstrideP, int vstride1,
                                               int vstride2, int st, long ca, long cb, double phi[5])
{
    const long N = a.dm.ncell;
    const Phys &ph = a.ph;
    const double *m = a.m;
    double nt = m[GBR_SLOT_FACE_HATT(D) * N + ca];
    double nx = m[GBR_SLOT_FACE_HAT(D, 0) * N + ca];
    double ny = m[GBR_SLOT_FACE_HAT(D, 1) * N + ca];
    double nz = (NDIM == 3) ? m[GBR_SLOT_FACE_HAT(D, 2) * N + ca] : 0.0;

    // cell values: P[q][v] at offsets q = -1..2 (index q + 1)
    double P[4][5], P2[4][5], P1[2][5];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            P[q][v] = sP[v * vstrideP + (q - 1) * st];
            P2[q][v] = s2[v * vstride2 + (q - 1) * st];
        }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 5; ++v) P1[q][v] = s1[v * vstride1 + q * st];

    bool limited = ph.limiter == GBR_LIM_MP;
    if (ph.limiter == GBR_LIM_DUCROS) limited = fmax(a.theta[ca], a.theta[cb]) > ph.theta_c;

    double PL[5], PR[5];
    if (limited) {
        // Step-2: left eigenvectors of the averaged state (App. A) with the
        // unit interface normal; the projection of a primitive vector is
        //   W0 = p - ra (n.u),  W4 = p + ra (n.u),
        //   (W1, W2, W3) = (n_x s + (n x u)_x, n_z s + (n x u)_z, -n_y s - (n x u)_y),
        // with s = a^2 rho - p.
        double rb = 0.5 * (P[1][0] + P[2][0]);
        double pb = 0.5 * (P[1][4] + P[2][4]);
        double ab2 = ph.gamma * pb / rb;
        double ab = sqrt(ab2);
        double ra = rb * ab;
        double inn = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
        double ex = nx * inn, ey = ny * inn, ez = nz * inn;
        auto project = [&](const double *x, double W[5]) {
            double un = ex * x[1] + ey * x[2] + ez * x[3];
            double s = ab2 * x[0] - x[4];
            double cx = ey * x[3] - ez * x[2];
            double cy = ez * x[1] - ex * x[3];
            double cz = ex * x[2] - ey * x[1];
            W[0] = x[4] - ra * un;
            W[1] = ex * s + cx;
            W[2] = ez * s + cz;
            W[3] = -ey * s - cy;
            W[4] = x[4] + ra * un;
        };
        double W[4][5], W2[4][5], W1[2][5];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            project(P[q], W[q]);
            project(P2[q], W2[q]);
        }
        project(P1[0], W1[0]);
        project(P1[1], W1[1]);
        // Step-3 and Step-4 per characteristic field
        double WL[5], WR[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            double wl = W[1][v] + 0.5 * W1[0][v] + W2[1][v] / 12.0;
            double wr = W[2][v] - 0.5 * W1[1][v] + W2[2][v] / 12.0;
            WL[v] = mp_limit(W[0][v], W[1][v], W[2][v], W2[0][v], W2[1][v], W2[2][v], wl,
                             ph.alpha_mp, ph.beta_mp);
            WR[v] = mp_limit(W[3][v], W[2][v], W[1][v], W2[3][v], W2[2][v], W2[1][v], wr,
                             ph.alpha_mp, ph.beta_mp);
        }
        // Step-5: right eigenvectors (App. A)
        auto back = [&](const double *w, double *x) {
            double ia2 = 1.0 / ab2;
            double h = (w[4] - w[0]) / (2.0 * ra);
            x[0] = 0.5 * (w[0] + w[4]) * ia2 + (ex * w[1] + ez * w[2] - ey * w[3]) * ia2;
            x[1] = ex * h - ey * w[2] - ez * w[3];
            x[2] = ey * h - ez * w[1] + ex * w[2];
            x[3] = ez * h + ey * w[1] + ex * w[3];
            x[4] = 0.5 * (w[0] + w[4]);
        };
        back(WL, PL);
        back(WR, PR);
    } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            PL[v] = P[1][v] + 0.5 * P1[0][v] + P2[1][v] / 12.0;
            PR[v] = P[2][v] - 0.5 * P1[1][v] + P2[2][v] / 12.0;
        }
    }
    if (NDIM == 2) {
        PL[3] = 0.0;
        PR[3] = 0.0;
    }
    bool ok = PL[0] > 0.0 && PL[4] > 0.0 && PR[0] > 0.0 && PR[4] > 0.0;

    // Step-6: HLLC
    hllc(PL, PR, nt, nx, ny, nz, ph.gamma, ph.gm1, phi);

    if (VISC) {
        // Sec. 5.2 Step-1: interface gradients of (u, v, w, T) along each
        // computational direction; normal one from Eq. AD-eqn1, tangential
        // ones from the average of the two cell gradients.
        const double *gr = a.grad;
        double c0[4] = {P[1][1], P[1][2], P[1][3], ph.gM2 * P[1][4] / P[1][0]};
        double c1[4] = {P[2][1], P[2][2], P[2][3], ph.gM2 * P[2][4] / P[2][0]};
        double g0[4] = {P1[0][1], P1[0][2], P1[0][3], gr[(D * 4 + 3) * N + ca]};
        double g1[4] = {P1[1][1], P1[1][2], P1[1][3], gr[(D * 4 + 3) * N + cb]};
        double sL[4], sR[4], gf[3][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            sL[s] = c0[s] + 0.5 * g0[s];
            sR[s] = c1[s] - 0.5 * g1[s];
            gf[D][s] = 0.5 * (g0[s] + g1[s]) + 0.5 * ph.alpha_d * (sR[s] - sL[s]);
        }
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if (e == D) continue;
#pragma unroll
            for (int s = 0; s < 4; ++s)
                gf[e][s] = (e < NDIM) ? 0.5 * (gr[(e * 4 + s) * N + ca] + gr[(e * 4 + s) * N + cb]) : 0.0;
        }
        // Step-2: chain rule with the interface unhatted metrics
        double Dx[4][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
#pragma unroll
                for (int e = 0; e < NDIM; ++e)
                    if (b < NDIM) acc += m[GBR_SLOT_FACE_UNHAT(D, e, b) * N + ca] * gf[e][s];
                Dx[s][b] = acc;
            }
        // Step-3: stresses and heat flux
        double Tf = 0.5 * (sL[3] + sR[3]);
        double mu = viscosity(Tf, ph.suth, ph.inv_re);
        double lam = -2.0 / 3.0 * mu;
        double kap = mu * ph.kfac;
        double uf = 0.5 * (sL[0] + sR[0]), vf = 0.5 * (sL[1] + sR[1]), wf = 0.5 * (sL[2] + sR[2]);
        double div = Dx[0][0] + Dx[1][1] + Dx[2][2];
        double txx = 2.0 * mu * Dx[0][0] + lam * div;
        double tyy = 2.0 * mu * Dx[1][1] + lam * div;
        double tzz = 2.0 * mu * Dx[2][2] + lam * div;
        double txy = mu * (Dx[0][1] + Dx[1][0]);
        double txz = mu * (Dx[0][2] + Dx[2][0]);
        double tyz = mu * (Dx[1][2] + Dx[2][1]);
        double bx = uf * txx + vf * txy + wf * txz + kap * Dx[3][0];
        double by = uf * txy + vf * tyy + wf * tyz + kap * Dx[3][1];
        double bz = uf * txz + vf * tyz + wf * tzz + kap * Dx[3][2];
        // Step-4: viscous interface flux with hatted interface metrics
        phi[1] -= nx * txx + ny * txy + nz * txz;
        phi[2] -= nx * txy + ny * tyy + nz * tyz;
        phi[3] -= nx * txz + ny * tyz + nz * tzz;
        phi[4] -= nx * bx + ny * by + nz * bz;
    }
    ok = ok && isfinite(phi[0]) && isfinite(phi[4]);
    return ok;
}

template <int D, int NDIM, bool VISC, bool FIRST>
__global__ void __launch_bounds__(kBlock) k_sweep(RhsArgs a)
{
    using T = Tile<D>;
    constexpr int TS = T::TS, TC = T::TC, NP = T::NP, N1 = T::N1, N2 = T::N2;
    __shared__ double sP[5 * NP * TC];
    __shared__ double s1[5 * N1 * TC];
    __shared__ double s2[5 * N2 * TC];

    const Dims &dm = a.dm;
    const long N = dm.ncell;
    const int ns = dm.n[T::SD], nc = dm.n[T::CD];
    const int tiles_s = (ns + TS - 2) / (TS - 1);
    const int ts = blockIdx.x % tiles_s;
    const int tcb = blockIdx.x / tiles_s;
    const int s0 = ts * (TS - 1);
    const int c0 = tcb * TC;
    const int o = blockIdx.y;
    const int tid = threadIdx.x;

    // Phase 1: primitives of cells s0-6 .. s0+TS+4 into LDS
    for (int e = tid; e < NP * TC; e += kBlock) {
        int sl = (D == 0) ? e % NP : e / TC;
        int cl = (D == 0) ? e / NP : e % TC;
        int sg = wrap_index(s0 - 6 + sl, ns);
        int cg = min(c0 + cl, nc - 1);
        double r, u, v, w, p;
        load_prim<NDIM>(a, cell_of(dm, T::SD, T::CD, sg, cg, o), r, u, v, w, p);
        int at = T::at(sl, cl, NP);
        sP[0 * NP * TC + at] = r;
        sP[1 * NP * TC + at] = u;
        sP[2 * NP * TC + at] = v;
        sP[3 * NP * TC + at] = w;
        sP[4 * NP * TC + at] = p;
    }
    __syncthreads();
    // Phase 2: E6 first derivatives of cells s0-3 .. s0+TS+1
    constexpr int stP = (D == 0) ? 1 : TC;
    for (int e = tid; e < N1 * TC; e += kBlock) {
        int sl = (D == 0) ? e % N1 : e / TC;
        int cl = (D == 0) ? e / N1 : e % TC;
        int pc = T::at(sl + 3, cl, NP);
        int at = T::at(sl, cl, N1);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double *x = sP + v * NP * TC + pc;
            s1[v * N1 * TC + at] = e6(x[-3 * stP], x[-2 * stP], x[-stP], x[stP], x[2 * stP], x[3 * stP]);
        }
    }
    __syncthreads();
    // Phase 3: Hermite second derivatives of cells s0-2 .. s0+TS
    for (int e = tid; e < N2 * TC; e += kBlock) {
        int sl = (D == 0) ? e % N2 : e / TC;
        int cl = (D == 0) ? e / N2 : e % TC;
        int pc = T::at(sl + 4, cl, NP);
        int dc = T::at(sl + 1, cl, N1);
        int at = T::at(sl, cl, N2);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            const double *x = sP + v * NP * TC + pc;
            const double *g = s1 + v * N1 * TC + dc;
            s2[v * N2 * TC + at] = hermite2(x[-stP], x[0], x[stP], g[-stP], g[stP]);
        }
    }
    __syncthreads();
    // Phase 4: one interface per thread: between cells s0+t-1 and s0+t
    const int t = (D == 0) ? tid % TS : tid / TC;
    const int cl = (D == 0) ? tid / TS : tid % TC;
    const int cg = c0 + cl;
    const int cgc = min(cg, nc - 1);
    const long ca = cell_of(dm, T::SD, T::CD, wrap_index(s0 + t - 1, ns), cgc, o);
    const long cb = cell_of(dm, T::SD, T::CD, wrap_index(s0 + t, ns), cgc, o);
    double phi[5];
    bool ok = interface_flux<D, NDIM, VISC>(a, sP + T::at(t + 5, cl, NP), s1 + T::at(t + 2, cl, N1),
                                             s2 + T::at(t + 1, cl, N2), NP * TC, N1 * TC, N2 * TC,
                                             stP, ca, cb, phi);
    if (!ok && cg < nc) atomicOr(a.flags, 1);
    __syncthreads();
    // interface fluxes back to LDS (reusing the primitive buffer)
#pragma unroll
    for (int v = 0; v < 5; ++v) sP[v * TS * TC + T::at(t, cl, TS)] = phi[v];
    __syncthreads();
    // Phase 5: Res of cell s0+t from its two interfaces
    if (t < TS - 1 && s0 + t < ns && cg < nc) {
        const long cc = cb;
        const int nv = NDIM + 2;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            if (NDIM == 2 && v == 3) continue;
            int ov = (NDIM == 2 && v == 4) ? 3 : v;
            double d = sP[v * TS * TC + T::at(t + 1, cl, TS)] - sP[v * TS * TC + T::at(t, cl, TS)];
            double *r = a.res + (long)ov * N + cc;
            if (FIRST)
                *r = -d;
            else
                *r = *r - d;
        }
        (void)nv;
    }
}

// ----------------------------------------------------------------------------
// SSP-RK3 stage and time step
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_rk_stage(long n, long ncell, double ca, double cb,
                                                       const double *__restrict__ dtp,
                                                       const double *__restrict__ Qn,
                                                       double *__restrict__ Q,
                                                       const double *__restrict__ res,
                                                       const double *__restrict__ jac,
                                                       const double *__restrict__ invjt)
{
    long e = blockIdx.x * (long)kBlock + threadIdx.x;
    if (e >= n) return;
    long c = e % ncell;
    double dt = *dtp;
    double q = Q[e];
    double L = jac[c] * (res[e] - invjt[c] * q);
    Q[e] = ca * Qn[e] + cb * (q + dt * L);
}

template <int NDIM, bool VISC>
__global__ void __launch_bounds__(kBlock) k_cfl(RhsArgs a, unsigned long long *out)
{
    long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    const long N = a.dm.ncell;
    double best = __builtin_inf(), bestv = __builtin_inf();
    if (idx < N) {
        double r, u, v, w, p;
        load_prim<NDIM>(a, idx, r, u, v, w, p);
        double c = sqrt(a.ph.gamma * p / r);
        double nu = VISC ? viscosity(a.ph.gM2 * p / r, a.ph.suth, a.ph.inv_re) / r : 0.0;
        for (int d = 0; d < NDIM; ++d) {
            double dx = a.m[GBR_SLOT_CELL_UNHAT(d, 0) * N + idx];
            double dy = a.m[GBR_SLOT_CELL_UNHAT(d, 1) * N + idx];
            double dz = a.m[GBR_SLOT_CELL_UNHAT(d, 2) * N + idx];
            double U = a.m[GBR_SLOT_CELL_UNHATT(d) * N + idx] + dx * u + dy * v + dz * w;
            double g2 = dx * dx + dy * dy + dz * dz;
            best = fmin(best, 1.0 / (fabs(U) + c * sqrt(g2)));
            if (VISC) bestv = fmin(bestv, 1.0 / (nu * g2));
        }
        if (VISC) best = fmin(best, bestv / a.ph.alpha_d);
    }
    // wavefront minimum, then one atomic per wavefront (positive doubles
    // order like their bit patterns)
    for (int off = warpSize / 2; off > 0; off >>= 1) best = fmin(best, __shfl_xor(best, off));
    if ((threadIdx.x & (warpSize - 1)) == 0 && best < __builtin_inf())
        atomicMin(out, (unsigned long long)__double_as_longlong(best));
}

__global__ void k_dt_finish(const unsigned long long *minbits, double cfl, double *dt)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) dt[0] = cfl * __longlong_as_double((long long)*minbits);
}

__global__ void k_set_word(unsigned long long *p, unsigned long long v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void __launch_bounds__(kBlock) k_fill(double *p, long n, double v)
{
    long e = blockIdx.x * (long)kBlock + threadIdx.x;
    if (e < n) p[e] = v;
}

__global__ void __launch_bounds__(kBlock) k_copy(double *__restrict__ d, const double *__restrict__ s, long n)
{
    long e = blockIdx.x * (long)kBlock + threadIdx.x;
    if (e < n) d[e] = s[e];
}

template <int D, int NDIM, bool VISC>
hipError_t sweep(gbr_grid_s *g, const RhsArgs &a)
{
    using T = Tile<D>;
    hipStream_t st = g->stream;
    Timed timed(g, GBR_K_SWEEP_XI + D);
    const int ns = a.dm.n[T::SD], nc = a.dm.n[T::CD], no = a.dm.n[T::OD];
    const int tiles_s = (ns + T::TS - 2) / (T::TS - 1);
    const int tiles_c = (nc + T::TC - 1) / T::TC;
    dim3 grid(unsigned(tiles_s * tiles_c), unsigned(no));
    if (D == 0)
        hipLaunchKernelGGL((k_sweep<D, NDIM, VISC, true>), grid, dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL((k_sweep<D, NDIM, VISC, false>), grid, dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

template <int NDIM, bool VISC>
hipError_t rhs_all(gbr_grid_s *g, const RhsArgs &a)
{
    unsigned blocks = unsigned((a.dm.ncell + kBlock - 1) / kBlock);
    hipError_t e;
    {
        Timed timed(g, GBR_K_CELL_GRAD);
        if (a.ph.limiter == GBR_LIM_DUCROS)
            hipLaunchKernelGGL((k_cell_grad<NDIM, true>), dim3(blocks), dim3(kBlock), 0, g->stream, a);
        else
            hipLaunchKernelGGL((k_cell_grad<NDIM, false>), dim3(blocks), dim3(kBlock), 0, g->stream, a);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    if ((e = sweep<0, NDIM, VISC>(g, a)) != hipSuccess) return e;
    if ((e = sweep<1, NDIM, VISC>(g, a)) != hipSuccess) return e;
    if (NDIM == 3) e = sweep<NDIM == 3 ? 2 : 1, NDIM, VISC>(g, a);
    return e;
}

RhsArgs make_args(gbr_grid_s *g, const double *Q, double *res)
{
    RhsArgs a;
    a.dm = dims_of(g);
    a.ph = phys_of(g);
    a.Q = Q;
    a.res = res;
    a.grad = g->scratch;
    a.theta = g->theta;
    a.m = g->metrics;
    a.flags = g->flags;
    return a;
}

}  // namespace

hipError_t launch_rhs(gbr_grid_s *g, const double *Q, double *res)
{
    RhsArgs a = make_args(g, Q, res);
    const bool visc = g->cfg.viscous != 0;
    if (g->cfg.ndim == 3)
        return visc ? rhs_all<3, true>(g, a) : rhs_all<3, false>(g, a);
    return visc ? rhs_all<2, true>(g, a) : rhs_all<2, false>(g, a);
}

hipError_t launch_rk_stage(gbr_grid_s *g, int stage, const double *dt, const double *Qn, double *Q,
                           const double *res)
{
    static const double A[3] = {0.0, 0.75, 1.0 / 3.0};
    static const double B[3] = {1.0, 0.25, 2.0 / 3.0};
    long n = (long)g->nvar * g->ncell;
    unsigned blocks = unsigned((n + kBlock - 1) / kBlock);
    Timed timed(g, GBR_K_RK_STAGE);
    hipLaunchKernelGGL(k_rk_stage, dim3(blocks), dim3(kBlock), 0, g->stream, n, g->ncell, A[stage],
                       B[stage], dt, Qn, Q, res, g->metrics + (long)GBR_SLOT_CELL_J * g->ncell,
                       g->metrics + (long)GBR_SLOT_CELL_INVJT * g->ncell);
    return hipGetLastError();
}

hipError_t launch_cfl(gbr_grid_s *g, const double *Q, double cfl, double *dt)
{
    RhsArgs a = make_args(g, Q, nullptr);
    unsigned blocks = unsigned((g->ncell + kBlock - 1) / kBlock);
    Timed timed(g, GBR_K_CFL);
    hipLaunchKernelGGL(k_set_word, dim3(1), dim3(1), 0, g->stream, g->dtmin, ~0ull >> 1);
    const bool visc = g->cfg.viscous != 0;
    if (g->cfg.ndim == 3) {
        if (visc)
            hipLaunchKernelGGL((k_cfl<3, true>), dim3(blocks), dim3(kBlock), 0, g->stream, a, g->dtmin);
        else
            hipLaunchKernelGGL((k_cfl<3, false>), dim3(blocks), dim3(kBlock), 0, g->stream, a, g->dtmin);
    } else {
        if (visc)
            hipLaunchKernelGGL((k_cfl<2, true>), dim3(blocks), dim3(kBlock), 0, g->stream, a, g->dtmin);
        else
            hipLaunchKernelGGL((k_cfl<2, false>), dim3(blocks), dim3(kBlock), 0, g->stream, a, g->dtmin);
    }
    hipLaunchKernelGGL(k_dt_finish, dim3(1), dim3(1), 0, g->stream, g->dtmin, cfl, dt);
    return hipGetLastError();
}

hipError_t launch_fill(gbr_grid_s *g, double *p, long n, double value)
{
    unsigned blocks = unsigned((n + kBlock - 1) / kBlock);
    Timed timed(g, GBR_K_COPY);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(kBlock), 0, g->stream, p, n, value);
    return hipGetLastError();
}

hipError_t launch_copy(gbr_grid_s *g, double *dst, const double *src, long n)
{
    unsigned blocks = unsigned((n + kBlock - 1) / kBlock);
    Timed timed(g, GBR_K_COPY);
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(kBlock), 0, g->stream, dst, src, n);
    return hipGetLastError();
}

}  // namespace gbr

// Device-side building blocks of the gradient-based-reconstruction RHS.
// Each function states the passage of the paper it evaluates.
#pragma once

#include <hip/hip_runtime.h>

#include "gbr.h"

namespace gbr {

// Periodic index: a in any range, n >= 1.
__device__ __forceinline__ int wrap_index(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

// wrap_index for indices that leave [0, n) only when `edge` is set; tiles
// away from the ends of their lines (edge false, uniform across a
// workgroup) skip the modulo.
__device__ __forceinline__ int wrap_if(bool edge, int a, int n) { return edge ? wrap_index(a, n) : a; }

// Division and square root in the compute type of the flux kernels:
// correctly rounded in double; in float (the FP32-bulk path) the hardware
// reciprocal and square root, within about one unit in the last place,
// far inside that path's error bound.
__device__ __forceinline__ double cdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float cdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double csqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float csqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Number of periods crossed going from [0, n) to index a (floor(a / n)).
__device__ __forceinline__ int wrap_count(int a, int n)
{
    int r = a % n;
    if (r < 0) r += n;
    return (a - r) / n;
}

// Position of the periodic image x + wr * off relative to org, with one
// rounding of the small result: the metrics are invariant under a translation
// (Sec. 4.2), so every window is measured from its target cell, but the image
// x + wr * off of a cell across the seam is not representable in general and,
// rounded first, would carry an error of eps |x| that the metrics divide by
// the spacing. The product and the sum are split into exact value and error
// pairs (the product error from a fused multiply-add, the sum error from
// Knuth's two-sum), the leading part minus org is exact when the image lies
// near org, and the error terms are added last. No contraction may merge
// these operations. With wr = 0 every error term is zero and the result is
// x - org exactly, so the function serves whole windows without a branch.
__device__ __forceinline__ double image_rel(double x, int wr, double off, double org)
{
#pragma clang fp contract(off)
    const double w = double(wr);
    const double p = w * off;
    const double pe = __builtin_fma(w, off, -p);
    const double s = x + p;
    const double bp = s - x;
    const double se = (x - (s - bp)) + (p - bp);
    return (s - org) + (se + pe);
}

// Composite central derivative of Sec. 7: the difference of two interface
// values of the averaged van Leer states built on E6 gradients and Hermite
// second derivatives, which collapses to sum_m c_m (v[+m] - v[-m]) with
// c = (2282, -546, 89, -3, -1) / 2880. v points at the centre of v[-5..5].
__device__ __forceinline__ double dcomp(const double *v)
{
    constexpr double c1 = 2282.0 / 2880.0, c2 = -546.0 / 2880.0, c3 = 89.0 / 2880.0,
                     c4 = -3.0 / 2880.0, c5 = -1.0 / 2880.0;
    return c1 * (v[1] - v[-1]) + c2 * (v[2] - v[-2]) + c3 * (v[3] - v[-3]) +
           c4 * (v[4] - v[-4]) + c5 * (v[5] - v[-5]);
}

// Central interface value at +1/2 (Eq. interp-formulae): the average of the
// unlimited left and right states of Eq. vanleer-poly with E6 / Hermite
// derivatives, as a 10-point stencil over v[-4..5] with weights
// (-2, -8, 170, -922, 3642, 3642, -922, 170, -8, -2) / 5760.
__device__ __forceinline__ double face_interp(const double *v)
{
    constexpr double w1 = 3642.0 / 5760.0, w2 = -922.0 / 5760.0, w3 = 170.0 / 5760.0,
                     w4 = -8.0 / 5760.0, w5 = -2.0 / 5760.0;
    return w1 * (v[0] + v[1]) + w2 * (v[-1] + v[2]) + w3 * (v[-2] + v[3]) +
           w4 * (v[-3] + v[4]) + w5 * (v[-4] + v[5]);
}

// The RHS arithmetic below is templated on the compute type R: double for
// the FP64 path, float for the FP32-bulk path.

// E6 first derivative (Eq. E6_grads, as differences) from the six neighbours.
template <class R>
__device__ __forceinline__ R e6(R m3, R m2, R m1, R p1, R p2, R p3)
{
    return R(0.75) * (p1 - m1) - R(0.15) * (p2 - m2) + R(1.0 / 60.0) * (p3 - m3);
}

// Hermite second derivative (Step-1 of Sec. 5.1).
template <class R>
__device__ __forceinline__ R hermite2(R vm, R v0, R vp, R gm, R gp)
{
    return R(2) * (vp - R(2) * v0 + vm) - R(0.5) * (gp - gm);
}

// minmod(a, b) = 0.5 (sign a + sign b) min(|a|, |b|) with sign(0) = 0, which
// is the median of a, b and 0 (the smaller magnitude when the signs agree,
// else zero): one med3 instruction in float, two min / max pairs in double.
__device__ __forceinline__ float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ __forceinline__ double minmod(double a, double b) { return fmax(fmin(a, b), fmin(fmax(a, b), 0.0)); }

// Improved MP limiter of App. E for one characteristic component at the left
// state of an interface: wm1, w0, wp1 are the cell values upwind, at and
// downwind of the reconstructing cell, dm1, d0, dp1 their gradient-based
// curvatures, wf the unlimited interface value. The right state is the same
// procedure on the stencil reflected about its own cell.
template <class R>
__device__ __forceinline__ R mp_limit(R wm1, R w0, R wp1, R dm1, R d0, R dp1, R wf, R alpha, R beta)
{
    R wmp = w0 + minmod(wp1 - w0, beta * (w0 - wm1));
    if ((wf - w0) * (wf - wmp) <= R(1e-20)) return wf;
    R dmp = minmod(d0, dp1);
    R dmm = minmod(dm1, d0);
    R wmd = R(0.5) * (w0 + wp1) - R(0.5) * dmp;
    R wul = w0 + alpha * (w0 - wm1);
    R wlc = R(0.5) * (R(3) * w0 - wm1) + R(4.0 / 3.0) * dmm;
    R lo = fmax(fmin(w0, fmin(wp1, wmd)), fmin(w0, fmin(wul, wlc)));
    R hi = fmin(fmax(w0, fmax(wp1, wmd)), fmax(w0, fmax(wul, wlc)));
    return wf + minmod(lo - wf, hi - wf);
}

// Sutherland viscosity normalised to 1 at T = 1, divided by Re (Sec. 2).
template <class R>
__device__ __forceinline__ R viscosity(R T, R suth, R re)
{
    return cdiv(T * csqrt(T) * (R(1) + suth), (T + suth) * re);
}

// Curvilinear HLLC flux of Sec. 5.1.1 for primitive states L, R and
// interface metrics (nt, nx, ny, nz) = (hat xi_t, hat xi_x, hat xi_y, hat xi_z);
// igm1 = 1 / (gamma - 1).
// One physical flux and at most one star state are formed: the selected side
// K is L when S_L >= 0, R when S_R <= 0, else the side of S*. The wave speeds
// and S* are evaluated as the paper prints them; the star state uses the two
// shared reciprocals 1 / |grad xi|^2 and 1 / (S_K - S*), which is the printed
// expression with the factor rho_K (S_K - U_K) / (S_K - S*) multiplied in.
template <class R>
__device__ __forceinline__ void hllc(const R PL[5], const R PR[5], R nt, R nx, R ny, R nz, R gamma,
                                     R igm1, R F[5])
{
    R nn = nx * nx + ny * ny + nz * nz;
    R sn = csqrt(nn);
    R UL = nt + nx * PL[1] + ny * PL[2] + nz * PL[3];
    R UR = nt + nx * PR[1] + ny * PR[2] + nz * PR[3];
    R cL = csqrt(cdiv(gamma * PL[4], PL[0]));
    R cR = csqrt(cdiv(gamma * PR[4], PR[0]));
    R SL = fmin(UL - cL * sn, UR - cR * sn);
    R SR = fmax(UL + cL * sn, UR + cR * sn);
    R Ss = cdiv(PR[0] * UR * (SR - UR) - PL[0] * UL * (SL - UL) + (PL[4] - PR[4]) * nn,
                PR[0] * (SR - UR) - PL[0] * (SL - UL));

    bool useL = (R(0) <= SL) || (!(R(0) >= SR) && (R(0) <= Ss));
    bool star = !(R(0) <= SL) && !(R(0) >= SR);
    const R *P = useL ? PL : PR;
    R U = useL ? UL : UR;
    R SK = useL ? SL : SR;
    R r = P[0], u = P[1], v = P[2], w = P[3], p = P[4];
    R E = p * igm1 + R(0.5) * r * (u * u + v * v + w * w);
    F[0] = r * U;
    F[1] = r * u * U + nx * p;
    F[2] = r * v * U + ny * p;
    F[3] = r * w * U + nz * p;
    F[4] = (E + p) * U - nt * p;
    if (star) {
        const R inn = cdiv(R(1), nn);
        const R isk = cdiv(R(1), SK - Ss);
        const R d = SK - U;
        const R fac = r * d * isk;
        const R fn = fac * inn;
        R q1 = fn * (nx * (Ss - nt) + (ny * ny + nz * nz) * u - ny * nx * v - nz * nx * w);
        R q2 = fn * (ny * (Ss - nt) - nx * ny * u + (nx * nx + nz * nz) * v - nz * ny * w);
        R q3 = fn * (nz * (Ss - nt) - nx * nz * u - ny * nz * v + (nx * nx + ny * ny) * w);
        // fac (E / rho + (S* - U) ((S* - xi_t) / |grad xi|^2 + p / (rho (S_K - U))))
        R q4 = isk * (d * E + (Ss - U) * p) + fn * (Ss - U) * (Ss - nt);
        F[0] += SK * (fac - r);
        F[1] += SK * (q1 - r * u);
        F[2] += SK * (q2 - r * v);
        F[3] += SK * (q3 - r * w);
        F[4] += SK * (q4 - E);
    }
}

// Time-step bound of one cell (App. B): min over the directions d of
// 1 / (|U_d| + c |grad d|) from the unhatted cell metrics, and, for viscous
// flow, min_d 1 / (nu |grad d|^2) divided by alpha_D, with nu = mu / rho.
// The step is dt = CFL * (minimum over all cells). The temporal metrics are
// read only on moving grids (they are zero on static ones).
template <int NDIM, bool VISC>
__device__ __forceinline__ double cell_dt_bound(const double *Q, const double *m, long N, long idx, double gamma,
                                                double gm1, double gM2, double suth, double re, double alpha_d,
                                                bool moving)
{
    double r = Q[idx];
    double u = Q[N + idx] / r, v = Q[2 * N + idx] / r;
    double w = (NDIM == 3) ? Q[3 * N + idx] / r : 0.0;
    double p = gm1 * (Q[(NDIM + 1) * N + idx] - 0.5 * r * (u * u + v * v + w * w));
    double c = sqrt(gamma * p / r);
    double nu = VISC ? viscosity(gM2 * p / r, suth, re) / r : 0.0;
    double best = __builtin_inf(), bv = __builtin_inf();
#pragma unroll
    for (int d = 0; d < NDIM; ++d) {
        double dx = m[GBR_SLOT_CELL_UNHAT(d, 0) * N + idx];
        double dy = m[GBR_SLOT_CELL_UNHAT(d, 1) * N + idx];
        double dz = m[GBR_SLOT_CELL_UNHAT(d, 2) * N + idx];
        double U = (moving ? m[GBR_SLOT_CELL_UNHATT(d) * N + idx] : 0.0) + dx * u + dy * v + dz * w;
        double g2 = dx * dx + dy * dy + dz * dz;
        best = fmin(best, 1.0 / (fabs(U) + c * sqrt(g2)));
        if (VISC) bv = fmin(bv, 1.0 / (nu * g2));
    }
    if (VISC) best = fmin(best, bv / alpha_d);
    return best;
}

// Primitive pencils and their first derivatives in LDS: NVL variables at a
// stride vs. With NVL = 5 they are (rho, u, v, w, p); with NVL = 4 (2-D)
// they are (rho, u, v, p) and w is identically zero.
template <int NVL, class R>
__device__ __forceinline__ R pencil(const R *x, int vs, int v, int o)
{
    if (NVL == 4) {
        if (v == 3) return R(0);
        if (v == 4) v = 3;
    }
    return x[v * vs + o];
}

// Hermite second derivatives of the four cells a-1 .. a+2 of an interface
// (Step-1 of Sec. 5.1) from primitives P and first derivatives G of one
// variable, both pointing at cell a, with stride ST between cells (a
// constant stride folds into the LDS offsets once inlined).
template <class R>
__device__ __forceinline__ void second_derivs(const R *P, const R *G, int ST, R h[4])
{
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int o = (q - 1) * ST;
        h[q] = hermite2(P[o - ST], P[o], P[o + ST], G[o - ST], G[o + ST]);
    }
}

// Limited interface states of Step-2..Step-5 of Sec. 5.1: characteristic
// projection with the left eigenvectors of the averaged state and the unit
// interface normal (App. A), unlimited van Leer states, MP limiter per
// field (App. E), back projection. P, G point at the pencil primitives and
// first derivatives of cell a (the left cell), ST is the stride between
// cells and vsP, vsG the strides between variables.
template <int NVL, class R>
__device__ __forceinline__ void limited_states(const R *P, const R *G, int ST, int vsP, int vsG, R nx, R ny, R nz,
                                               R gamma, R alpha_mp, R beta_mp, R PL[5], R PR[5])
{
    const R twelfth = R(1.0 / 12.0);
    const int ip = (NVL == 4) ? 3 : 4;
    R rb = R(0.5) * (P[0] + P[ST]);
    R pb = R(0.5) * (P[ip * vsP] + P[ip * vsP + ST]);
    R ab2 = cdiv(gamma * pb, rb);
    R ra = rb * csqrt(ab2);
    R inn = cdiv(R(1), csqrt(nx * nx + ny * ny + nz * nz));
    R ex = nx * inn, ey = ny * inn, ez = nz * inn;
    // projection of a primitive vector x:
    //   W0 = p - ra (e.u),  W4 = p + ra (e.u),
    //   (W1, W2, W3) = (ex s + (e x u)_x, ez s + (e x u)_z, -ey s - (e x u)_y),
    //   s = a^2 rho - p
    auto project = [&](R x0, R x1, R x2, R x3, R x4, R W[5]) {
        R un = ex * x1 + ey * x2 + ez * x3;
        R s = ab2 * x0 - x4;
        W[0] = x4 - ra * un;
        W[1] = ex * s + (ey * x3 - ez * x2);
        W[2] = ez * s + (ex * x2 - ey * x1);
        W[3] = -ey * s - (ez * x1 - ex * x3);
        W[4] = x4 + ra * un;
    };
    auto ld = [&](const R *x, int vs, int v, int o) { return pencil<NVL>(x, vs, v, o); };
    // cell values W[q] (q = 0..3 -> cells a-1 .. a+2), curvatures W2[q],
    // first derivatives W1[0..1] (cells a, a+1)
    R W[4][5], W2[4][5], W1[2][5];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int o = (q - 1) * ST;
        project(ld(P, vsP, 0, o), ld(P, vsP, 1, o), ld(P, vsP, 2, o), ld(P, vsP, 3, o), ld(P, vsP, 4, o), W[q]);
    }
    {
        R h[5][4];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            if (NVL == 4 && v == 3) {
#pragma unroll
                for (int q = 0; q < 4; ++q) h[v][q] = R(0);
            } else {
                const int vv = (NVL == 4 && v == 4) ? 3 : v;
                second_derivs(P + vv * vsP, G + vv * vsG, ST, h[v]);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) project(h[0][q], h[1][q], h[2][q], h[3][q], h[4][q], W2[q]);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int o = q * ST;
        project(ld(G, vsG, 0, o), ld(G, vsG, 1, o), ld(G, vsG, 2, o), ld(G, vsG, 3, o), ld(G, vsG, 4, o), W1[q]);
    }
    R WL[5], WR[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        R wl = W[1][v] + R(0.5) * W1[0][v] + twelfth * W2[1][v];
        R wr = W[2][v] - R(0.5) * W1[1][v] + twelfth * W2[2][v];
        WL[v] = mp_limit(W[0][v], W[1][v], W[2][v], W2[0][v], W2[1][v], W2[2][v], wl, alpha_mp, beta_mp);
        WR[v] = mp_limit(W[3][v], W[2][v], W[1][v], W2[3][v], W2[2][v], W2[1][v], wr, alpha_mp, beta_mp);
    }
    // right eigenvectors (App. A)
    R ia2 = cdiv(R(1), ab2);
    R i2ra = cdiv(R(0.5), ra);
    auto back = [&](const R *w, R *x) {
        R h = (w[4] - w[0]) * i2ra;
        x[0] = (R(0.5) * (w[0] + w[4]) + ex * w[1] + ez * w[2] - ey * w[3]) * ia2;
        x[1] = ex * h - ey * w[2] - ez * w[3];
        x[2] = ey * h - ez * w[1] + ex * w[2];
        x[3] = ez * h + ey * w[1] + ex * w[3];
        x[4] = R(0.5) * (w[0] + w[4]);
    };
    back(WL, PL);
    back(WR, PR);
}

// Unlimited van Leer states of Eq. vanleer-poly, formed directly in
// primitive variables (identical to projecting and back-projecting since
// R R^-1 = I). Same pointer conventions as limited_states.
template <int NVL, class R>
__device__ __forceinline__ void direct_states(const R *P, const R *G, int ST, int vsP, int vsG, R PL[5], R PR[5])
{
    const R twelfth = R(1.0 / 12.0);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        if (NVL == 4 && v == 3) {
            PL[v] = R(0);
            PR[v] = R(0);
            continue;
        }
        const int vv = (NVL == 4 && v == 4) ? 3 : v;
        const R *x = P + vv * vsP;
        const R *g = G + vv * vsG;
        R ha = hermite2(x[-ST], x[0], x[ST], g[-ST], g[ST]);
        R hb = hermite2(x[0], x[ST], x[2 * ST], g[0], g[2 * ST]);
        PL[v] = x[0] + R(0.5) * g[0] + twelfth * ha;
        PR[v] = x[ST] - R(0.5) * g[ST] + twelfth * hb;
    }
}

// Limited interface states as in limited_states, with the Hermite second
// derivatives precomputed per cell (CURV: H, variable stride vsH, same cell
// indexing as P) or formed per characteristic field from its values and
// first derivatives (not CURV: P and G are read at cells a-2 .. a+3, H is
// not read). The characteristic fields are formed and limited one at a
// time straight from the pencils, so few projected values are live at
// once.
template <int NVL, bool REREAD, bool CURV = true, class R>
__device__ __forceinline__ void limited_states_pre(const R *P0, const R *G0, const R *H0, int ST, int vsP, int vsG,
                                                   int vsH, R nx, R ny, R nz, R gamma, R alpha_mp, R beta_mp,
                                                   R PL[5], R PR[5])
{
    const R twelfth = R(1.0 / 12.0);
    const int ip = (NVL == 4) ? 3 : 4;
    R rb = R(0.5) * (P0[0] + P0[ST]);
    R pb = R(0.5) * (P0[ip * vsP] + P0[ip * vsP + ST]);
    R ab2 = cdiv(gamma * pb, rb);
    R ra = rb * csqrt(ab2);
    R inn = cdiv(R(1), csqrt(nx * nx + ny * ny + nz * nz));
    R ex = nx * inn, ey = ny * inn, ez = nz * inn;
    auto ld = [&](const R *x, int vs, int v, int o) { return pencil<NVL>(x, vs, v, o); };
    // point k = 0..3: cells a-1 .. a+2 (values and curvatures), k = 0..1:
    // cells a, a+1 (first derivatives)
    R WL[5], WR[5];
    auto limit = [&](int v, const R w[4], const R d[4], const R g[2]) {
        R wl = w[1] + R(0.5) * g[0] + twelfth * d[1];
        R wr = w[2] - R(0.5) * g[1] + twelfth * d[2];
        WL[v] = mp_limit(w[0], w[1], w[2], d[0], d[1], d[2], wl, alpha_mp, beta_mp);
        WR[v] = mp_limit(w[3], w[2], w[1], d[3], d[2], d[1], wr, alpha_mp, beta_mp);
    };
    // one field's values w and curvatures d at cells a-1 .. a+2 and first
    // derivatives g at a, a+1, through its projection F(pencil, stride,
    // offset). Without CURV the curvatures are formed from the field's
    // values and first derivatives at a-2 .. a+3 (the Hermite formula is
    // linear, so this equals projecting the primitive curvatures up to
    // rounding).
    auto field = [&](auto F, const R *P, const R *G, const R *H, R w[4], R d[4], R g[2]) {
        if constexpr (CURV) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                w[k] = F(P, vsP, (k - 1) * ST);
                d[k] = F(H, vsH, (k - 1) * ST);
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) g[k] = F(G, vsG, k * ST);
        } else {
            R w6[6], g6[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                w6[k] = F(P, vsP, (k - 2) * ST);
                g6[k] = F(G, vsG, (k - 2) * ST);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                w[k] = w6[k + 1];
                d[k] = hermite2(w6[k], w6[k + 1], w6[k + 2], g6[k], g6[k + 2]);
            }
            g[0] = g6[2];
            g[1] = g6[3];
        }
    };
    // W0 = p - ra (e.u), W4 = p + ra (e.u), one field at a time (fewer live
    // registers at the limiter's peak). With REREAD each field reads the
    // pencils from LDS again: an opaque zero offset keeps the compiler from
    // merging the reads of the five fields and holding every pencil value
    // across all of them (FP64 sweeps: xi 148 -> 106 VGPRs, eta / zeta
    // without the curvature array 168 with spills -> 108, a fourth wave per
    // SIMD).
#pragma unroll
    for (int sgn = -1; sgn <= 1; sgn += 2) {
        R w[4], d[4], g[2];
        int z = 0;
        if (REREAD) __asm__ volatile("" : "+v"(z));
        const R *P = P0 + z, *G = G0 + z, *H = H0 + z;
        auto acoustic = [&](const R *x, int vs, int o) {
            R un = ex * ld(x, vs, 1, o) + ey * ld(x, vs, 2, o) + ez * ld(x, vs, 3, o);
            R x4 = ld(x, vs, 4, o);
            return sgn < 0 ? x4 - ra * un : x4 + ra * un;
        };
        field(acoustic, P, G, H, w, d, g);
        limit(sgn < 0 ? 0 : 4, w, d, g);
    }
    // W1 = ex s + (ey w - ez v), W2 = ez s + (ex v - ey u),
    // W3 = -ey s - (ez u - ex w), s = a^2 rho - p
    auto entropy_shear = [&](int v, const R *x, int vs, int o) {
        R s = ab2 * ld(x, vs, 0, o) - ld(x, vs, 4, o);
        R u = ld(x, vs, 1, o), vv = ld(x, vs, 2, o), w = ld(x, vs, 3, o);
        if (v == 1) return ex * s + (ey * w - ez * vv);
        if (v == 2) return ez * s + (ex * vv - ey * u);
        return -ey * s - (ez * u - ex * w);
    };
#pragma unroll
    for (int v = 1; v <= 3; ++v) {
        R w[4], d[4], g[2];
        int z = 0;
        if (REREAD) __asm__ volatile("" : "+v"(z));
        const R *P = P0 + z, *G = G0 + z, *H = H0 + z;
        field([&](const R *x, int vs, int o) { return entropy_shear(v, x, vs, o); }, P, G, H, w, d, g);
        limit(v, w, d, g);
    }
    // right eigenvectors (App. A)
    R ia2 = cdiv(R(1), ab2);
    R i2ra = cdiv(R(0.5), ra);
    auto back = [&](const R *w, R *x) {
        R h = (w[4] - w[0]) * i2ra;
        x[0] = (R(0.5) * (w[0] + w[4]) + ex * w[1] + ez * w[2] - ey * w[3]) * ia2;
        x[1] = ex * h - ey * w[2] - ez * w[3];
        x[2] = ey * h - ez * w[1] + ex * w[2];
        x[3] = ez * h + ey * w[1] + ex * w[3];
        x[4] = R(0.5) * (w[0] + w[4]);
    };
    back(WL, PL);
    back(WR, PR);
}

// Unlimited van Leer states with precomputed curvatures (see direct_states).
template <int NVL, class R>
__device__ __forceinline__ void direct_states_pre(const R *P, const R *G, const R *H, int ST, int vsP, int vsG,
                                                  int vsH, R PL[5], R PR[5])
{
    const R twelfth = R(1.0 / 12.0);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        if (NVL == 4 && v == 3) {
            PL[v] = R(0);
            PR[v] = R(0);
            continue;
        }
        const int vv = (NVL == 4 && v == 4) ? 3 : v;
        const R *x = P + vv * vsP;
        const R *g = G + vv * vsG;
        const R *h = H + vv * vsH;
        PL[v] = x[0] + R(0.5) * g[0] + twelfth * h[0];
        PR[v] = x[ST] - R(0.5) * g[ST] + twelfth * h[ST];
    }
}

}  // namespace gbr

// Device-side building blocks of the gradient-based-reconstruction RHS.
// Each function states the passage of the paper it evaluates.
#pragma once

#include <hip/hip_runtime.h>

namespace gbr {

// Periodic index: a in any range, n >= 1.
__device__ __forceinline__ int wrap_index(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Number of periods crossed going from [0, n) to index a (floor(a / n)).
__device__ __forceinline__ int wrap_count(int a, int n)
{
    int r = a % n;
    if (r < 0) r += n;
    return (a - r) / n;
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

template <class R>
__device__ __forceinline__ R minmod(R a, R b)
{
    // 0.5 (sign a + sign b) min(|a|, |b|) with sign(0) = 0
    R s = (a > R(0) ? R(0.5) : (a < R(0) ? R(-0.5) : R(0))) + (b > R(0) ? R(0.5) : (b < R(0) ? R(-0.5) : R(0)));
    return s * fmin(fabs(a), fabs(b));
}

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
    return T * sqrt(T) * (R(1) + suth) / (T + suth) / re;
}

// Curvilinear HLLC flux of Sec. 5.1.1 for primitive states L, R and
// interface metrics (nt, nx, ny, nz) = (hat xi_t, hat xi_x, hat xi_y, hat xi_z).
// One physical flux and at most one star state are formed: the selected side
// K is L when S_L >= 0, R when S_R <= 0, else the side of S*. The wave speeds,
// S* and the star state are evaluated in the order the paper prints them.
template <class R>
__device__ __forceinline__ void hllc(const R PL[5], const R PR[5], R nt, R nx, R ny, R nz, R gamma,
                                     R gm1, R F[5])
{
    R nn = nx * nx + ny * ny + nz * nz;
    R sn = sqrt(nn);
    R UL = nt + nx * PL[1] + ny * PL[2] + nz * PL[3];
    R UR = nt + nx * PR[1] + ny * PR[2] + nz * PR[3];
    R cL = sqrt(gamma * PL[4] / PL[0]);
    R cR = sqrt(gamma * PR[4] / PR[0]);
    R SL = fmin(UL - cL * sn, UR - cR * sn);
    R SR = fmax(UL + cL * sn, UR + cR * sn);
    R Ss = (PR[0] * UR * (SR - UR) - PL[0] * UL * (SL - UL) + (PL[4] - PR[4]) * nn) /
           (PR[0] * (SR - UR) - PL[0] * (SL - UL));

    bool useL = (R(0) <= SL) || (!(R(0) >= SR) && (R(0) <= Ss));
    bool star = !(R(0) <= SL) && !(R(0) >= SR);
    const R *P = useL ? PL : PR;
    R U = useL ? UL : UR;
    R SK = useL ? SL : SR;
    R r = P[0], u = P[1], v = P[2], w = P[3], p = P[4];
    R E = p / gm1 + R(0.5) * r * (u * u + v * v + w * w);
    F[0] = r * U;
    F[1] = r * u * U + nx * p;
    F[2] = r * v * U + ny * p;
    F[3] = r * w * U + nz * p;
    F[4] = (E + p) * U - nt * p;
    if (star) {
        R fac = r * (SK - U) / (SK - Ss);
        R q1 = fac * (nx * (Ss - nt) + (ny * ny + nz * nz) * u - ny * nx * v - nz * nx * w) / nn;
        R q2 = fac * (ny * (Ss - nt) - nx * ny * u + (nx * nx + nz * nz) * v - nz * ny * w) / nn;
        R q3 = fac * (nz * (Ss - nt) - nx * nz * u - ny * nz * v + (nx * nx + ny * ny) * w) / nn;
        R q4 = fac * (E / r + (Ss - U) * ((Ss - nt) / nn + p / (r * (SK - U))));
        F[0] += SK * (fac - r);
        F[1] += SK * (q1 - r * u);
        F[2] += SK * (q2 - r * v);
        F[3] += SK * (q3 - r * w);
        F[4] += SK * (q4 - E);
    }
}

}  // namespace gbr

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

// E6 first derivative (Eq. E6_grads, as differences) from the six neighbours.
__device__ __forceinline__ double e6(double m3, double m2, double m1, double p1, double p2, double p3)
{
    return 0.75 * (p1 - m1) - 0.15 * (p2 - m2) + (1.0 / 60.0) * (p3 - m3);
}

// Hermite second derivative (Step-1 of Sec. 5.1).
__device__ __forceinline__ double hermite2(double vm, double v0, double vp, double gm, double gp)
{
    return 2.0 * (vp - 2.0 * v0 + vm) - 0.5 * (gp - gm);
}

__device__ __forceinline__ double minmod(double a, double b)
{
    // 0.5 (sign a + sign b) min(|a|, |b|) with sign(0) = 0
    double s = (a > 0.0 ? 0.5 : (a < 0.0 ? -0.5 : 0.0)) + (b > 0.0 ? 0.5 : (b < 0.0 ? -0.5 : 0.0));
    return s * fmin(fabs(a), fabs(b));
}

// Improved MP limiter of App. E for one characteristic component at the left
// state of an interface: wm1, w0, wp1 are the cell values upwind, at and
// downwind of the reconstructing cell, dm1, d0, dp1 their gradient-based
// curvatures, wf the unlimited interface value. The right state is the same
// procedure on the stencil reflected about its own cell.
__device__ __forceinline__ double mp_limit(double wm1, double w0, double wp1, double dm1, double d0,
                                           double dp1, double wf, double alpha, double beta)
{
    double wmp = w0 + minmod(wp1 - w0, beta * (w0 - wm1));
    if ((wf - w0) * (wf - wmp) <= 1e-20) return wf;
    double dmp = minmod(d0, dp1);
    double dmm = minmod(dm1, d0);
    double wmd = 0.5 * (w0 + wp1) - 0.5 * dmp;
    double wul = w0 + alpha * (w0 - wm1);
    double wlc = 0.5 * (3.0 * w0 - wm1) + (4.0 / 3.0) * dmm;
    double lo = fmax(fmin(w0, fmin(wp1, wmd)), fmin(w0, fmin(wul, wlc)));
    double hi = fmin(fmax(w0, fmax(wp1, wmd)), fmax(w0, fmax(wul, wlc)));
    return wf + minmod(lo - wf, hi - wf);
}

// Sutherland viscosity normalised to 1 at T = 1, divided by Re (Sec. 2).
__device__ __forceinline__ double viscosity(double T, double suth, double inv_re)
{
    return T * sqrt(T) * (1.0 + suth) / (T + suth) * inv_re;
}

// Curvilinear HLLC flux of Sec. 5.1.1 for primitive states L, R and
// interface metrics (nt, nx, ny, nz) = (hat xi_t, hat xi_x, hat xi_y, hat xi_z).
// One physical flux and at most one star state are formed: the selected side
// K is L when S_L >= 0, R when S_R <= 0, else the side of S*. Reciprocals
// are formed once and reused.
__device__ __forceinline__ void hllc(const double PL[5], const double PR[5], double nt, double nx,
                                     double ny, double nz, double gamma, double inv_gm1, double F[5])
{
    double nn = nx * nx + ny * ny + nz * nz;
    double sn = sqrt(nn);
    double irL = 1.0 / PL[0], irR = 1.0 / PR[0];
    double UL = nt + nx * PL[1] + ny * PL[2] + nz * PL[3];
    double UR = nt + nx * PR[1] + ny * PR[2] + nz * PR[3];
    double cL = sqrt(gamma * PL[4] * irL);
    double cR = sqrt(gamma * PR[4] * irR);
    double SL = fmin(UL - cL * sn, UR - cR * sn);
    double SR = fmax(UL + cL * sn, UR + cR * sn);
    double mL = PL[0] * (SL - UL), mR = PR[0] * (SR - UR);
    double Ss = (mR * UR - mL * UL + (PL[4] - PR[4]) * nn) / (mR - mL);

    bool useL = (0.0 <= SL) || (!(0.0 >= SR) && (0.0 <= Ss));
    bool star = !(0.0 <= SL) && !(0.0 >= SR);
    const double *P = useL ? PL : PR;
    double ir = useL ? irL : irR;
    double U = useL ? UL : UR;
    double SK = useL ? SL : SR;
    double r = P[0], u = P[1], v = P[2], w = P[3], p = P[4];
    double E = p * inv_gm1 + 0.5 * r * (u * u + v * v + w * w);
    F[0] = r * U;
    F[1] = r * u * U + nx * p;
    F[2] = r * v * U + ny * p;
    F[3] = r * w * U + nz * p;
    F[4] = (E + p) * U - nt * p;
    if (star) {
        double sku = SK - U;
        double fac = r * sku / (SK - Ss);
        double dS = Ss - U;
        double inn = 1.0 / nn;
        // star momentum: u + n_a (S* - U) / |n|^2 (the printed components)
        double g = dS * inn;
        double q1 = fac * (u + nx * g);
        double q2 = fac * (v + ny * g);
        double q3 = fac * (w + nz * g);
        double q4 = fac * (E * ir + dS * ((Ss - nt) * inn + p * ir / sku));
        F[0] += SK * (fac - r);
        F[1] += SK * (q1 - r * u);
        F[2] += SK * (q2 - r * v);
        F[3] += SK * (q3 - r * w);
        F[4] += SK * (q4 - E);
    }
}

}  // namespace gbr

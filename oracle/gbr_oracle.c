/*
 * FP64 CPU oracle of the gradient-based-reconstruction (MEG6 + alpha-damping)
 * right-hand side on periodic generalized-curvilinear, optionally moving,
 * grids, after Chandravamsi, Chamarthi, Hoffmann and Frankel (arXiv 2303.10785).
 *
 * TEST INFRASTRUCTURE ONLY: this is the plain, slow, obviously-correct
 * reference that the HIP product path is checked against. Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it. It shares no
 * code, header or table with the HIP path.
 *
 * Style: scalar loops in the order the paper states the steps; no blocking, no
 * fusion beyond what the equations say. Built with -O2 -ffp-contract=off and
 * no fast-math. OpenMP (if enabled) only splits independent cells.
 *
 * Readings of points the paper leaves open (each is also listed in the design
 * notes of the repository):
 *  - Eq. E6_grads and the composite stencil of Sec. 7 fix the E6 gradient as a
 *    difference formula, 3/4 (f[i+1]-f[i-1]) - 3/20 (f[i+2]-f[i-2]) + 1/60 (...).
 *  - The van Leer polynomial is used in its simplified form with 1/12 on the
 *    second derivative (Eq. vanleer-poly); the composite stencil pins this.
 *  - The averaged state for the eigenvectors is the arithmetic mean of rho and
 *    p of the two cells; a = sqrt(gamma p / rho).                 [unpinned]
 *  - MP limiter constants alpha = beta = 4 (Suresh & Huynh); the right state
 *    is the mirror image of the left-state procedure of App. E.   [unpinned]
 *  - HLLC branch order at ties: S_L >= 0 -> F_L; else S* >= 0 -> F*L; else
 *    S_R >= 0 -> F*R; else F_R.
 *  - Viscous tangential face derivatives: average of the two cell gradients
 *    (the damping term of Eq. AD-eqn1 only applies to the normal one). T uses
 *    E6 like the other gradients.                                 [unpinned]
 *  - Non-dimensional state: p = rho T / (gamma Mref^2), mu = Sutherland(T)/Re,
 *    kappa = mu / ((gamma - 1) Mref^2 Pr).
 *  - Shock sensor (not in the paper): Ducros theta = div^2 / (div^2 + |curl|^2
 *    + 1e-30); a face takes the limited path if max(theta_i, theta_i+1) > theta_c.
 *  - GCL: (1/J)_t = -sum_d Delta_d (I_d hat(d)_t), the hatted temporal metric
 *    interpolated to faces with the same central scheme (Eq. Jacb2).
 *  - Time step: CFL * min over cells and directions of 1/(|U|+c|grad d|), and
 *    for viscous runs also (1/alpha_d) min 1/(nu |grad d|^2), nu = mu/rho.
 *  - RK3 advances Q with L(Q) = J (Res - (1/J)_t Q) (App. B, Eq. time-split);
 *    moving-grid metrics are evaluated once per step at t^n.
 */
#include "gbr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* indexing and periodic neighbours                                         */
/* ------------------------------------------------------------------------ */
static long ncell_of(const ref_cfg *g) { return (long)g->n[0] * g->n[1] * g->n[2]; }

static long cell_index(const ref_cfg *g, const int ijk[3])
{
    return ijk[0] + (long)g->n[0] * (ijk[1] + (long)g->n[1] * ijk[2]);
}

/* Neighbour m steps along direction d of cell ijk: returns its linear index
 * and the number of times the index wrapped (negative when going below 0). */
static long neighbour(const ref_cfg *g, const int ijk[3], int d, int m, int *wraps)
{
    int t[3] = {ijk[0], ijk[1], ijk[2]};
    int n = g->n[d];
    int a = t[d] + m;
    int r = a % n;
    if (r < 0) r += n;
    if (wraps) *wraps = (a - r) / n;
    t[d] = r;
    return cell_index(g, t);
}

static void unpack(const ref_cfg *g, long idx, int ijk[3])
{
    ijk[0] = (int)(idx % g->n[0]);
    ijk[1] = (int)((idx / g->n[0]) % g->n[1]);
    ijk[2] = (int)(idx / ((long)g->n[0] * g->n[1]));
}

/* ------------------------------------------------------------------------ */
/* 1-D stencils of Sec. 5.1 (Step-1) and Sec. 7                             */
/* Each takes a pointer to the centre of a window of consecutive values.    */
/* ------------------------------------------------------------------------ */

/* E6 first derivative at the window centre (Eq. E6_grads, differences). */
static double e6(const double *v)
{
    return 0.75 * (v[1] - v[-1]) - (3.0 / 20.0) * (v[2] - v[-2]) + (1.0 / 60.0) * (v[3] - v[-3]);
}

/* Hermite second derivative at the centre from values and first derivatives
 * (Step-1 of Sec. 5.1): 2 (v+1 - 2 v + v-1) - (g+1 - g-1) / 2. */
static double hermite(const double *v, const double *gv)
{
    return 2.0 * (v[1] - 2.0 * v[0] + v[-1]) - 0.5 * (gv[1] - gv[-1]);
}

/* Central interface value at +1/2 of the window centre: the average of the
 * unlimited left- and right-biased states of Eq. vanleer-poly (Eq. FP-interp,
 * Eq. interp-formulae). Needs v[-4 .. 5]. */
static double face_central(const double *v)
{
    double gv[4], h[2];
    for (int m = -1; m <= 2; ++m) gv[m + 1] = e6(v + m);
    h[0] = hermite(v, gv + 1);
    h[1] = hermite(v + 1, gv + 2);
    double left = v[0] + 0.5 * gv[1] + h[0] / 12.0;
    double right = v[1] - 0.5 * gv[2] + h[1] / 12.0;
    return 0.5 * (left + right);
}

/* Derivative at the centre as the difference of the two central interface
 * values (Eq. FP-interp2). Needs v[-5 .. 5]. */
static double dcomp(const double *v) { return face_central(v) - face_central(v - 1); }

/* ------------------------------------------------------------------------ */
/* line wrappers exported for the stencil pins                              */
/* v[0..n-1] periodic with v[i+n] = v[i] + shift                            */
/* ------------------------------------------------------------------------ */
static void line_window(const double *v, int n, double shift, int i, int lo, int hi, double *w)
{
    for (int m = lo; m <= hi; ++m) {
        int a = i + m, r = a % n;
        if (r < 0) r += n;
        w[m - lo] = v[r] + (double)((a - r) / n) * shift;
    }
}

void ref_line_e6(const double *v, int n, double shift, double *out)
{
    double w[7];
    for (int i = 0; i < n; ++i) { line_window(v, n, shift, i, -3, 3, w); out[i] = e6(w + 3); }
}

void ref_line_hermite(const double *v, int n, double shift, double *out)
{
    double w[9], gv[3];
    for (int i = 0; i < n; ++i) {
        line_window(v, n, shift, i, -4, 4, w);
        for (int m = -1; m <= 1; ++m) gv[m + 1] = e6(w + 4 + m);
        out[i] = hermite(w + 4, gv + 1);
    }
}

void ref_line_face(const double *v, int n, double shift, double *out)
{
    double w[10];
    for (int i = 0; i < n; ++i) { line_window(v, n, shift, i, -4, 5, w); out[i] = face_central(w + 4); }
}

void ref_line_dcomp(const double *v, int n, double shift, double *out)
{
    double w[11];
    for (int i = 0; i < n; ++i) { line_window(v, n, shift, i, -5, 5, w); out[i] = dcomp(w + 5); }
}

/* ------------------------------------------------------------------------ */
/* Metrics (Sec. 4, Sec. 7)                                                 */
/* ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ */
/* IG4 gradients of the MIG4 scheme (Eq. IG4_grads), read as differences as */
/* Eq. E6_grads is, with alpha = 5/14:                                      */
/*   alpha f'_{k-1} + f'_k + alpha f'_{k+1}                                  */
/*     = a (f_{k+1} - f_{k-1}) + b (f_{k+2} - f_{k-2}),                     */
/*   a = 2 (2 + alpha) / 6,  b = (4 alpha - 1) / 12.                         */
/* On a periodic line the system is cyclic. A line whose periodic extension */
/* satisfies F_{k+n} = F_k + J_k with J periodic (a coordinate, J = its     */
/* period offset, or a coordinate times a periodic factor) has a derivative */
/* whose extension satisfies F'_{k+n} = F'_k + (IG4 J)_k; the two rows that */
/* reach across the ends carry that jump on their right-hand side. Each     */
/* system is solved densely (Gaussian elimination with partial pivoting),   */
/* which is slow and plain; lines are short in every use here.              */
/* Pins: Fourier symbol of the scheme, linear-plus-periodic lines, fourth   */
/* order, MIG4 metric identities and freestream.                            */
/* ------------------------------------------------------------------------ */
static const double ig4_alpha = 5.0 / 14.0;
#define IG4_A (2.0 * (2.0 + ig4_alpha) / 6.0)
#define IG4_B ((4.0 * ig4_alpha - 1.0) / 12.0)

static int floor_div(int a, int n)
{
    int r = a % n;
    if (r < 0) r += n;
    return (a - r) / n;
}

static int mod_n(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* Solve A y = r, A n x n row-major; A and r are overwritten. */
static int solve_dense(double *A, double *r, int n, double *y)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int k = c + 1; k < n; ++k)
            if (fabs(A[k * n + c]) > fabs(A[piv * n + c])) piv = k;
        if (A[piv * n + c] == 0.0) return 1;
        if (piv != c) {
            for (int k = 0; k < n; ++k) {
                double t = A[c * n + k]; A[c * n + k] = A[piv * n + k]; A[piv * n + k] = t;
            }
            double t = r[c]; r[c] = r[piv]; r[piv] = t;
        }
        for (int k = c + 1; k < n; ++k) {
            double f = A[k * n + c] / A[c * n + c];
            if (f == 0.0) continue;
            for (int q = c; q < n; ++q) A[k * n + q] -= f * A[c * n + q];
            r[k] -= f * r[c];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        double s = r[c];
        for (int q = c + 1; q < n; ++q) s -= A[c * n + q] * y[q];
        y[c] = s / A[c * n + c];
    }
    return 0;
}

/* F_ext(m) of a line with jump J (J == NULL: periodic). */
static double ext_val(const double *F, const double *J, int n, int m)
{
    int r = mod_n(m, n);
    return J ? F[r] + (double)floor_div(m, n) * J[r] : F[r];
}

/* IG4 derivative y[0..n-1] of the line F with jump J; dj[0..n-1] (may be
 * NULL) receives the jump of the derivative, IG4 of J. */
static int ig4_ext(const double *F, const double *J, int n, double *y, double *dj)
{
    double *A = (double *)calloc((size_t)n * n, sizeof(double));
    double *r = (double *)malloc(sizeof(double) * n);
    double *djl = (double *)calloc((size_t)n, sizeof(double));
    int rc = (!A || !r || !djl) ? -1 : 0;
    if (!rc && J) rc = ig4_ext(J, NULL, n, djl, NULL);
    if (!rc) {
        for (int k = 0; k < n; ++k) {
            r[k] = IG4_A * (ext_val(F, J, n, k + 1) - ext_val(F, J, n, k - 1))
                 + IG4_B * (ext_val(F, J, n, k + 2) - ext_val(F, J, n, k - 2));
            A[k * n + k] += 1.0;
            for (int s = -1; s <= 1; s += 2) {
                int m = k + s, col = mod_n(m, n);
                A[k * n + col] += ig4_alpha;
                /* y_m = y_col + floor(m / n) * dj_col */
                r[k] -= ig4_alpha * (double)floor_div(m, n) * djl[col];
            }
        }
        rc = solve_dense(A, r, n, y);
    }
    if (!rc && dj) memcpy(dj, djl, sizeof(double) * n);
    free(A); free(r); free(djl);
    return rc;
}

/* Interface values I_{k+1/2}, k = -1 .. n-1 (face[k + 1]), of the line F
 * with jump J: the average of the unlimited left and right states of
 * Eq. vanleer-poly built on IG4 first derivatives and the Hermite second
 * derivative (Eq. FP-interp). */
static int ig4_faces(const double *F, const double *J, int n, double *face)
{
    double *y = (double *)malloc(sizeof(double) * n);
    double *dj = (double *)malloc(sizeof(double) * n);
    int rc = (!y || !dj) ? -1 : ig4_ext(F, J, n, y, dj);
    if (!rc) {
        for (int k = -1; k <= n - 1; ++k) {
            double v[4], g[4];  /* cells k-1 .. k+2 */
            for (int q = 0; q < 4; ++q) {
                int m = k - 1 + q;
                v[q] = ext_val(F, J, n, m);
                g[q] = y[mod_n(m, n)] + (J ? (double)floor_div(m, n) * dj[mod_n(m, n)] : 0.0);
            }
            double hl = hermite(v + 1, g + 1);
            double hr = hermite(v + 2, g + 2);
            double left = v[1] + 0.5 * g[1] + hl / 12.0;
            double right = v[2] - 0.5 * g[2] + hr / 12.0;
            face[k + 1] = 0.5 * (left + right);
        }
    }
    free(y); free(dj);
    return rc;
}

int ref_line_ig4(const double *v, int n, double shift, double *out)
{
    double *J = (double *)malloc(sizeof(double) * n);
    if (!J) return -1;
    for (int i = 0; i < n; ++i) J[i] = shift;
    int rc = ig4_ext(v, J, n, out, NULL);
    free(J);
    return rc;
}

int ref_line_ig4_face(const double *v, int n, double shift, double *out)
{
    double *J = (double *)calloc((size_t)n, sizeof(double));
    double *f = (double *)malloc(sizeof(double) * (n + 1));
    int rc = (!J || !f) ? -1 : 0;
    if (!rc) {
        for (int i = 0; i < n; ++i) J[i] = shift;
        rc = ig4_faces(v, J, n, f);
        if (!rc) for (int i = 0; i < n; ++i) out[i] = f[i + 1];
    }
    free(J); free(f);
    return rc;
}

int ref_line_ig4_dcomp(const double *v, int n, double shift, double *out)
{
    double *J = (double *)calloc((size_t)n, sizeof(double));
    double *f = (double *)malloc(sizeof(double) * (n + 1));
    int rc = (!J || !f) ? -1 : 0;
    if (!rc) {
        for (int i = 0; i < n; ++i) J[i] = shift;
        rc = ig4_faces(v, J, n, f);
        if (!rc) for (int i = 0; i < n; ++i) out[i] = f[i + 1] - f[i];
    }
    free(J); free(f);
    return rc;
}

/* Cells of the line along d through ijk, in order k = 0 .. n_d - 1. */
static void line_cells(const ref_cfg *g, const int ijk[3], int d, long *cells)
{
    int t[3] = {ijk[0], ijk[1], ijk[2]};
    for (int k = 0; k < g->n[d]; ++k) {
        t[d] = k;
        cells[k] = cell_index(g, t);
    }
}

/* Visit every line along d: calls fn(ctx, cells) once per line. */
static int for_lines(const ref_cfg *g, int d, int (*fn)(void *, const long *), void *ctx)
{
    long *cells = (long *)malloc(sizeof(long) * g->n[d]);
    if (!cells) return -1;
    int a = (d + 1) % 3, b = (d + 2) % 3, rc = 0;
    for (int ib = 0; ib < g->n[b] && !rc; ++ib)
        for (int ia = 0; ia < g->n[a] && !rc; ++ia) {
            int ijk[3];
            ijk[d] = 0; ijk[a] = ia; ijk[b] = ib;
            line_cells(g, ijk, d, cells);
            rc = fn(ctx, cells);
        }
    free(cells);
    return rc;
}

/* (x + wraps * off) - org, the position of a periodic image of x relative to
 * org, with one rounding of the small result. The image x + wraps * off is
 * not representable in general (x and off of the size of the domain, the
 * result of the size of a cell): formed in one rounded step it carries an
 * error of eps |x| that the metrics divide by the spacing. Here the product
 * and the sum are split into exact value and error pairs (the product error
 * from a fused multiply-add, the sum error from the two-sum of Knuth), the
 * leading part minus org is exact when the image lies near org, and the
 * error terms are added last. In exact arithmetic this is the periodic
 * extension of the coordinates (Sec. 4.2); only the rounding changes. */
static double image_rel(double x, int wraps, double off, double org)
{
    if (wraps == 0) return x - org;
    const double p = (double)wraps * off;
    const double pe = fma((double)wraps, off, -p);
    const double s = x + p;
    const double bp = s - x;
    const double se = (x - (s - bp)) + (p - bp);
    return (s - org) + (se + pe);
}

/* Coordinate c of the periodic extension at neighbour m along d of a cell. */
static double coord_ext(const ref_cfg *g, const double *xyz, const int ijk[3], int d, int m, int c)
{
    int wraps;
    long nb = neighbour(g, ijk, d, m, &wraps);
    return xyz[c * ncell_of(g) + nb] + (double)wraps * g->off[d][c];
}

/* Coordinate c of the periodic extension at neighbour m along d of a cell,
 * measured from org. */
static double coord_rel(const ref_cfg *g, const double *xyz, const int ijk[3], int d, int m, int c, double org)
{
    int wraps;
    long nb = neighbour(g, ijk, d, m, &wraps);
    return image_rel(xyz[c * ncell_of(g) + nb], wraps, g->off[d][c], org);
}

/* Window of a periodic cell field along d (no shift). */
static void field_window(const ref_cfg *g, const double *f, const int ijk[3], int d, int lo, int hi, double *w)
{
    for (int m = lo; m <= hi; ++m) w[m - lo] = f[neighbour(g, ijk, d, m, NULL)];
}

/* Conservative metrics of Thomas & Lombard (Eq. GCL_metrics) discretised with
 * the central derivative of Sec. 7, their Jacobian (Eq. Jac-matrix), the
 * interface values (Eq. interp-formulae) and, on moving grids, the temporal
 * metrics (Sec. 4.2) and the GCL rate (Eq. Jacb2).
 * Pins: composite stencil and 3-D identity coefficients (Sec. 7), discrete
 * metric identities, freestream on static and deforming grids.            */
static int metrics_mig4(const ref_cfg *g, const double *xyz, const double *xyz_t, double *m);

static int metrics_bounded(const ref_cfg *g, const double *xyz, const double *xyz_t, double *m);
static int any_bounded(const ref_cfg *g);

int ref_metrics(const ref_cfg *g, const double *xyz, const double *xyz_t, double *m)
{
    if (any_bounded(g)) return metrics_bounded(g, xyz, xyz_t, m);
    if (g->scheme == REF_SCHEME_MIG4) return metrics_mig4(g, xyz, xyz_t, m);
    const long N = ncell_of(g);
    double *dx = (double *)malloc(sizeof(double) * 9 * N); /* dx[(d*3+c)*N] = D_d of coord c */
    if (!dx) return -1;
    int bad = 0;

    /* The metrics are invariant under a translation of the coordinates (in
     * the products below the shift multiplies D_d2 D_d1 - D_d1 D_d2 of a
     * coordinate, which vanishes since the central derivatives commute), so
     * every cell evaluates its windows with coordinates measured from its own
     * centre. This only removes cancellation of O(|x| / dx) on grids far from
     * the origin; across the periodic seam the image is placed relative to
     * the centre with one rounding (image_rel).
     * Step 1: coordinate derivatives D_d(x_c) at cell centres. */
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; ++idx) {
        int ijk[3];
        double w[11];
        unpack(g, idx, ijk);
        for (int d = 0; d < 3; ++d)
            for (int c = 0; c < 3; ++c) {
                for (int q = -5; q <= 5; ++q) w[q + 5] = coord_rel(g, xyz, ijk, d, q, c, xyz[c * N + idx]);
                dx[(d * 3 + c) * N + idx] = dcomp(w + 5);
            }
    }

    /* Step 2: hatted metrics. For direction d and coordinate c, with (d, d1, d2)
     * and (c, c1, c2) cyclic:  hat(d)_c = D_d2[(c1)_d1 * c2] - D_d1[(c1)_d2 * c2].
     * The product is formed from the periodic extension of c2 around the cell.
     * Step 3: 1/J = det[D_d x_c]; unhatted metrics d_c = J hat(d)_c.        */
#pragma omp parallel for schedule(static) reduction(|| : bad)
    for (long idx = 0; idx < N; ++idx) {
        int ijk[3];
        double w[11];
        unpack(g, idx, ijk);
        for (int d = 0; d < 3; ++d) {
            int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
            for (int c = 0; c < 3; ++c) {
                int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
                const double org = xyz[c2 * N + idx];
                for (int q = -5; q <= 5; ++q)
                    w[q + 5] = dx[(d1 * 3 + c1) * N + neighbour(g, ijk, d2, q, NULL)]
                               * coord_rel(g, xyz, ijk, d2, q, c2, org);
                double ta = dcomp(w + 5);
                for (int q = -5; q <= 5; ++q)
                    w[q + 5] = dx[(d2 * 3 + c1) * N + neighbour(g, ijk, d1, q, NULL)]
                               * coord_rel(g, xyz, ijk, d1, q, c2, org);
                double tb = dcomp(w + 5);
                m[REF_M_HAT(d, c) * N + idx] = ta - tb;
            }
        }
        const double *a = dx + idx;
#define DX(d, c) a[((d) * 3 + (c)) * N]
        double invj = DX(0, 0) * (DX(1, 1) * DX(2, 2) - DX(1, 2) * DX(2, 1))
                    - DX(0, 1) * (DX(1, 0) * DX(2, 2) - DX(1, 2) * DX(2, 0))
                    + DX(0, 2) * (DX(1, 0) * DX(2, 1) - DX(1, 1) * DX(2, 0));
#undef DX
        if (!(invj > 0.0)) bad = 1;
        m[REF_M_INVJ * N + idx] = invj;
        m[REF_M_J * N + idx] = 1.0 / invj;
        for (int d = 0; d < 3; ++d)
            for (int c = 0; c < 3; ++c)
                m[REF_M_UNHAT(d, c) * N + idx] = m[REF_M_HAT(d, c) * N + idx] / invj;
    }
    free(dx);

    /* Step 4 (moving grids): hatted temporal metrics hat(d)_t = -(x_t hat(d)_x
     * + y_t hat(d)_y + z_t hat(d)_z) and their unhatted values.             */
    for (long idx = 0; idx < N; ++idx)
        for (int d = 0; d < 3; ++d) {
            double ht = 0.0;
            if (g->moving && xyz_t)
                ht = -(xyz_t[idx] * m[REF_M_HAT(d, 0) * N + idx]
                       + xyz_t[N + idx] * m[REF_M_HAT(d, 1) * N + idx]
                       + xyz_t[2 * N + idx] * m[REF_M_HAT(d, 2) * N + idx]);
            m[REF_M_HATT(d) * N + idx] = ht;
            m[REF_M_UNHATT(d) * N + idx] = ht * m[REF_M_J * N + idx];
        }

    /* Step 5: interface values for each family f with the central formula:
     * the three hatted f-metrics, hatted f_t, and all nine unhatted metrics. */
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; ++idx) {
        int ijk[3];
        double w[10];
        unpack(g, idx, ijk);
        for (int f = 0; f < 3; ++f) {
            for (int c = 0; c < 3; ++c) {
                field_window(g, m + REF_M_HAT(f, c) * N, ijk, f, -4, 5, w);
                m[REF_M_FHAT(f, c) * N + idx] = face_central(w + 4);
            }
            field_window(g, m + REF_M_HATT(f) * N, ijk, f, -4, 5, w);
            m[REF_M_FHATT(f) * N + idx] = face_central(w + 4);
            for (int e = 0; e < 3; ++e)
                for (int c = 0; c < 3; ++c) {
                    field_window(g, m + REF_M_UNHAT(e, c) * N, ijk, f, -4, 5, w);
                    m[REF_M_FUNHAT(f, e, c) * N + idx] = face_central(w + 4);
                }
        }
    }

    /* Step 6: GCL rate (1/J)_t = -sum_f [I_f hat(f)_t](+1/2) - [..](-1/2). */
    for (long idx = 0; idx < N; ++idx) {
        int ijk[3];
        unpack(g, idx, ijk);
        double s = 0.0;
        for (int f = 0; f < 3; ++f) {
            const double *ft = m + REF_M_FHATT(f) * N;
            s += ft[idx] - ft[neighbour(g, ijk, f, -1, NULL)];
        }
        m[REF_M_INVJT * N + idx] = -s;
    }
    return bad ? 1 : 0;
}

/* MIG4 metrics: the formulae and steps of ref_metrics (Eq. GCL_metrics,
 * Jac-matrix, Jacb2) with D_d = difference of interface values built on IG4
 * gradients (Eq. FP-interp, FP-interp2 with Eq. IG4_grads, as the paper
 * directs for MIG4), and the interface values of the metrics from the same
 * IG4 interpolation. The IG4 system couples a whole line; the derivatives
 * of coordinates and coordinate products are taken, as in ref_metrics, with
 * the coordinate measured from the target cell (the metrics are invariant
 * under a translation), one line per target cell, with the inverse of the
 * cyclic IG4 matrix formed once per line length.
 * Pins: discrete metric identities, freestream, convergence of the metrics,
 * translation invariance.                                                  */
typedef struct {
    const ref_cfg *g;
    int d;              /* line direction                                  */
    const double *fac;  /* per-cell factor (NULL: 1)                       */
    const double *xc;   /* coordinate array (derivative jobs)              */
    double jump;        /* coordinate shift per wrap along d               */
    const double *src;  /* periodic field (interpolation jobs)             */
    double *out;        /* per-cell result                                 */
    int faces;          /* 0: D_d of fac * x, 1: interface values of src   */
    const double *org;  /* derivative jobs on bounded grids: per-cell origin
                         * subtracted from x (NULL: none)                  */
} line_job;

static int line_job_fn(void *ctx, const long *cells)
{
    line_job *jb = (line_job *)ctx;
    const int n = jb->g->n[jb->d];
    double *F = (double *)calloc((size_t)n, sizeof(double));
    double *J = (double *)calloc((size_t)n, sizeof(double));
    double *f = (double *)malloc(sizeof(double) * (n + 1));
    int rc = (!F || !J || !f) ? -1 : 0;
    if (!rc) {
        for (int k = 0; k < n; ++k) {
            if (jb->faces) {
                F[k] = jb->src[cells[k]];
            } else {
                double a = jb->fac ? jb->fac[cells[k]] : 1.0;
                F[k] = a * jb->xc[cells[k]];
                J[k] = a * jb->jump;
            }
        }
        rc = ig4_faces(F, jb->faces ? NULL : J, n, f);
        if (!rc)
            for (int k = 0; k < n; ++k) jb->out[cells[k]] = jb->faces ? f[k + 1] : f[k + 1] - f[k];
    }
    free(F); free(J); free(f);
    return rc;
}

static int run_job(line_job jb) { return for_lines(jb.g, jb.d, line_job_fn, &jb); }

/* Inverse of the cyclic IG4 matrix of order n (1 on the diagonal, alpha on
 * the two neighbours, cyclically: the left-hand side of Eq. IG4_grads on a
 * periodic line), row-major, by Gauss-Jordan elimination with partial
 * pivoting. NULL on allocation failure or a singular matrix.              */
static double *ig4_inverse(int n)
{
    double *A = (double *)calloc((size_t)n * n, sizeof(double));
    double *X = (double *)calloc((size_t)n * n, sizeof(double));
    if (!A || !X) { free(A); free(X); return NULL; }
    for (int k = 0; k < n; ++k) {
        A[k * n + k] += 1.0;
        A[k * n + mod_n(k - 1, n)] += ig4_alpha;
        A[k * n + mod_n(k + 1, n)] += ig4_alpha;
        X[k * n + k] = 1.0;
    }
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int k = c + 1; k < n; ++k)
            if (fabs(A[k * n + c]) > fabs(A[piv * n + c])) piv = k;
        if (A[piv * n + c] == 0.0) { free(A); free(X); return NULL; }
        if (piv != c)
            for (int q = 0; q < n; ++q) {
                double t = A[c * n + q]; A[c * n + q] = A[piv * n + q]; A[piv * n + q] = t;
                t = X[c * n + q]; X[c * n + q] = X[piv * n + q]; X[piv * n + q] = t;
            }
        double p = A[c * n + c];
        for (int q = 0; q < n; ++q) { A[c * n + q] /= p; X[c * n + q] /= p; }
        for (int k = 0; k < n; ++k) {
            if (k == c) continue;
            double f = A[k * n + c];
            if (f == 0.0) continue;
            for (int q = 0; q < n; ++q) { A[k * n + q] -= f * A[c * n + q]; X[k * n + q] -= f * X[c * n + q]; }
        }
    }
    free(A);
    return X;
}

/* D_d of the line F = fac * x (fac NULL: 1) at every cell i, with x measured
 * from cell i: Eq. FP-interp2 applied to G(m) = fac_m ((x_m + w off) - x_i),
 * w the number of periods the index m crossed (the image relative to x_i
 * rounded once, image_rel, as in ref_metrics). G extends with the jump
 * fac * off per period, so its IG4 derivative (Eq. IG4_grads) is that of
 * ig4_ext, here y = Ainv (r - jump rows) + w dj with dj = IG4 of the jump
 * line; the interface values at i -+ 1/2 follow ig4_faces.               */
typedef struct {
    const ref_cfg *g;
    int d;
    const double *fac, *xc;
    double jump;
    double *out;
    const double *ainv;   /* inverse of the cyclic IG4 matrix of order n[d] */
} dloc_job;

static int dloc_fn(void *ctx, const long *cells)
{
    dloc_job *jb = (dloc_job *)ctx;
    const int n = jb->g->n[jb->d];
    double *fa = (double *)malloc(sizeof(double) * n);
    double *x = (double *)malloc(sizeof(double) * n);
    double *J = (double *)calloc((size_t)n, sizeof(double));
    double *dj = (double *)malloc(sizeof(double) * n);
    double *r = (double *)malloc(sizeof(double) * n);
    int rc = (!fa || !x || !J || !dj || !r) ? -1 : 0;
    if (!rc) {
        for (int k = 0; k < n; ++k) {
            fa[k] = jb->fac ? jb->fac[cells[k]] : 1.0;
            x[k] = jb->xc[cells[k]];
            J[k] = fa[k] * jb->jump;
        }
        rc = ig4_ext(J, NULL, n, dj, NULL);
    }
    /* The cyclic system is posed on the period of the extended line that
     * starts at b = i - n/2, so that the target sits mid-period: the values
     * it couples most strongly are then those of the cells around it, all
     * measured from x_i (and small), while the cells half a period away enter
     * through weights of order 0.42^(n/2). The line F(k) = G(b + k) extends
     * with the rotated jump, whose IG4 derivative is dj rotated by b (the
     * circulant inverse is unchanged by the rotation). */
    for (int i = 0; i < n && !rc; ++i) {
        const int b = i - n / 2;
#define GEXT(m) (fa[mod_n((m), n)] * image_rel(x[mod_n((m), n)], floor_div((m), n), jb->jump, x[i]))
        for (int k = 0; k < n; ++k) {
            r[k] = IG4_A * (GEXT(b + k + 1) - GEXT(b + k - 1)) + IG4_B * (GEXT(b + k + 2) - GEXT(b + k - 2));
            for (int s = -1; s <= 1; s += 2)
                r[k] -= ig4_alpha * (double)floor_div(k + s, n) * dj[mod_n(b + k + s, n)];
        }
        double v[5], y[5];  /* cells i-2 .. i+2 */
        for (int q = 0; q < 5; ++q) {
            int m = i - 2 + q - b, row = mod_n(m, n);  /* position in the rotated period */
            double acc = 0.0;
            for (int k = 0; k < n; ++k) acc += jb->ainv[(long)row * n + k] * r[k];
            y[q] = acc + (double)floor_div(m, n) * dj[mod_n(m + b, n)];
            v[q] = GEXT(i - 2 + q);
        }
#undef GEXT
        double face[2];  /* i - 1/2 (cells i-2 .. i+1), i + 1/2 (cells i-1 .. i+2) */
        for (int h = 0; h < 2; ++h) {
            const double *vv = v + h, *gg = y + h;  /* vv[0..3] = cells (i-2+h) .. (i+1+h) */
            double hl = hermite(vv + 1, gg + 1);
            double hr = hermite(vv + 2, gg + 2);
            double left = vv[1] + 0.5 * gg[1] + hl / 12.0;
            double right = vv[2] - 0.5 * gg[2] + hr / 12.0;
            face[h] = 0.5 * (left + right);
        }
        jb->out[cells[i]] = face[1] - face[0];
    }
    free(fa); free(x); free(J); free(dj); free(r);
    return rc;
}

static int metrics_mig4(const ref_cfg *g, const double *xyz, const double *xyz_t, double *m)
{
    const long N = ncell_of(g);
    double *dx = (double *)malloc(sizeof(double) * 9 * N);
    double *ta = (double *)malloc(sizeof(double) * N);
    double *tb = (double *)malloc(sizeof(double) * N);
    double *ainv[3] = {NULL, NULL, NULL};
    int rc = (!dx || !ta || !tb) ? -1 : 0;
    for (int d = 0; d < 3 && !rc; ++d)
        if (!(ainv[d] = ig4_inverse(g->n[d]))) rc = -1;
    /* Step 1: coordinate derivatives D_d(x_c). */
    for (int d = 0; d < 3 && !rc; ++d)
        for (int c = 0; c < 3 && !rc; ++c) {
            dloc_job jb = {g, d, NULL, xyz + c * N, g->off[d][c], dx + (d * 3 + c) * N, ainv[d]};
            rc = for_lines(g, d, dloc_fn, &jb);
        }
    /* Step 2: hat(d)_c = D_d2[(c1)_d1 * c2] - D_d1[(c1)_d2 * c2]; the product
     * shifts by (c1)_d1 * off[d2][c2] when the d2 index wraps.            */
    for (int d = 0; d < 3 && !rc; ++d) {
        int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        for (int c = 0; c < 3 && !rc; ++c) {
            int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            dloc_job ja = {g, d2, dx + (d1 * 3 + c1) * N, xyz + c2 * N, g->off[d2][c2], ta, ainv[d2]};
            dloc_job jc = {g, d1, dx + (d2 * 3 + c1) * N, xyz + c2 * N, g->off[d1][c2], tb, ainv[d1]};
            rc = for_lines(g, d2, dloc_fn, &ja);
            if (!rc) rc = for_lines(g, d1, dloc_fn, &jc);
            if (!rc)
                for (long idx = 0; idx < N; ++idx) m[REF_M_HAT(d, c) * N + idx] = ta[idx] - tb[idx];
        }
    }
    int bad = 0;
    if (!rc) {
        /* Step 3: 1/J = det[D_d x_c]; unhatted d_c = J hat(d)_c. */
        for (long idx = 0; idx < N; ++idx) {
            const double *a = dx + idx;
#define DX(d, c) a[((d) * 3 + (c)) * N]
            double invj = DX(0, 0) * (DX(1, 1) * DX(2, 2) - DX(1, 2) * DX(2, 1))
                        - DX(0, 1) * (DX(1, 0) * DX(2, 2) - DX(1, 2) * DX(2, 0))
                        + DX(0, 2) * (DX(1, 0) * DX(2, 1) - DX(1, 1) * DX(2, 0));
#undef DX
            if (!(invj > 0.0)) bad = 1;
            m[REF_M_INVJ * N + idx] = invj;
            m[REF_M_J * N + idx] = 1.0 / invj;
            for (int d = 0; d < 3; ++d)
                for (int c = 0; c < 3; ++c)
                    m[REF_M_UNHAT(d, c) * N + idx] = m[REF_M_HAT(d, c) * N + idx] / invj;
        }
        /* Step 4: temporal metrics on moving grids. */
        for (long idx = 0; idx < N; ++idx)
            for (int d = 0; d < 3; ++d) {
                double ht = 0.0;
                if (g->moving && xyz_t)
                    ht = -(xyz_t[idx] * m[REF_M_HAT(d, 0) * N + idx]
                           + xyz_t[N + idx] * m[REF_M_HAT(d, 1) * N + idx]
                           + xyz_t[2 * N + idx] * m[REF_M_HAT(d, 2) * N + idx]);
                m[REF_M_HATT(d) * N + idx] = ht;
                m[REF_M_UNHATT(d) * N + idx] = ht * m[REF_M_J * N + idx];
            }
    }
    /* Step 5: interface values per family f with the IG4 interpolation. */
    for (int f = 0; f < 3 && !rc; ++f) {
        int src[13], dst[13], q = 0;
        for (int c = 0; c < 3; ++c) { src[q] = REF_M_HAT(f, c); dst[q++] = REF_M_FHAT(f, c); }
        src[q] = REF_M_HATT(f); dst[q++] = REF_M_FHATT(f);
        for (int e = 0; e < 3; ++e)
            for (int c = 0; c < 3; ++c) { src[q] = REF_M_UNHAT(e, c); dst[q++] = REF_M_FUNHAT(f, e, c); }
        for (q = 0; q < 13 && !rc; ++q) {
            line_job jb = {g, f, NULL, NULL, 0.0, m + (long)src[q] * N, m + (long)dst[q] * N, 1, NULL};
            rc = run_job(jb);
        }
    }
    /* Step 6: GCL rate. */
    if (!rc)
        for (long idx = 0; idx < N; ++idx) {
            int ijk[3];
            unpack(g, idx, ijk);
            double sum = 0.0;
            for (int f = 0; f < 3; ++f) {
                const double *ft = m + REF_M_FHATT(f) * N;
                sum += ft[idx] - ft[neighbour(g, ijk, f, -1, NULL)];
            }
            m[REF_M_INVJT * N + idx] = -sum;
        }
    free(dx); free(ta); free(tb);
    for (int d = 0; d < 3; ++d) free(ainv[d]);
    if (rc) return -1;
    return bad ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Non-periodic boundaries (Sec. 6, App. C).                                */
/* A non-periodic direction d stores REF_NG ghost layers on each side: the  */
/* interior cells are REF_NG .. n[d] - REF_NG - 1. Ghost cells carry        */
/* primitive states set from the boundary type; they have no metrics of     */
/* their own (Sec. 6), so the metrics of interior cells come from App. C    */
/* and every ghost slot holds a copy of the nearest interior value.         */
/* ------------------------------------------------------------------------ */
static int is_bounded(const ref_cfg *g, int d) { return d < g->ndim && g->bc[d][0] != REF_BC_PERIODIC; }

static int any_bounded(const ref_cfg *g)
{
    for (int d = 0; d < 3; ++d)
        if (is_bounded(g, d)) return 1;
    return 0;
}

static int in_interior(const ref_cfg *g, const int ijk[3])
{
    for (int d = 0; d < 3; ++d)
        if (is_bounded(g, d) && (ijk[d] < REF_NG || ijk[d] >= g->n[d] - REF_NG)) return 0;
    return 1;
}

/* Nearest interior cell; for a face slot of family f (face_of >= 0) the
 * f index is clamped to the faces REF_NG - 1 .. n - REF_NG - 1, which hold
 * the interfaces from the low boundary face to the high one.              */
static long clamp_cell(const ref_cfg *g, const int ijk[3], int face_of)
{
    int t[3] = {ijk[0], ijk[1], ijk[2]};
    for (int d = 0; d < 3; ++d) {
        if (!is_bounded(g, d)) continue;
        int lo = (d == face_of) ? REF_NG - 1 : REF_NG, hi = g->n[d] - REF_NG - 1;
        if (t[d] < lo) t[d] = lo;
        if (t[d] > hi) t[d] = hi;
    }
    return cell_index(g, t);
}

/* App. C closures. s = +1 at the low end (v[0] is the boundary cell), s = -1
 * at the high end (the mirror image: derivatives change sign).
 * Second-order one-sided first derivative at the boundary cell.           */
static double one_sided2(const double *v, int s)
{
    return s * (-1.5 * v[0] + 2.0 * v[s] - 0.5 * v[2 * s]);
}

/* Fourth-order partially one-sided derivative at the second cell. The
 * printed stencil runs over cells i .. i+4, which is this formula centred
 * one cell further in; the closure is read as the standard one on cells
 * i-1 .. i+3 (fourth order at cell i; the quadratic-exactness pin fails for
 * the printed placement).                                                 */
static double part_one_sided4(const double *v, int s)
{
    return s * (-0.25 * v[-s] - (5.0 / 6.0) * v[0] + 1.5 * v[s] - 0.5 * v[2 * s] + (1.0 / 12.0) * v[3 * s]);
}

/* Fourth-order central first derivative at the third cell. */
static double central4(const double *v) { return (2.0 / 3.0) * (v[1] - v[-1]) - (1.0 / 12.0) * (v[2] - v[-2]); }

int ref_bline_derivs(const double *v, int m, double *p, double *h)
{
    if (m < 12) return -1;
    /* x': one-sided, partially one-sided, central-4 closures, E6 inside */
    p[0] = one_sided2(v, 1);
    p[1] = part_one_sided4(v + 1, 1);
    p[2] = central4(v + 2);
    for (int c = 3; c <= m - 4; ++c) p[c] = e6(v + c);
    p[m - 3] = central4(v + m - 3);
    p[m - 2] = part_one_sided4(v + m - 2, -1);
    p[m - 1] = one_sided2(v + m - 1, -1);
    /* x'': the same two closures applied to x' at the first two cells; at
     * the third cell the printed formula is the Hermite form of Step-1 with
     * the sign of the second difference flipped, read as the Hermite form
     * (exact for quadratics only with that sign); Hermite inside.         */
    h[0] = one_sided2(p, 1);
    h[1] = part_one_sided4(p + 1, 1);
    for (int c = 2; c <= m - 3; ++c) h[c] = hermite(v + c, p + c);
    h[m - 2] = part_one_sided4(p + m - 2, -1);
    h[m - 1] = one_sided2(p + m - 1, -1);
    return 0;
}

/* Interface values (App. C): the face next to the boundary face takes the
 * inward cell's biased state alone (as printed for i = 1), the next faces
 * the central average of Eq. FP-interp. The boundary face itself, which the
 * appendix leaves out, takes the boundary cell's state extrapolated to it.
 * The high end mirrors the low one.                                       */
int ref_bline_faces(const double *v, int m, double *F)
{
    if (m < 12) return -1;
    double *p = (double *)malloc(sizeof(double) * m), *h = (double *)malloc(sizeof(double) * m);
    if (!p || !h) { free(p); free(h); return -2; }
    ref_bline_derivs(v, m, p, h);
#define LEFT(c) (v[c] + 0.5 * p[c] + h[c] / 12.0)   /* state at c + 1/2 */
#define RIGHT(c) (v[c] - 0.5 * p[c] + h[c] / 12.0)  /* state at c - 1/2 */
    F[0] = RIGHT(0);
    F[1] = RIGHT(1);
    for (int f = 2; f <= m - 2; ++f) F[f] = 0.5 * (LEFT(f - 1) + RIGHT(f));
    F[m - 1] = LEFT(m - 2);
    F[m] = LEFT(m - 1);
#undef LEFT
#undef RIGHT
    free(p); free(h);
    return 0;
}

/* Periodic line extended by F[k + n] = F[k] + J[k] (J may be NULL): the
 * central interface value at a + 1/2 for any integer a. */
static double pline_face_at(const double *F, const double *J, int n, int a)
{
    double w[10];
    for (int q = -4; q <= 5; ++q) {
        int b = a + q, r = mod_n(b, n);
        w[q + 4] = F[r] + (J ? (double)floor_div(b, n) * J[r] : 0.0);
    }
    return face_central(w + 4);
}

/* Line job on a grid with non-periodic directions: along a periodic d the
 * central operators of ref_metrics on the extended line; along a bounded d
 * App. C on the interior cells of the line (ghost entries are left alone). */
static int bjob_fn(void *ctx, const long *cells)
{
    line_job *jb = (line_job *)ctx;
    const ref_cfg *g = jb->g;
    const int n = g->n[jb->d];
    double *F = (double *)calloc((size_t)n + 1, sizeof(double));
    double *J = (double *)calloc((size_t)n + 1, sizeof(double));
    double *f = (double *)calloc((size_t)n + 1, sizeof(double));
    int rc = (!F || !J || !f) ? -1 : 0;
    for (int k = 0; k < n && !rc; ++k) {
        if (jb->faces) {
            F[k] = jb->src[cells[k]];
        } else {
            double a = jb->fac ? jb->fac[cells[k]] : 1.0;
            F[k] = a * jb->xc[cells[k]];
            J[k] = a * jb->jump;
        }
    }
    /* Derivative jobs measure x from the target cell's own coordinate: the
     * metrics are invariant under a translation (the shift multiplies
     * D_d2 D_d1 - D_d1 D_d2 of a coordinate, zero because the operators along
     * different directions commute, App. C rows included), and this keeps
     * round-off at O(eps) on strongly stretched grids. */
    double *G = (double *)calloc((size_t)n + 1, sizeof(double));
    if (!G) rc = -1;
    const int bnd = is_bounded(g, jb->d);
    const int m = n - 2 * REF_NG;
    for (int k = 0; k < n && !rc; ++k) {
        if (bnd && (k < REF_NG || k >= n - REF_NG) && !jb->faces) continue;
        const double *V = F;
        if (!jb->faces && jb->org) {
            const double o = jb->org[cells[k]];
            for (int q = 0; q < n; ++q) G[q] = (jb->fac ? jb->fac[cells[q]] : 1.0) * (jb->xc[cells[q]] - o);
            V = G;
        }
        if (!bnd && !jb->faces && jb->org) {
            /* periodic direction: the window of the extended line around k,
             * each image measured from the target with one rounding */
            const double o = jb->org[cells[k]];
            double w[11];
            for (int q = -5; q <= 5; ++q) {
                int b = k + q, r = mod_n(b, n);
                w[q + 5] = (jb->fac ? jb->fac[cells[r]] : 1.0) * image_rel(jb->xc[cells[r]], floor_div(b, n), jb->jump, o);
            }
            jb->out[cells[k]] = dcomp(w + 5);
        } else if (!bnd) {
            double up = pline_face_at(V, jb->faces ? NULL : J, n, k);
            jb->out[cells[k]] = jb->faces ? up : up - pline_face_at(V, J, n, k - 1);
        } else if (jb->faces) {
            if (k == 0) {
                rc = ref_bline_faces(V + REF_NG, m, f);
                for (int q = 0; q <= m && !rc; ++q) jb->out[cells[REF_NG - 1 + q]] = f[q];
            }
        } else {
            rc = ref_bline_faces(V + REF_NG, m, f);
            if (!rc) jb->out[cells[k]] = f[k - REF_NG + 1] - f[k - REF_NG];
        }
    }
    free(F); free(J); free(f); free(G);
    return rc;
}

static int run_bjob(line_job jb) { return for_lines(jb.g, jb.d, bjob_fn, &jb); }

/* Metrics of a static grid with non-periodic directions: the steps of
 * ref_metrics (Eq. GCL_metrics, Jac-matrix, interp-formulae) with App. C
 * along the bounded directions, lines processed whole in the coordinates
 * as given; then every ghost slot copies the nearest interior one.
 * Pins: exactness on affine grids, discrete metric identities and
 * freestream with the boundary faces included, and the App. C line pins. */
static int metrics_bounded(const ref_cfg *g, const double *xyz, const double *xyz_t, double *m)
{
    if (g->moving || xyz_t || g->scheme != REF_SCHEME_MEG6) return -2;
    for (int d = 0; d < 3; ++d)
        if (is_bounded(g, d) && g->n[d] - 2 * REF_NG < 12) return -2;
    const long N = ncell_of(g);
    double *dx = (double *)calloc((size_t)9 * N, sizeof(double));
    double *ta = (double *)calloc((size_t)N, sizeof(double));
    double *tb = (double *)calloc((size_t)N, sizeof(double));
    int rc = (!dx || !ta || !tb) ? -1 : 0;
    /* Step 1: coordinate derivatives D_d(x_c). */
    for (int d = 0; d < 3 && !rc; ++d)
        for (int c = 0; c < 3 && !rc; ++c) {
            line_job jb = {g, d, NULL, xyz + c * N, g->off[d][c], NULL, dx + (d * 3 + c) * N, 0, xyz + c * N};
            rc = run_bjob(jb);
        }
    /* Step 2: hat(d)_c = D_d2[(c1)_d1 * c2] - D_d1[(c1)_d2 * c2]. */
    for (int d = 0; d < 3 && !rc; ++d) {
        int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        for (int c = 0; c < 3 && !rc; ++c) {
            int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            line_job ja = {g, d2, dx + (d1 * 3 + c1) * N, xyz + c2 * N, g->off[d2][c2], NULL, ta, 0, xyz + c2 * N};
            line_job jc = {g, d1, dx + (d2 * 3 + c1) * N, xyz + c2 * N, g->off[d1][c2], NULL, tb, 0, xyz + c2 * N};
            rc = run_bjob(ja);
            if (!rc) rc = run_bjob(jc);
            if (!rc)
                for (long idx = 0; idx < N; ++idx) m[REF_M_HAT(d, c) * N + idx] = ta[idx] - tb[idx];
        }
    }
    int bad = 0;
    if (!rc) {
        /* Step 3: 1/J = det[D_d x_c]; unhatted d_c = J hat(d)_c. Step 4:
         * static grid, no temporal metrics. */
        for (long idx = 0; idx < N; ++idx) {
            int ijk[3];
            unpack(g, idx, ijk);
            const double *a = dx + idx;
#define DX(d, c) a[((d) * 3 + (c)) * N]
            double invj = DX(0, 0) * (DX(1, 1) * DX(2, 2) - DX(1, 2) * DX(2, 1))
                        - DX(0, 1) * (DX(1, 0) * DX(2, 2) - DX(1, 2) * DX(2, 0))
                        + DX(0, 2) * (DX(1, 0) * DX(2, 1) - DX(1, 1) * DX(2, 0));
#undef DX
            if (in_interior(g, ijk) && !(invj > 0.0)) bad = 1;
            m[REF_M_INVJ * N + idx] = invj;
            m[REF_M_J * N + idx] = 1.0 / invj;
            for (int d = 0; d < 3; ++d) {
                for (int c = 0; c < 3; ++c)
                    m[REF_M_UNHAT(d, c) * N + idx] = m[REF_M_HAT(d, c) * N + idx] / invj;
                m[REF_M_HATT(d) * N + idx] = 0.0;
                m[REF_M_UNHATT(d) * N + idx] = 0.0;
            }
            m[REF_M_INVJT * N + idx] = 0.0;
        }
    }
    /* Step 5: interface values per family f. */
    for (int f = 0; f < 3 && !rc; ++f) {
        int src[13], dst[13], q = 0;
        for (int c = 0; c < 3; ++c) { src[q] = REF_M_HAT(f, c); dst[q++] = REF_M_FHAT(f, c); }
        src[q] = REF_M_HATT(f); dst[q++] = REF_M_FHATT(f);
        for (int e = 0; e < 3; ++e)
            for (int c = 0; c < 3; ++c) { src[q] = REF_M_UNHAT(e, c); dst[q++] = REF_M_FUNHAT(f, e, c); }
        for (q = 0; q < 13 && !rc; ++q) {
            line_job jb = {g, f, NULL, NULL, 0.0, m + (long)src[q] * N, m + (long)dst[q] * N, 1, NULL};
            rc = run_bjob(jb);
        }
    }
    /* Step 6: ghost slots copy the nearest interior (or boundary-face) value. */
    if (!rc)
        for (long idx = 0; idx < N; ++idx) {
            int ijk[3];
            unpack(g, idx, ijk);
            long cc = clamp_cell(g, ijk, -1);
            if (cc != idx)
                for (int sl = 0; sl < 27; ++sl) m[(long)sl * N + idx] = m[(long)sl * N + cc];
            for (int f = 0; f < 3; ++f) {
                long fc = clamp_cell(g, ijk, f);
                if (fc == idx) continue;
                for (int sl = REF_M_FHAT(f, 0); sl < REF_M_FHAT(f, 0) + 13; ++sl)
                    m[(long)sl * N + idx] = m[(long)sl * N + fc];
            }
        }
    free(dx); free(ta); free(tb);
    if (rc) return rc;
    return bad ? 1 : 0;
}

/* Ghost cells of Q (Sec. 6; the table of ghost-cell expressions is not in
 * the text available, so the standard forms are used): Dirichlet inflow
 * ghosts keep the state stored in them; zero-gradient outflow ghosts copy
 * the boundary cell of their line; slip-wall ghosts mirror the interior
 * cell at the same depth with the momentum component along the unit normal
 * of the boundary face reversed. Directions are filled in order over the
 * full extent of the others, so corner ghosts take the later direction's
 * rule applied to the earlier one's values.
 * Pins: a wall (mirror) or Dirichlet boundary on an affine grid reproduces
 * the periodic residual of the mirrored / extended flow.                 */
void ref_apply_bc(const ref_cfg *g, const double *m, double *Q)
{
    const long N = ncell_of(g);
    const int nv = g->ndim + 2;
    for (int d = 0; d < g->ndim; ++d) {
        if (!is_bounded(g, d)) continue;
        const int n = g->n[d];
        for (long idx = 0; idx < N; ++idx) {
            int ijk[3];
            unpack(g, idx, ijk);
            int side = -1, depth = 0;
            if (ijk[d] < REF_NG) { side = 0; depth = REF_NG - 1 - ijk[d]; }
            else if (ijk[d] >= n - REF_NG) { side = 1; depth = ijk[d] - (n - REF_NG); }
            if (side < 0) continue;
            const int type = g->bc[d][side];
            if (type == REF_BC_INFLOW) continue;
            int src[3] = {ijk[0], ijk[1], ijk[2]}, face[3] = {ijk[0], ijk[1], ijk[2]};
            if (type == REF_BC_OUTFLOW) src[d] = side ? n - REF_NG - 1 : REF_NG;
            else src[d] = side ? n - REF_NG - 1 - depth : REF_NG + depth;
            face[d] = side ? n - REF_NG - 1 : REF_NG - 1;
            const long sc = cell_index(g, src);
            for (int v = 0; v < nv; ++v) Q[v * N + idx] = Q[v * N + sc];
            if (type == REF_BC_WALL) {
                const long fc = cell_index(g, face);
                double nr[3], nn = 0.0, mn = 0.0;
                for (int c = 0; c < 3; ++c) { nr[c] = m[REF_M_FHAT(d, c) * N + fc]; nn += nr[c] * nr[c]; }
                nn = sqrt(nn);
                for (int c = 0; c < g->ndim; ++c) { nr[c] /= nn; mn += Q[(1 + c) * N + idx] * nr[c]; }
                for (int c = 0; c < g->ndim; ++c) Q[(1 + c) * N + idx] -= 2.0 * mn * nr[c];
            }
        }
    }
}

/* Non-freestream-preserving metrics of App. D (negative control only):
 * hat(d)_c = (c1)_d1 (c2)_d2 - (c1)_d2 (c2)_d1 from fourth-order central
 * derivatives (Eq. 4thorder-grads), interface values from Eq. interp-formulae
 * with that derivative in place of E6. The printed zeta_y entry has a zeta
 * where the cyclic pattern has xi; the cyclic form is used. Static grids. */
static double c4(const double *v) { return (2.0 / 3.0) * (v[1] - v[-1]) - (1.0 / 12.0) * (v[2] - v[-2]); }

/* Interface value at +1/2 with the fourth-order derivative: derivatives at
 * the cells -1 .. 2 of the window reach two cells further, so v[-3 .. 4]. */
static double face_central_c4(const double *v)
{
    double gv[4], h[2];
    for (int q = -1; q <= 2; ++q) gv[q + 1] = c4(v + q);
    h[0] = hermite(v, gv + 1);
    h[1] = hermite(v + 1, gv + 2);
    return 0.5 * ((v[0] + 0.5 * gv[1] + h[0] / 12.0) + (v[1] - 0.5 * gv[2] + h[1] / 12.0));
}

int ref_metrics_nonfp(const ref_cfg *g, const double *xyz, double *m)
{
    const long N = ncell_of(g);
    double *dx = (double *)malloc(sizeof(double) * 9 * N);
    if (!dx) return -1;
    int bad = 0;
    for (long idx = 0; idx < N; ++idx) {
        int ijk[3];
        double w[5];
        unpack(g, idx, ijk);
        for (int d = 0; d < 3; ++d)
            for (int c = 0; c < 3; ++c) {
                for (int q = -2; q <= 2; ++q) w[q + 2] = coord_ext(g, xyz, ijk, d, q, c);
                dx[(d * 3 + c) * N + idx] = c4(w + 2);
            }
    }
    for (long idx = 0; idx < N; ++idx) {
        const double *a = dx + idx;
#define DX(d, c) a[((d) * 3 + (c)) * N]
        for (int d = 0; d < 3; ++d) {
            int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
            for (int c = 0; c < 3; ++c) {
                int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
                m[REF_M_HAT(d, c) * N + idx] = DX(d1, c1) * DX(d2, c2) - DX(d2, c1) * DX(d1, c2);
            }
        }
        double invj = DX(0, 0) * (DX(1, 1) * DX(2, 2) - DX(1, 2) * DX(2, 1))
                    - DX(0, 1) * (DX(1, 0) * DX(2, 2) - DX(1, 2) * DX(2, 0))
                    + DX(0, 2) * (DX(1, 0) * DX(2, 1) - DX(1, 1) * DX(2, 0));
#undef DX
        if (!(invj > 0.0)) bad = 1;
        m[REF_M_INVJ * N + idx] = invj;
        m[REF_M_J * N + idx] = 1.0 / invj;
        for (int d = 0; d < 3; ++d) {
            for (int c = 0; c < 3; ++c)
                m[REF_M_UNHAT(d, c) * N + idx] = m[REF_M_HAT(d, c) * N + idx] / invj;
            m[REF_M_HATT(d) * N + idx] = 0.0;
            m[REF_M_UNHATT(d) * N + idx] = 0.0;
        }
        m[REF_M_INVJT * N + idx] = 0.0;
    }
    free(dx);
    for (long idx = 0; idx < N; ++idx) {
        int ijk[3];
        double w[8];
        unpack(g, idx, ijk);
        for (int f = 0; f < 3; ++f) {
            for (int c = 0; c < 3; ++c) {
                field_window(g, m + REF_M_HAT(f, c) * N, ijk, f, -3, 4, w);
                m[REF_M_FHAT(f, c) * N + idx] = face_central_c4(w + 3);
            }
            m[REF_M_FHATT(f) * N + idx] = 0.0;
            for (int e = 0; e < 3; ++e)
                for (int c = 0; c < 3; ++c) {
                    field_window(g, m + REF_M_UNHAT(e, c) * N, ijk, f, -3, 4, w);
                    m[REF_M_FUNHAT(f, e, c) * N + idx] = face_central_c4(w + 3);
                }
        }
    }
    return bad ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Thermodynamics (Sec. 2)                                                  */
/* ------------------------------------------------------------------------ */
typedef struct { double r, u, v, w, p, T; } prim_t;

static prim_t primitive(const ref_cfg *g, const double *Q, long idx)
{
    const long N = ncell_of(g);
    prim_t s;
    int nv = g->ndim + 2;
    s.r = Q[idx];
    s.u = Q[N + idx] / s.r;
    s.v = Q[2 * N + idx] / s.r;
    s.w = (nv == 5) ? Q[3 * N + idx] / s.r : 0.0;
    double E = Q[(nv - 1) * N + idx];
    s.p = (g->gamma - 1.0) * (E - 0.5 * s.r * (s.u * s.u + s.v * s.v + s.w * s.w));
    s.T = g->gamma * g->Mref * g->Mref * s.p / s.r;
    return s;
}

/* Sutherland's law, normalised to 1 at T = 1, divided by Re. */
static double viscosity(const ref_cfg *g, double T)
{
    return T * sqrt(T) * (1.0 + g->suth) / (T + g->suth) / g->Re;
}

/* ------------------------------------------------------------------------ */
/* Eigenvectors of App. A (Eq. for R and R^-1) with a unit normal.          */
/* Pins: R R^-1 = I and R^-1 B R = diag(U - a, U, U, U, U + a) with the     */
/* primitive-form matrix B of App. A.                                       */
/* ------------------------------------------------------------------------ */
void ref_eigvec(const double nrm[3], double rho, double a, double R[25], double Rinv[25])
{
    double nx = nrm[0], ny = nrm[1], nz = nrm[2];
    double a2 = a * a, ra = rho * a;
    double Rm[25] = {
        1.0 / (2.0 * a2), nx / a2, nz / a2, -ny / a2, 1.0 / (2.0 * a2),
        -nx / (2.0 * ra), 0.0, -ny, -nz, nx / (2.0 * ra),
        -ny / (2.0 * ra), -nz, nx, 0.0, ny / (2.0 * ra),
        -nz / (2.0 * ra), ny, 0.0, nx, nz / (2.0 * ra),
        0.5, 0.0, 0.0, 0.0, 0.5};
    double Li[25] = {
        0.0, -nx * ra, -ny * ra, -nz * ra, 1.0,
        nx * a2, 0.0, -nz, ny, -nx,
        nz * a2, -ny, nx, 0.0, -nz,
        -ny * a2, -nz, 0.0, nx, ny,
        0.0, nx * ra, ny * ra, nz * ra, 1.0};
    memcpy(R, Rm, sizeof Rm);
    memcpy(Rinv, Li, sizeof Li);
}

static void matvec5(const double A[25], const double x[5], double y[5])
{
    for (int r = 0; r < 5; ++r) {
        double s = 0.0;
        for (int c = 0; c < 5; ++c) s += A[r * 5 + c] * x[c];
        y[r] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Improved MP limiter of App. E for one characteristic component, written  */
/* for the left state at i+1/2; the right state calls it with the stencil   */
/* reflected about i+1 (wm1 <- W[i+2], w0 <- W[i+1], wp1 <- W[i], ...).      */
/* d* are the gradient-based curvatures d_k (= R^-1 P''_k).                 */
/* ------------------------------------------------------------------------ */
static double sgn(double x) { return (x > 0.0) - (x < 0.0); }
static double minmod(double a, double b) { return 0.5 * (sgn(a) + sgn(b)) * fmin(fabs(a), fabs(b)); }
static double min3(double a, double b, double c) { return fmin(a, fmin(b, c)); }
static double max3(double a, double b, double c) { return fmax(a, fmax(b, c)); }

double ref_mp_limit(double wm1, double w0, double wp1, double dm1, double d0,
                    double dp1, double wface, double alpha, double beta)
{
    double wmp = w0 + minmod(wp1 - w0, beta * (w0 - wm1));
    if ((wface - w0) * (wface - wmp) <= 1e-20) return wface;
    double dm_plus = minmod(d0, dp1);   /* d^M at i+1/2 */
    double dm_minus = minmod(dm1, d0);  /* d^M at i-1/2 */
    double wmd = 0.5 * (w0 + wp1) - 0.5 * dm_plus;
    double wul = w0 + alpha * (w0 - wm1);
    double wlc = 0.5 * (3.0 * w0 - wm1) + (4.0 / 3.0) * dm_minus;
    double wmin = fmax(min3(w0, wp1, wmd), min3(w0, wul, wlc));
    double wmax = fmin(max3(w0, wp1, wmd), max3(w0, wul, wlc));
    return wface + minmod(wmin - wface, wmax - wface);
}

/* ------------------------------------------------------------------------ */
/* Inviscid flux vector (Eq. inv_fluxes) and curvilinear HLLC (Sec. 5.1.1). */
/* nt_n = (hat xi_t, hat xi_x, hat xi_y, hat xi_z) at the interface.        */
/* Pins: F(P, P) = F(P); textbook Cartesian HLLC for n = (1,0,0), n_t = 0;  */
/* rotation and scaling invariance; Rankine-Hugoniot across S*.             */
/* ------------------------------------------------------------------------ */
void ref_euler_flux(const double P[5], const double nt_n[4], double gamma, double F[5])
{
    double r = P[0], u = P[1], v = P[2], w = P[3], p = P[4];
    double U = nt_n[0] + nt_n[1] * u + nt_n[2] * v + nt_n[3] * w;
    double E = p / (gamma - 1.0) + 0.5 * r * (u * u + v * v + w * w);
    F[0] = r * U;
    F[1] = r * u * U + nt_n[1] * p;
    F[2] = r * v * U + nt_n[2] * p;
    F[3] = r * w * U + nt_n[3] * p;
    F[4] = (E + p) * U - nt_n[0] * p;
}

static void star_state(const double P[5], double E, double U, double SK, double Ss,
                       const double nt_n[4], double nn, double Qs[5])
{
    double r = P[0], u = P[1], v = P[2], w = P[3], p = P[4];
    double nt = nt_n[0], nx = nt_n[1], ny = nt_n[2], nz = nt_n[3];
    double fac = r * (SK - U) / (SK - Ss);
    Qs[0] = fac;
    Qs[1] = fac * (nx * (Ss - nt) + (ny * ny + nz * nz) * u - ny * nx * v - nz * nx * w) / nn;
    Qs[2] = fac * (ny * (Ss - nt) - nx * ny * u + (nx * nx + nz * nz) * v - nz * ny * w) / nn;
    Qs[3] = fac * (nz * (Ss - nt) - nx * nz * u - ny * nz * v + (nx * nx + ny * ny) * w) / nn;
    Qs[4] = fac * (E / r + (Ss - U) * ((Ss - nt) / nn + p / (r * (SK - U))));
}

void ref_hllc(const double PL[5], const double PR[5], const double nt_n[4], double gamma, double F[5])
{
    double nt = nt_n[0], nx = nt_n[1], ny = nt_n[2], nz = nt_n[3];
    double nn = nx * nx + ny * ny + nz * nz, sn = sqrt(nn);
    double UL = nt + nx * PL[1] + ny * PL[2] + nz * PL[3];
    double UR = nt + nx * PR[1] + ny * PR[2] + nz * PR[3];
    double cL = sqrt(gamma * PL[4] / PL[0]), cR = sqrt(gamma * PR[4] / PR[0]);
    double SL = fmin(UL - cL * sn, UR - cR * sn);
    double SR = fmax(UL + cL * sn, UR + cR * sn);
    double Ss = (PR[0] * UR * (SR - UR) - PL[0] * UL * (SL - UL) + (PL[4] - PR[4]) * nn)
              / (PR[0] * (SR - UR) - PL[0] * (SL - UL));
    double FL[5], FR[5];
    ref_euler_flux(PL, nt_n, gamma, FL);
    ref_euler_flux(PR, nt_n, gamma, FR);
    if (0.0 <= SL) { memcpy(F, FL, sizeof FL); return; }
    if (0.0 >= SR) { memcpy(F, FR, sizeof FR); return; }
    const double *P = (0.0 <= Ss) ? PL : PR;
    const double *FK = (0.0 <= Ss) ? FL : FR;
    double SK = (0.0 <= Ss) ? SL : SR;
    double U = (0.0 <= Ss) ? UL : UR;
    double E = P[4] / (gamma - 1.0) + 0.5 * P[0] * (P[1] * P[1] + P[2] * P[2] + P[3] * P[3]);
    double QK[5] = {P[0], P[0] * P[1], P[0] * P[2], P[0] * P[3], E};
    double Qs[5];
    star_state(P, E, U, SK, Ss, nt_n, nn, Qs);
    for (int q = 0; q < 5; ++q) F[q] = FK[q] + SK * (Qs[q] - QK[q]);
}

/* ------------------------------------------------------------------------ */
/* Cell gradients (Step-1, Sec. 5.1; reused by Sec. 5.2 and the sensor).    */
/* grad[(d * 4 + s) * N + cell], s = u, v, w, T; E6 along d.                */
/* ------------------------------------------------------------------------ */
/* IG4 derivative along d of a periodic cell field, every line. */
typedef struct { const ref_cfg *g; int d; const double *src; double *out; } grad_job;

static int grad_job_fn(void *ctx, const long *cells)
{
    grad_job *jb = (grad_job *)ctx;
    const int n = jb->g->n[jb->d];
    double *F = (double *)calloc((size_t)n, sizeof(double));
    double *y = (double *)malloc(sizeof(double) * n);
    int rc = (!F || !y) ? -1 : 0;
    if (!rc) {
        for (int k = 0; k < n; ++k) F[k] = jb->src[cells[k]];
        rc = ig4_ext(F, NULL, n, y, NULL);
        if (!rc) for (int k = 0; k < n; ++k) jb->out[cells[k]] = y[k];
    }
    free(F); free(y);
    return rc;
}

/* Primitive fields (rho, u, v, w, p, T), 6 * N. */
static void primitive_fields(const ref_cfg *g, const double *Q, double *pr)
{
    const long N = ncell_of(g);
    for (long idx = 0; idx < N; ++idx) {
        prim_t s = primitive(g, Q, idx);
        pr[idx] = s.r; pr[N + idx] = s.u; pr[2 * N + idx] = s.v;
        pr[3 * N + idx] = s.w; pr[4 * N + idx] = s.p; pr[5 * N + idx] = s.T;
    }
}

/* MIG4: IG4 derivatives of all six primitive fields along every direction,
 * pg[(d * 6 + s) * N], s = rho, u, v, w, p, T. */
static int ig4_prim_grads(const ref_cfg *g, const double *Q, double *pg)
{
    const long N = ncell_of(g);
    double *pr = (double *)malloc(sizeof(double) * 6 * N);
    if (!pr) return -1;
    primitive_fields(g, Q, pr);
    int rc = 0;
    for (int d = 0; d < 3 && !rc; ++d)
        for (int q = 0; q < 6 && !rc; ++q) {
            grad_job jb = {g, d, pr + q * N, pg + (d * 6 + q) * N};
            rc = for_lines(g, d, grad_job_fn, &jb);
        }
    free(pr);
    return rc;
}

void ref_gradients(const ref_cfg *g, const double *Q, double *grad)
{
    const long N = ncell_of(g);
    if (g->scheme == REF_SCHEME_MIG4) {
        /* (u, v, w, T) gradients from the IG4 primitive gradients, whose
         * fields are ordered (rho, u, v, w, p, T) */
        static const int from[4] = {1, 2, 3, 5};
        double *pg = (double *)malloc(sizeof(double) * 18 * N);
        if (pg && !ig4_prim_grads(g, Q, pg))
            for (int d = 0; d < 3; ++d)
                for (int s = 0; s < 4; ++s)
                    memcpy(grad + (d * 4 + s) * N, pg + (d * 6 + from[s]) * N, sizeof(double) * N);
        free(pg);
        return;
    }
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; ++idx) {
        int ijk[3];
        unpack(g, idx, ijk);
        for (int d = 0; d < 3; ++d) {
            double wu[7], wv[7], ww[7], wT[7];
            for (int q = -3; q <= 3; ++q) {
                prim_t s = primitive(g, Q, neighbour(g, ijk, d, q, NULL));
                wu[q + 3] = s.u; wv[q + 3] = s.v; ww[q + 3] = s.w; wT[q + 3] = s.T;
            }
            grad[(d * 4 + 0) * N + idx] = e6(wu + 3);
            grad[(d * 4 + 1) * N + idx] = e6(wv + 3);
            grad[(d * 4 + 2) * N + idx] = e6(ww + 3);
            grad[(d * 4 + 3) * N + idx] = e6(wT + 3);
        }
    }
}

/* Ducros sensor from the cell gradients and the cell (unhatted) metrics:
 * du_a/dx_b = sum_d (d_{x_b}) du_a/dd. Not part of the paper.            */
void ref_sensor(const ref_cfg *g, const double *m, const double *grad, double *theta)
{
    const long N = ncell_of(g);
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; ++idx) {
        double G[3][3]; /* G[a][b] = d u_a / d x_b */
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int d = 0; d < 3; ++d)
                    s += m[REF_M_UNHAT(d, b) * N + idx] * grad[(d * 4 + a) * N + idx];
                G[a][b] = s;
            }
        double div = G[0][0] + G[1][1] + G[2][2];
        double wx = G[2][1] - G[1][2], wy = G[0][2] - G[2][0], wz = G[1][0] - G[0][1];
        double d2 = div * div;
        theta[idx] = d2 / (d2 + (wx * wx + wy * wy + wz * wz) + 1e-30);
    }
}

/* ------------------------------------------------------------------------ */
/* Interface flux along direction f at the face between cell idx and its +1 */
/* neighbour: Steps 1-6 of Sec. 5.1 and Steps 1-4 of Sec. 5.2.             */
/* ------------------------------------------------------------------------ */
static int face_flux(const ref_cfg *g, const double *m, const double *Q, const double *grad,
                     const double *pgrad, const double *theta, int f, const int ijk[3], long idx,
                     double phi[5])
{
    const long N = ncell_of(g);
    /* primitives on the line, offsets -5 .. +6 about cell i */
    double P[12][5], T[12];
    long nb[12];
    for (int q = -5; q <= 6; ++q) {
        nb[q + 5] = neighbour(g, ijk, f, q, NULL);
        prim_t s = primitive(g, Q, nb[q + 5]);
        P[q + 5][0] = s.r; P[q + 5][1] = s.u; P[q + 5][2] = s.v; P[q + 5][3] = s.w; P[q + 5][4] = s.p;
        T[q + 5] = s.T;
    }
    /* Step-1: first derivatives at offsets -2..3 (E6 for MEG6; the IG4 line
     * derivatives for MIG4), Hermite second derivatives at -1..2 */
    double D1[6][5], D2[4][5];
    for (int q = -2; q <= 3; ++q)
        for (int s = 0; s < 5; ++s) {
            if (pgrad) {
                D1[q + 2][s] = pgrad[(f * 6 + s) * N + nb[q + 5]];
                continue;
            }
            double w[7];
            for (int t = -3; t <= 3; ++t) w[t + 3] = P[q + t + 5][s];
            D1[q + 2][s] = e6(w + 3);
        }
    for (int q = -1; q <= 2; ++q)
        for (int s = 0; s < 5; ++s) {
            double w[3] = {P[q + 4][s], P[q + 5][s], P[q + 6][s]};
            double gv[3] = {D1[q + 1][s], D1[q + 2][s], D1[q + 3][s]};
            D2[q + 1][s] = hermite(w + 1, gv + 1);
        }
#define PC(q) P[(q) + 5]
#define P1(q) D1[(q) + 2]
#define P2(q) D2[(q) + 1]

    double nt_n[4] = {m[REF_M_FHATT(f) * N + idx], m[REF_M_FHAT(f, 0) * N + idx],
                      m[REF_M_FHAT(f, 1) * N + idx], m[REF_M_FHAT(f, 2) * N + idx]};

    int limited = 0;
    if (g->limiter == REF_LIM_MP) limited = 1;
    else if (g->limiter == REF_LIM_DUCROS)
        limited = fmax(theta[idx], theta[nb[6]]) > g->theta_c;

    double PL[5], PR[5];
    if (limited) {
        /* Step-2: project P, P', P'' with the left eigenvectors of the
         * averaged state and the unit interface normal.                  */
        double rb = 0.5 * (PC(0)[0] + PC(1)[0]);
        double pb = 0.5 * (PC(0)[4] + PC(1)[4]);
        double ab = sqrt(g->gamma * pb / rb);
        double nn = sqrt(nt_n[1] * nt_n[1] + nt_n[2] * nt_n[2] + nt_n[3] * nt_n[3]);
        double nu[3] = {nt_n[1] / nn, nt_n[2] / nn, nt_n[3] / nn};
        double R[25], Ri[25];
        ref_eigvec(nu, rb, ab, R, Ri);
        double W[4][5], W1[2][5], W2[4][5];
        for (int q = -1; q <= 2; ++q) { matvec5(Ri, PC(q), W[q + 1]); matvec5(Ri, P2(q), W2[q + 1]); }
        for (int q = 0; q <= 1; ++q) matvec5(Ri, P1(q), W1[q]);
        /* Step-3 and Step-4 per characteristic field. */
        double WL[5], WR[5];
        for (int s = 0; s < 5; ++s) {
            double wl = W[1][s] + 0.5 * W1[0][s] + (1.0 / 12.0) * W2[1][s];
            double wr = W[2][s] - 0.5 * W1[1][s] + (1.0 / 12.0) * W2[2][s];
            WL[s] = ref_mp_limit(W[0][s], W[1][s], W[2][s], W2[0][s], W2[1][s], W2[2][s],
                                 wl, g->alpha_mp, g->beta_mp);
            WR[s] = ref_mp_limit(W[3][s], W[2][s], W[1][s], W2[3][s], W2[2][s], W2[1][s],
                                 wr, g->alpha_mp, g->beta_mp);
        }
        /* Step-5: back to primitive variables. */
        matvec5(R, WL, PL);
        matvec5(R, WR, PR);
    } else {
        /* Unlimited states of Eq. vanleer-poly directly in primitive form
         * (identical to projecting and back-projecting, as R R^-1 = I). */
        for (int s = 0; s < 5; ++s) {
            PL[s] = PC(0)[s] + 0.5 * P1(0)[s] + (1.0 / 12.0) * P2(0)[s];
            PR[s] = PC(1)[s] - 0.5 * P1(1)[s] + (1.0 / 12.0) * P2(1)[s];
        }
    }
    if (g->ndim == 2) { PL[3] = 0.0; PR[3] = 0.0; }
    int bad = !(PL[0] > 0.0 && PL[4] > 0.0 && PR[0] > 0.0 && PR[4] > 0.0);

    /* Step-6: HLLC. */
    double F[5];
    ref_hllc(PL, PR, nt_n, g->gamma, F);

    double Fv[5] = {0, 0, 0, 0, 0};
    if (g->viscous) {
        /* Sec. 5.2, Step-1: interface gradients of (u, v, w, T). */
        double dT[2], wT[7];
        for (int q = 0; q <= 1; ++q) {
            if (pgrad) {
                dT[q] = pgrad[(f * 6 + 5) * N + nb[q + 5]];
                continue;
            }
            for (int t = -3; t <= 3; ++t) wT[t + 3] = T[q + t + 5];
            dT[q] = e6(wT + 3);
        }
        double sc[2][4] = {{PC(0)[1], PC(0)[2], PC(0)[3], T[5]}, {PC(1)[1], PC(1)[2], PC(1)[3], T[6]}};
        double sd[2][4] = {{P1(0)[1], P1(0)[2], P1(0)[3], dT[0]}, {P1(1)[1], P1(1)[2], P1(1)[3], dT[1]}};
        double sL[4], sR[4], gf[3][4]; /* gf[e][s]: d s / d e at the face */
        for (int s = 0; s < 4; ++s) {
            sL[s] = sc[0][s] + 0.5 * sd[0][s];
            sR[s] = sc[1][s] - 0.5 * sd[1][s];
            gf[f][s] = 0.5 * (sd[0][s] + sd[1][s]) + 0.5 * g->alpha_d * (sR[s] - sL[s]);
            for (int e = 0; e < 3; ++e) {
                if (e == f) continue;
                gf[e][s] = 0.5 * (grad[(e * 4 + s) * N + idx] + grad[(e * 4 + s) * N + nb[6]]);
            }
        }
        /* Step-2: chain rule with interface unhatted metrics. */
        double Dx[4][3]; /* Dx[s][b] = d s / d x_b */
        for (int s = 0; s < 4; ++s)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int e = 0; e < 3; ++e) acc += m[REF_M_FUNHAT(f, e, b) * N + idx] * gf[e][s];
                Dx[s][b] = acc;
            }
        /* Step-3: stresses and heat flux at the interface. */
        double Tf = 0.5 * (sL[3] + sR[3]);
        double mu = viscosity(g, Tf);
        double lam = -2.0 / 3.0 * mu;
        double kap = mu / ((g->gamma - 1.0) * g->Mref * g->Mref * g->Pr);
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
        /* Step-4: interface viscous flux with hatted interface metrics. */
        double hx = nt_n[1], hy = nt_n[2], hz = nt_n[3];
        Fv[1] = hx * txx + hy * txy + hz * txz;
        Fv[2] = hx * txy + hy * tyy + hz * tyz;
        Fv[3] = hx * txz + hy * tyz + hz * tzz;
        Fv[4] = hx * bx + hy * by + hz * bz;
    }
    for (int s = 0; s < 5; ++s) {
        phi[s] = F[s] - Fv[s];
        if (!isfinite(phi[s])) bad = 1;
    }
    return bad;
#undef PC
#undef P1
#undef P2
}

/* ------------------------------------------------------------------------ */
/* Right-hand side (Sec. 3): Res = -sum_f [Phi(+1/2) - Phi(-1/2)], the three */
/* directions accumulated in the order xi, eta, zeta.                       */
/* Pins: freestream, conservation, accuracy order, exact Riemann solution.  */
/* Returns 1 if a reconstructed or cell state is non-physical.             */
/* ------------------------------------------------------------------------ */
int ref_rhs(const ref_cfg *g, const double *m, const double *Q, double *res)
{
    const long N = ncell_of(g);
    const int nv = g->ndim + 2;
    const int nf = g->ndim;
    const int bnd = any_bounded(g);
    const double *Qs = Q;  /* the state as given (sponge term) */
    double *Qb = NULL;
    if (bnd) {
        /* ghost states from the boundary types (Sec. 6) */
        if (g->scheme != REF_SCHEME_MEG6) return -2;
        Qb = (double *)malloc(sizeof(double) * nv * N);
        if (!Qb) return -1;
        memcpy(Qb, Q, sizeof(double) * nv * N);
        ref_apply_bc(g, m, Qb);
        Q = Qb;
    }
    double *grad = (double *)calloc((size_t)12 * N, sizeof(double));
    double *theta = (double *)calloc((size_t)N, sizeof(double));
    double *phi = (double *)malloc(sizeof(double) * 5 * N);
    double *pgrad = NULL;
    if (!grad || !theta || !phi) { free(grad); free(theta); free(phi); free(Qb); return -1; }
    ref_gradients(g, Q, grad);
    if (g->scheme == REF_SCHEME_MIG4) {
        pgrad = (double *)malloc(sizeof(double) * 18 * N);
        if (!pgrad || ig4_prim_grads(g, Q, pgrad)) { free(grad); free(theta); free(phi); free(pgrad); return -1; }
    }
    if (g->limiter == REF_LIM_DUCROS) {
        ref_sensor(g, m, grad, theta);
        /* ghost cells have no metrics of their own: their sensor value is
         * that of the nearest interior cell */
        if (bnd)
            for (long idx = 0; idx < N; ++idx) {
                int ijk[3];
                unpack(g, idx, ijk);
                theta[idx] = theta[clamp_cell(g, ijk, -1)];
            }
    }
    int bad = 0;
    for (long idx = 0; idx < N; ++idx) {
        prim_t s = primitive(g, Q, idx);
        if (!(s.r > 0.0 && s.p > 0.0 && isfinite(s.r) && isfinite(s.p))) bad = 1;
    }
    for (long idx = 0; idx < (long)nv * N; ++idx) res[idx] = 0.0;
    for (int f = 0; f < nf && !bad; ++f) {
#pragma omp parallel for schedule(static) reduction(|| : bad)
        for (long idx = 0; idx < N; ++idx) {
            int ijk[3];
            double ph[5];
            unpack(g, idx, ijk);
            int fail = face_flux(g, m, Q, grad, pgrad, theta, f, ijk, idx, ph);
            if (fail && bnd) {
                /* only interfaces of interior cells count */
                int up[3] = {ijk[0], ijk[1], ijk[2]};
                up[f] = (ijk[f] + 1) % g->n[f];
                fail = in_interior(g, ijk) || in_interior(g, up);
            }
            if (fail) bad = 1;
            for (int s = 0; s < 5; ++s) phi[s * N + idx] = ph[s];
        }
#pragma omp parallel for schedule(static)
        for (long idx = 0; idx < N; ++idx) {
            int ijk[3];
            unpack(g, idx, ijk);
            long lo = neighbour(g, ijk, f, -1, NULL);
            for (int v = 0; v < nv; ++v) {
                int s = (nv == 4 && v == 3) ? 4 : v; /* 2-D: skip the w-momentum */
                res[v * N + idx] -= phi[s * N + idx] - phi[s * N + lo];
            }
        }
    }
    if (bnd)
        for (long idx = 0; idx < N; ++idx) {
            int ijk[3];
            unpack(g, idx, ijk);
            if (!in_interior(g, ijk))
                for (int v = 0; v < nv; ++v) res[v * N + idx] = 0.0;
        }
    if (g->sigma) {
        /* sponge (Sec. 8.3, after Bodony): d Q / dt gains -sigma (Q - Q_ref),
         * i.e. Res gains -sigma (Q - Q_ref) / J with 1/J the cell volume */
        const double *P = g->qref;
        double qr[5];
        qr[0] = P[0];
        qr[1] = P[0] * P[1];
        qr[2] = P[0] * P[2];
        qr[3] = P[0] * P[3];
        qr[4] = P[4] / (g->gamma - 1.0) + 0.5 * P[0] * (P[1] * P[1] + P[2] * P[2] + P[3] * P[3]);
        for (long idx = 0; idx < N; ++idx) {
            int ijk[3];
            unpack(g, idx, ijk);
            if (!in_interior(g, ijk)) continue;
            for (int v = 0; v < nv; ++v) {
                int s = (nv == 4 && v == 3) ? 4 : v;
                res[v * N + idx] -= g->sigma[idx] * (Qs[v * N + idx] - qr[s]) * m[REF_M_INVJ * N + idx];
            }
        }
    }
    free(grad);
    free(theta);
    free(phi);
    free(pgrad);
    free(Qb);
    return bad ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Post-processing diagnostics from the shared gradients (Sec. 3 lists      */
/* vorticity, enstrophy, density-gradient magnitude and the Q-criterion as  */
/* uses of the cell gradients; Eq. KE-Ens defines the volume averages of    */
/* rho |u|^2 / 2 and rho |Omega|^2 / 2). The physical velocity gradient is  */
/* G[a][b] = sum_d (d_{x_b}) du_a/dd with the cell gradients of the scheme  */
/* (E6 or IG4) and the unhatted cell metrics; Omega = curl u; Q = (|W|^2 -  */
/* |S|^2) / 2 with S, W the symmetric and antisymmetric parts of G (the     */
/* usual definition; the paper names it without a formula). Integrals are   */
/* sums of cell values times the cell volume 1/J.                           */
/* Pins: closed-form shear flows (vorticity, Q, integrals), exact volume    */
/* and kinetic energy on affine grids, convergence on curvilinear grids.    */
/* ------------------------------------------------------------------------ */
int ref_diagnostics(const ref_cfg *g, const double *m, const double *Q, double *fields, double *integrals)
{
    if (any_bounded(g)) return -2;
    const long N = ncell_of(g);
    double *grad = (double *)calloc((size_t)12 * N, sizeof(double));
    double *rgrad = (double *)calloc((size_t)3 * N, sizeof(double));
    double *pr = (double *)malloc(sizeof(double) * 6 * N);
    if (!grad || !rgrad || !pr) { free(grad); free(rgrad); free(pr); return -1; }
    ref_gradients(g, Q, grad);
    primitive_fields(g, Q, pr);
    /* density gradients along each computational direction */
    int rc = 0;
    if (g->scheme == REF_SCHEME_MIG4) {
        for (int d = 0; d < g->ndim && !rc; ++d) {
            grad_job jb = {g, d, pr, rgrad + d * N};
            rc = for_lines(g, d, grad_job_fn, &jb);
        }
    } else {
        for (long idx = 0; idx < N; ++idx) {
            int ijk[3];
            unpack(g, idx, ijk);
            for (int d = 0; d < g->ndim; ++d) {
                double w[7];
                field_window(g, pr, ijk, d, -3, 3, w);
                rgrad[d * N + idx] = e6(w + 3);
            }
        }
    }
    double ke = 0.0, ens = 0.0, vol = 0.0;
    for (long idx = 0; idx < N && !rc; ++idx) {
        double G[3][3], gr[3];
        for (int b = 0; b < 3; ++b) {
            for (int a = 0; a < 3; ++a) {
                double s = 0.0;
                for (int d = 0; d < g->ndim; ++d) s += m[REF_M_UNHAT(d, b) * N + idx] * grad[(d * 4 + a) * N + idx];
                G[a][b] = s;
            }
            double s = 0.0;
            for (int d = 0; d < g->ndim; ++d) s += m[REF_M_UNHAT(d, b) * N + idx] * rgrad[d * N + idx];
            gr[b] = s;
        }
        double om[3] = {G[2][1] - G[1][2], G[0][2] - G[2][0], G[1][0] - G[0][1]};
        double s2 = 0.0, w2 = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double sab = 0.5 * (G[a][b] + G[b][a]), wab = 0.5 * (G[a][b] - G[b][a]);
                s2 += sab * sab;
                w2 += wab * wab;
            }
        fields[0 * N + idx] = om[0];
        fields[1 * N + idx] = om[1];
        fields[2 * N + idx] = om[2];
        fields[3 * N + idx] = 0.5 * (w2 - s2);
        fields[4 * N + idx] = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
        double rho = pr[idx], u = pr[N + idx], v = pr[2 * N + idx], w = pr[3 * N + idx];
        double dv = m[REF_M_INVJ * N + idx];
        ke += 0.5 * rho * (u * u + v * v + w * w) * dv;
        ens += 0.5 * rho * (om[0] * om[0] + om[1] * om[1] + om[2] * om[2]) * dv;
        vol += dv;
    }
    integrals[0] = ke / vol;
    integrals[1] = ens / vol;
    integrals[2] = vol;
    free(grad); free(rgrad); free(pr);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Time step (App. B) and SSP-RK3 stage (App. B with Eq. time-split).       */
/* ------------------------------------------------------------------------ */
double ref_cfl_min(const ref_cfg *g, const double *m, const double *Q)
{
    const long N = ncell_of(g);
    double best = INFINITY, bestv = INFINITY;
    for (long idx = 0; idx < N; ++idx) {
        int ijk[3];
        unpack(g, idx, ijk);
        if (!in_interior(g, ijk)) continue;  /* ghost cells are not advanced */
        prim_t s = primitive(g, Q, idx);
        double c = sqrt(g->gamma * s.p / s.r);
        double nu = g->viscous ? viscosity(g, s.T) / s.r : 0.0;
        for (int d = 0; d < g->ndim; ++d) {
            double dxv = m[REF_M_UNHAT(d, 0) * N + idx], dyv = m[REF_M_UNHAT(d, 1) * N + idx];
            double dzv = m[REF_M_UNHAT(d, 2) * N + idx];
            double U = m[REF_M_UNHATT(d) * N + idx] + dxv * s.u + dyv * s.v + dzv * s.w;
            double gn2 = dxv * dxv + dyv * dyv + dzv * dzv;
            double inv = 1.0 / (fabs(U) + c * sqrt(gn2));
            if (inv < best) best = inv;
            if (g->viscous) {
                double iv = 1.0 / (nu * gn2);
                if (iv < bestv) bestv = iv;
            }
        }
    }
    if (g->viscous) {
        double v = bestv / g->alpha_d;
        if (v < best) best = v;
    }
    return best;
}

void ref_rk_stage(const ref_cfg *g, const double *m, int stage, double dt,
                  const double *Qn, double *Q, const double *res)
{
    static const double A[3] = {0.0, 0.75, 1.0 / 3.0};
    static const double B[3] = {1.0, 0.25, 2.0 / 3.0};
    const long N = ncell_of(g);
    const int nv = g->ndim + 2;
    for (int v = 0; v < nv; ++v)
        for (long idx = 0; idx < N; ++idx) {
            int ijk[3];
            unpack(g, idx, ijk);
            if (!in_interior(g, ijk)) continue;  /* ghost cells are not advanced */
            long e = v * N + idx;
            double L = m[REF_M_J * N + idx] * (res[e] - m[REF_M_INVJT * N + idx] * Q[e]);
            Q[e] = A[stage] * Qn[e] + B[stage] * (Q[e] + dt * L);
        }
}

int ref_step(const ref_cfg *g, double *m, const double *xyz, const double *xyz_t,
             double *Q, double cfl_or_dt, int dt_mode, double *dt_out)
{
    const long N = ncell_of(g);
    const int nv = g->ndim + 2;
    if (g->moving) {
        int rc = ref_metrics(g, xyz, xyz_t, m);
        if (rc) return rc;
    }
    double dt = (dt_mode == REF_DT_CFL) ? cfl_or_dt * ref_cfl_min(g, m, Q) : cfl_or_dt;
    double *Qn = (double *)malloc(sizeof(double) * nv * N);
    double *res = (double *)malloc(sizeof(double) * nv * N);
    if (!Qn || !res) { free(Qn); free(res); return -1; }
    memcpy(Qn, Q, sizeof(double) * nv * N);
    int rc = 0;
    for (int s = 0; s < 3 && !rc; ++s) {
        rc = ref_rhs(g, m, Q, res);
        if (!rc) ref_rk_stage(g, m, s, dt, Qn, Q, res);
    }
    if (!rc && any_bounded(g)) ref_apply_bc(g, m, Q);  /* ghost cells of the new state */
    free(Qn);
    free(res);
    if (dt_out) *dt_out = dt;
    return rc;
}

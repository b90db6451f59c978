/*
 * FP64 CPU oracle of the gradient-based-reconstruction right-hand side on
 * periodic curvilinear (optionally moving) grids.
 *
 * TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The HIP product path
 * never includes, links or calls anything here, and this file includes nothing
 * of the product path.
 *
 * Layout: every field is a structure-of-arrays block [var][nk][nj][ni], i
 * fastest. Direction d = 0, 1, 2 is xi, eta, zeta; coordinate c = 0, 1, 2 is
 * x, y, z. A periodic direction has ``off[d][c]``, the shift of coordinate
 * c when the index along d wraps once; a non-periodic one carries ghost
 * layers (see ref_cfg.bc).
 *
 * Parity pins and their status are listed per function in gbr_oracle.c.
 */
#ifndef GBR_ORACLE_H
#define GBR_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { REF_LIM_NONE = 0, REF_LIM_MP = 1, REF_LIM_DUCROS = 2 };
enum { REF_SCHEME_MEG6 = 0, REF_SCHEME_MIG4 = 1 };
enum { REF_DT_CFL = 0, REF_DT_FIXED = 1 };
/* Boundary types per direction and side (Sec. 6): periodic (both sides of a
 * direction), Dirichlet inflow (ghost cells keep the state stored in them),
 * zero-gradient outflow, reflecting slip wall.                            */
enum { REF_BC_PERIODIC = 0, REF_BC_INFLOW = 1, REF_BC_OUTFLOW = 2, REF_BC_WALL = 3 };
#define REF_NG 6  /* ghost layers on each non-periodic side */

typedef struct {
    int n[3];          /* cells along xi, eta, zeta                          */
    int ndim;          /* 2 (n[2] == 1, nvar 4) or 3 (nvar 5)                */
    int viscous;       /* 0: Euler, 1: Navier-Stokes (alpha-damping)         */
    int limiter;       /* REF_LIM_*                                          */
    int moving;        /* 1: grid velocities given, GCL terms active         */
    int scheme;        /* REF_SCHEME_MEG6 (E6 gradients) or REF_SCHEME_MIG4 (IG4) */
    double off[3][3];  /* periodic coordinate shift per wrapped direction   */
    double gamma, Pr, Re, Mref, suth; /* suth = Sutherland S / T_ref        */
    double theta_c;    /* shock-sensor threshold                             */
    double alpha_mp, beta_mp; /* MP limiter constants                      */
    double alpha_d;    /* alpha-damping coefficient                          */
    /* Non-periodic directions: n[d] counts REF_NG ghost layers on each side
     * (interior cells REF_NG .. n[d] - REF_NG - 1). Static MEG6 grids only. */
    int bc[3][2];      /* REF_BC_* per direction, side 0 (low) and 1 (high)  */
    const double *sigma; /* sponge strength per cell, or NULL                */
    double qref[5];    /* sponge reference state (rho, u, v, w, p)           */
} ref_cfg;

/* Metric block: one contiguous array of REF_M_TOTAL * ncell doubles. Slot s
 * occupies [s * ncell, (s + 1) * ncell).                                   */
#define REF_M_HAT(d, c)      ((d) * 3 + (c))          /* cell hatted d_c/J     */
#define REF_M_UNHAT(d, c)    (9 + (d) * 3 + (c))      /* cell d_c             */
#define REF_M_INVJ           18                        /* cell 1/J             */
#define REF_M_J              19                        /* cell J               */
#define REF_M_HATT(d)        (20 + (d))                /* cell hatted d_t/J    */
#define REF_M_UNHATT(d)      (23 + (d))                /* cell d_t             */
#define REF_M_INVJT          26                        /* cell (1/J)_t         */
#define REF_M_FHAT(f, c)     (27 + (f) * 13 + (c))     /* face f: hatted f_c   */
#define REF_M_FHATT(f)       (27 + (f) * 13 + 3)       /* face f: hatted f_t   */
#define REF_M_FUNHAT(f, e, c) (27 + (f) * 13 + 4 + (e) * 3 + (c)) /* face f: e_c */
#define REF_M_TOTAL          66
/* A face value stored at cell index (i, j, k) for family f belongs to the
 * interface between that cell and its +1 neighbour along f.               */

/* --- line primitives (periodic 1-D lines, n >= 1) ---------------------- */
void ref_line_e6(const double *v, int n, double shift, double *out);
void ref_line_hermite(const double *v, int n, double shift, double *out);
void ref_line_face(const double *v, int n, double shift, double *out);
void ref_line_dcomp(const double *v, int n, double shift, double *out);
/* IG4 (Eq. IG4_grads) on a periodic line with v[i+n] = v[i] + shift; out[i]
 * = derivative. ref_line_ig4_face: interface values at i + 1/2 (Eq. FP-interp
 * with IG4 gradients); ref_line_ig4_dcomp: their difference (Eq. FP-interp2).
 * Return nonzero if the line system is singular.                           */
int ref_line_ig4(const double *v, int n, double shift, double *out);
int ref_line_ig4_face(const double *v, int n, double shift, double *out);
int ref_line_ig4_dcomp(const double *v, int n, double shift, double *out);

/* App. C on a non-periodic line of m >= 12 interior values: first and
 * second derivatives with the boundary closures (p, h: m values each) and
 * the interface values F[0..m] (F[f] between cells f - 1 and f). Return -1
 * if m < 12.                                                              */
int ref_bline_derivs(const double *v, int m, double *p, double *h);
int ref_bline_faces(const double *v, int m, double *F);

/* --- pointwise pieces --------------------------------------------------- */
void ref_eigvec(const double nrm[3], double rho, double a, double R[25], double Rinv[25]);
double ref_mp_limit(double wm1, double w0, double wp1, double dm1, double d0,
                    double dp1, double wface, double alpha, double beta);
void ref_hllc(const double PL[5], const double PR[5], const double nt_n[4],
              double gamma, double F[5]);
void ref_euler_flux(const double P[5], const double nt_n[4], double gamma, double F[5]);

/* --- whole-grid operations ---------------------------------------------- */
/* Ghost cells of Q from the boundary types (Sec. 6), directions in order. */
void ref_apply_bc(const ref_cfg *cfg, const double *m, double *Q);
int ref_metrics(const ref_cfg *cfg, const double *xyz, const double *xyz_t, double *m);
int ref_metrics_nonfp(const ref_cfg *cfg, const double *xyz, double *m);
void ref_gradients(const ref_cfg *cfg, const double *Q, double *grad);
void ref_sensor(const ref_cfg *cfg, const double *m, const double *grad, double *theta);
int ref_rhs(const ref_cfg *cfg, const double *m, const double *Q, double *res);
double ref_cfl_min(const ref_cfg *cfg, const double *m, const double *Q);
/* Diagnostics from the shared cell gradients: fields[5][cells] = vorticity
 * (x, y, z), Q-criterion, |grad rho|; integrals[3] = kinetic energy and
 * enstrophy per unit volume (Eq. KE-Ens) and the volume sum of 1/J.
 * Returns nonzero on allocation failure.                                  */
int ref_diagnostics(const ref_cfg *cfg, const double *m, const double *Q, double *fields, double *integrals);
void ref_rk_stage(const ref_cfg *cfg, const double *m, int stage, double dt,
                  const double *Qn, double *Q, const double *res);
int ref_step(const ref_cfg *cfg, double *m, const double *xyz, const double *xyz_t,
             double *Q, double cfl_or_dt, int dt_mode, double *dt_out);

#ifdef __cplusplus
}
#endif
#endif

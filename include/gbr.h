/*
 * gbr.h - C ABI of the MI355X gradient-based-reconstruction solver.
 *
 * The library evaluates the semi-discrete right-hand side of the compressible
 * Euler / Navier-Stokes equations in generalized curvilinear coordinates
 * (Chandravamsi, Chamarthi, Hoffmann, Frankel, arXiv 2303.10785): E6 central
 * gradients, gradient-based characteristic interface states with the improved
 * MP limiter (optionally gated by a Ducros shock sensor), the curvilinear HLLC
 * flux, the alpha-damping viscous flux, freestream-preserving conservative
 * metrics and the geometric conservation law on moving grids, and the SSP-RK3
 * stage update. All arithmetic runs in HIP kernels on the device.
 *
 * Conventions (all calls):
 *  - Pointers to field data are DEVICE pointers owned by the caller, on the
 *    device that was current when the grid was created.
 *  - Field layout is structure-of-arrays [var][nk][nj][ni], i fastest,
 *    FP64. Conserved variables in the order (rho, rho u, rho v, [rho w], E):
 *    nvar = ndim + 2. Coordinates are [3][nk][nj][ni] (x, y, z); for ndim = 2
 *    the z plane is ignored and z is taken as the zeta index.
 *  - A direction is periodic (off[d] is the (x, y, z) shift of the
 *    coordinates when the index along d wraps once) or, per bc[d], bounded
 *    on both sides: then the first and last GBR_NG cells along d are ghost
 *    cells (Sec. 6). Ghost cells are part of every field array; they are
 *    not advanced in time, their coordinates are ignored and their states
 *    follow the boundary type (see GBR_BC_*).
 *  - Work is enqueued on the HIP stream given at creation (or by
 *    gbr_set_stream); calls return without waiting unless stated.
 *  - Batch-first: calls take an array of n >= 0 grid handles and per-grid
 *    pointer arrays; n = 0 is a no-op that returns GBR_OK.
 *  - No exception or abort crosses the ABI. On error the status is returned
 *    and gbr_last_error(g) describes it until the next call on g. One host
 *    thread may use a handle at a time.
 */
#ifndef GBR_H
#define GBR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gbr_status {
    GBR_OK = 0,
    GBR_E_ARG = 1,         /* invalid argument (null pointer, bad size or mode)    */
    GBR_E_JACOBIAN = 2,    /* a cell has 1/J <= 0 (folded or left-handed grid)     */
    GBR_E_STATE = 3,       /* non-physical state: rho <= 0, p <= 0 or non-finite   */
    GBR_E_NOMEM = 4,       /* device allocation failed                             */
    GBR_E_DEVICE = 5,      /* HIP runtime error                                    */
    GBR_E_UNSUPPORTED = 6  /* option not implemented                              */
} gbr_status;

enum { GBR_LIM_NONE = 0, GBR_LIM_MP = 1, GBR_LIM_DUCROS = 2 };
/* Precision: GBR_FP64 computes everything in double. GBR_FP32_BULK keeps Q,
 * the metrics, J, (1/J)_t, the time step and the RK accumulation in double
 * and runs primitives, gradients, the sensor, reconstruction, limiter, HLLC,
 * viscous flux and Res in float; those float kernels read the metrics from
 * a float copy rounded once after each gbr_metrics call, and divide and take
 * square roots with the hardware reciprocal and square root (about 1 ulp). */
enum { GBR_FP64 = 0, GBR_FP32_BULK = 1 };
enum { GBR_DT_CFL = 0, GBR_DT_FIXED = 1 };
/* Gradient scheme of Sec. 5.1 Step-1: GBR_SCHEME_MEG6 uses the explicit
 * sixth-order gradients (Eq. E6_grads), GBR_SCHEME_MIG4 the fourth-order
 * implicit gradients (Eq. IG4_grads, alpha = 5/14), in the reconstruction,
 * the viscous gradients, the sensor and, as Sec. 7 directs, the metric
 * interpolation.                                                           */
enum { GBR_SCHEME_MEG6 = 0, GBR_SCHEME_MIG4 = 1 };
/* Boundary types (Sec. 6) per direction and side of gbr_config.bc:
 *  GBR_BC_PERIODIC: both sides of the direction (the default, all zero).
 *  GBR_BC_INFLOW:   Dirichlet; the ghost cells keep the conserved state the
 *                   caller stores in them (the library never writes them).
 *  GBR_BC_OUTFLOW:  zero gradient; ghost cells take the state of the
 *                   boundary cell of their grid line.
 *  GBR_BC_WALL:     reflecting slip wall; the ghost cell at depth k mirrors
 *                   the interior cell at depth k with the velocity component
 *                   along the unit normal of the boundary face reversed.
 * Directions are filled in order xi, eta, zeta over the full extent of the
 * others (corner ghosts take the later direction's rule). A bounded
 * direction needs n[d] >= 2 GBR_NG + 12 and d < ndim. Metrics near the
 * boundary use the one-sided closures of App. C; interfaces and gradients
 * of interior cells read up to GBR_NG ghost cells, as the paper notes the
 * flux formulae stay unchanged at boundaries. Bounded grids are static and
 * use GBR_SCHEME_MEG6.                                                    */
enum { GBR_BC_PERIODIC = 0, GBR_BC_INFLOW = 1, GBR_BC_OUTFLOW = 2, GBR_BC_WALL = 3 };
#define GBR_NG 6

typedef struct gbr_config {
    int32_t ndim;      /* 2 or 3 (n[2] must be 1 when ndim == 2)                  */
    int32_t n[3];      /* cells along xi, eta, zeta; each >= 1                    */
    int32_t viscous;   /* 0 Euler, 1 Navier-Stokes with alpha-damping (Sec. 5.2)  */
    int32_t limiter;   /* GBR_LIM_*: none, MP limiter on every interface (the     */
                       /* paper, App. E), or MP where a Ducros sensor flags       */
    int32_t moving;    /* 1: grid velocities are supplied, GCL terms (Sec. 4.2)   */
    int32_t precision; /* GBR_FP64 or GBR_FP32_BULK                               */
    int32_t scheme;    /* GBR_SCHEME_MEG6 or GBR_SCHEME_MIG4                      */
    double off[3][3];  /* periodic coordinate shift per wrapped direction         */
    double gamma;      /* ratio of specific heats (1.4 in the paper)              */
    double Pr;         /* Prandtl number (0.71)                                   */
    double Re;         /* Reynolds number: mu = Sutherland(T) / Re                */
    double Mref;       /* reference Mach number: p = rho T / (gamma Mref^2)       */
    double suth;       /* Sutherland constant over the reference temperature     */
    double theta_c;    /* shock-sensor threshold (GBR_LIM_DUCROS)                 */
    double alpha_mp;   /* MP limiter alpha (4)                                    */
    double beta_mp;    /* MP limiter beta (4)                                     */
    double alpha_d;    /* alpha-damping coefficient alpha^D (4, Sec. 5.2)         */
    int32_t bc[3][2];  /* GBR_BC_* per direction, side 0 (low) and 1 (high)      */
} gbr_config;

typedef struct gbr_grid_s *gbr_grid;

/* Metric inspection slots for gbr_metric_ptr. A face slot value stored at
 * cell (i, j, k) belongs to the interface between that cell and its +1
 * neighbour along the family direction f.                                   */
#define GBR_SLOT_FACE_HAT(f, c)      ((f) * 13 + (c))                 /* hat f_c      */
#define GBR_SLOT_FACE_HATT(f)        ((f) * 13 + 3)                   /* hat f_t      */
#define GBR_SLOT_FACE_UNHAT(f, e, c) ((f) * 13 + 4 + (e) * 3 + (c))   /* e_c at face f */
#define GBR_SLOT_CELL_UNHAT(e, c)    (39 + (e) * 3 + (c))             /* e_c          */
#define GBR_SLOT_CELL_J              48                               /* J            */
#define GBR_SLOT_CELL_INVJ           49                               /* 1/J          */
#define GBR_SLOT_CELL_INVJT          50                               /* (1/J)_t      */
#define GBR_SLOT_CELL_UNHATT(e)      (51 + (e))                       /* e_t          */
#define GBR_SLOT_CELL_HAT(e, c)      (54 + (e) * 3 + (c))             /* hat e_c      */
#define GBR_SLOT_CELL_HATT(e)        (63 + (e))                       /* hat e_t      */
#define GBR_SLOT_COUNT               66

/* Create a grid handle: validates cfg, allocates the library-owned device
 * buffers (metrics, gradient and sensor scratch, RK and time-step storage;
 * size given by gbr_grid_bytes) and binds hip_stream (a hipStream_t, or NULL
 * for the default stream). Metrics are undefined until gbr_metrics.
 * Errors: GBR_E_ARG (null pointer, ndim not 2/3, n < 1, n[2] != 1 in 2-D,
 * unknown limiter, precision or scheme, non-positive gamma/Re/Pr/Mref),
 * GBR_E_NOMEM, GBR_E_DEVICE. *out is NULL on error.                        */
gbr_status gbr_grid_create(const gbr_config *cfg, void *hip_stream, gbr_grid *out);

/* Release a handle and its device buffers (waits for its stream). NULL is
 * accepted.                                                                 */
gbr_status gbr_grid_destroy(gbr_grid g);

/* Device bytes gbr_grid_create allocates for cfg (0 if cfg is invalid): for
 * admission against an HBM budget.                                          */
size_t gbr_grid_bytes(const gbr_config *cfg);

/* Rebind the stream used by later calls on g.                               */
gbr_status gbr_set_stream(gbr_grid g, void *hip_stream);

/* Metrics (Sec. 4.2, Sec. 7): conservative Thomas-Lombard metrics with the
 * central derivative obtained from the inviscid interpolation (Eq. FP-interp,
 * FP-interp2), the Jacobian (Eq. Jac-matrix), interface values of every
 * metric with the same central formula (Eq. interp-formulae) and, if the grid
 * is moving, the temporal metrics and (1/J)_t from the GCL (Eq. Jacb2).
 * xyz[b]: cell-centre coordinates of grid b, [3][nk][nj][ni].
 * xyz_t[b]: grid velocity at the cell centres, same layout; required (non
 * NULL) for moving grids, ignored otherwise (xyz_t itself may be NULL).
 * On grids with bounded directions the derivatives and interface values
 * along them use the App. C closures on the interior cells (the first
 * and second derivatives of the first three cells from the one-sided,
 * partially one-sided and central formulas; the interface next to the
 * boundary face from the inward cell; the boundary face from the boundary
 * cell), and every ghost slot holds the value of the nearest interior cell
 * (nearest interface from the boundary face inwards for face slots).
 * Synchronises the stream and returns GBR_E_JACOBIAN if any interior
 * 1/J <= 0.                                                                 */
gbr_status gbr_metrics(const gbr_grid *g, int n, const double *const *xyz,
                       const double *const *xyz_t);

/* Negative control of App. D: non-freestream-preserving metrics in place
 * of gbr_metrics, for static grids. Coordinate derivatives from the
 * fourth-order central formula (Eq. 4thorder-grads), hat(d)_c =
 * (c1)_d1 (c2)_d2 - (c1)_d2 (c2)_d1 (the cyclic form; the printed zeta_y
 * entry has a zeta where the cycle has xi), interface values from
 * Eq. interp-formulae with that derivative in place of E6. A uniform flow
 * then does not stay uniform on curved grids (Sec. 8.1.1). Errors as
 * gbr_metrics; GBR_E_UNSUPPORTED for moving or bounded grids.             */
gbr_status gbr_metrics_nonfp(const gbr_grid *g, int n, const double *const *xyz);

/* Right-hand side Res = d(Q/J)/dt (Sec. 3, Sec. 5.1 Steps 1-7, Sec. 5.2
 * Steps 1-5): res[b] receives -sum_d [Phi(+1/2) - Phi(-1/2)] with
 * Phi = F - F^v, the directions accumulated in the order zeta, eta, xi
 * (eta, xi in 2-D).
 * Q[b]: conserved state (read only, double). res[b]: output, nvar arrays of
 * double (GBR_FP64) or float (GBR_FP32_BULK); must not alias Q[b].
 * Bounded grids: ghost primitives come from the boundary types (Q itself
 * is not written), Res is zero in ghost cells, and a sponge set with
 * gbr_set_sponge adds -sigma (Q - Q_ref) / J in interior cells.
 * Asynchronous; a non-physical interior state or reconstructed interface
 * state of an interior cell sets the grid's state flag, reported by
 * gbr_check_state.                                                          */
gbr_status gbr_rhs(const gbr_grid *g, int n, const double *const *Q, void *const *res);

/* One SSP-RK3 stage (App. B with Eq. time-split), in place on Q[b]:
 *   Q <- a_s Qn + b_s (Q + dt J (Res - (1/J)_t Q)),
 * (a_s, b_s) = (0, 1), (3/4, 1/4), (1/3, 2/3) for stage = 0, 1, 2.
 * dt[b]: device pointer to the grid's time step (one double). res[b] has the
 * grid's precision (double or float); the update itself is in double.
 * Ghost cells of bounded grids are left unchanged.                          */
gbr_status gbr_rk_stage(const gbr_grid *g, int n, int stage, const double *const *dt,
                        const double *const *Qn, double *const *Q, const void *const *res);

/* Time step (App. B): dt[b] <- cfl * min over cells and directions of
 * 1/(|U| + c |grad d|), and for viscous grids also (1/alpha_d) min
 * 1/(nu |grad d|^2), over interior cells. dt[b] is a device pointer; no
 * host synchronisation.                                                     */
gbr_status gbr_cfl(const gbr_grid *g, int n, const double *const *Q, double cfl,
                   double *const *dt);

/* One SSP-RK3 step in place on Q[b]: for moving grids first the metrics at
 * t^n from xyz[b], xyz_t[b] (Sec. 4.2: recomputed once per step), then the
 * time step (dt_mode GBR_DT_CFL: cfl_or_dt is the CFL number; GBR_DT_FIXED:
 * cfl_or_dt is dt), then three RHS evaluations and stages. Qn and Res are
 * library-owned. dt_out[b] (device pointer to one double, may be NULL / the
 * array may be NULL) receives the step's dt. t[b] (device pointer to one
 * double, the grid's time, may be NULL / the array may be NULL) is advanced
 * by the step's dt on the device (t^{n+1} = t^n + dt, App. B), so a caller
 * can step a grid without reading dt back; it must not alias dt_out[b]
 * (GBR_E_ARG). The coordinates of a moving grid are the caller's mesh at
 * t^n; the library evaluates no mesh motion itself. Bounded grids advance
 * interior cells only; each stage sets ghost primitives from the boundary
 * types, and at the end of the step the outflow and wall ghost cells of Q
 * receive their states (inflow ghost cells are never written).
 * Asynchronous.                                                            */
gbr_status gbr_step(const gbr_grid *g, int n, double *const *Q, const double *const *xyz,
                    const double *const *xyz_t, double cfl_or_dt, int dt_mode,
                    double *const *dt_out, double *const *t);

/* Synchronise g's stream and report flags raised since the last check:
 * GBR_E_STATE (non-physical state) or GBR_E_JACOBIAN (from a gbr_step metric
 * update). Clears the flags.                                                */
gbr_status gbr_check_state(gbr_grid g);

/* gbr_cfl for callers that cannot allocate device memory (code under HIP
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same time step, bitwise, with the per-block partial minima kept in a static
 * device array of the library (1 MiB per device, reserved until the process
 * ends; 32 slices of 4096 doubles, slice b for grid b of the call) instead of
 * the grid's own buffer. Calls no hipMalloc, hipFree or allocating routine
 * (the device address of the array is looked up once per device on first
 * use) and records no timing events. At most 32 grids per call (GBR_E_ARG
 * beyond, with a message in gbr_last_error(g[0])); other errors as gbr_cfl.
 * Every call on a device shares that device's array: calls whose work
 * overlaps on one device (different streams, or host threads) race and must
 * be ordered by the caller; grids of one call on different streams do not
 * race with each other. The array keeps the last call's partials; each
 * launch writes every slot it reads, so nothing needs clearing.            */
gbr_status gbr_cfl_noalloc(const gbr_grid *g, int n, const double *const *Q, double cfl,
                           double *const *dt);

/* Diagnostics from the cell gradients the scheme shares (Sec. 3 names
 * vorticity, enstrophy, density-gradient magnitude and the Q-criterion as
 * uses of them; Eq. KE-Ens defines the kinetic-energy and enstrophy
 * averages). With G = du_a/dx_b from the scheme's cell gradients (E6 or
 * IG4) and the unhatted cell metrics:
 *   fields[b] (device, 5 * ncell doubles, may be NULL): vorticity x, y, z
 *   (curl u), Q-criterion (|W|^2 - |S|^2) / 2 with S, W the symmetric and
 *   antisymmetric parts of G, and |grad rho|;
 *   integrals[b] (device, 3 doubles, may be NULL): volume averages of
 *   rho |u|^2 / 2 and rho |curl u|^2 / 2, and the volume sum of 1/J.
 * Cell volumes are 1/J; the sums are taken in a fixed order, so repeated
 * calls give identical results. Uses the grid's gradient scratch (not
 * concurrently with gbr_rhs / gbr_step on the same grid). Asynchronous.
 * GBR_E_UNSUPPORTED on bounded grids.                                       */
gbr_status gbr_diagnostics(const gbr_grid *g, int n, const double *const *Q, double *const *fields,
                           double *const *integrals);

/* Sponge layers (Sec. 8.3, after Bodony): the right-hand side gains the
 * relaxation source -sigma (Q - Q_ref), i.e. Res += -sigma (Q - Q_ref) / J,
 * in interior cells (every cell of a periodic grid). sigma: device pointer
 * to ncell doubles (>= 0; zero outside the layers), copied into library
 * memory (ncell doubles, allocated on the first call and kept until
 * gbr_grid_destroy or a call with sigma == NULL; not counted by
 * gbr_grid_bytes) on g's stream before the call returns (the caller may
 * free it afterwards). ref: host pointer to
 * the reference primitive state (rho, u, v, w, p); w is ignored in 2-D.
 * sigma == NULL removes the sponge. Errors: GBR_E_ARG (null g, null ref
 * with non-null sigma, rho or p <= 0), GBR_E_NOMEM, GBR_E_DEVICE.          */
gbr_status gbr_set_sponge(gbr_grid g, const double *sigma, const double *ref);

/* Read-only device pointer to one metric slot (GBR_SLOT_*), ncell doubles,
 * owned by the library; NULL on a bad slot. Valid until gbr_grid_destroy.  */
const double *gbr_metric_ptr(gbr_grid g, int slot);

/* Kernel classes for gbr_timing_collect.                                   */
enum {
    GBR_K_METRICS = 0,     /* metric and GCL kernels                             */
    GBR_K_CELL_GRAD = 1,   /* cell gradients and shock sensor                    */
    GBR_K_SWEEP_XI = 2,    /* interface sweep along xi (writes Res)              */
    GBR_K_SWEEP_ETA = 3,   /* interface sweep along eta                          */
    GBR_K_SWEEP_ZETA = 4,  /* interface sweep along zeta                         */
    GBR_K_RK_STAGE = 5,    /* SSP-RK3 stage update                               */
    GBR_K_CFL = 6,         /* time-step reduction (in gbr_step fused with the
                              first stage's primitives)                          */
    GBR_K_COPY = 7,        /* state copies and fills                             */
    GBR_K_PRIMS = 8,       /* primitive variables of the state                   */
    GBR_K_DIAG = 9,        /* diagnostics                                        */
    GBR_K_COUNT = 10
};

/* Per-kernel timing for benchmarks: while enabled (on != 0), every kernel
 * launch on g is bracketed by two HIP events on g's stream. Disabling drops
 * pending records.                                                          */
gbr_status gbr_timing_enable(gbr_grid g, int on);

/* Synchronise g's stream, add the duration of every recorded launch to
 * ms[class] and count it in launches[class] (both arrays of GBR_K_COUNT
 * entries, caller-owned host memory, accumulated into), and clear the
 * records.                                                                  */
gbr_status gbr_timing_collect(gbr_grid g, double *ms, long *launches);

/* ------------------------------------------------------------------------
 * Batched stepping of many small 2-D Euler grids. One step of all grids is
 * a handful of launches, each over every grid at once: a persistent kernel
 * per SSP-RK3 stage walks a work list of (grid, tile) pairs and does all of
 * Sec. 5.1 Steps 1-7 and the App. B stage update for its tile in LDS. The
 * step can be captured once as a HIP graph and replayed.
 * ---------------------------------------------------------------------- */
typedef struct gbr_batch_s *gbr_batch;

/* Tile shapes (cells along xi x eta) of the batched kernels.              */
enum { GBR_TILE_AUTO = -1, GBR_TILE_16X16 = 0, GBR_TILE_32X8 = 1, GBR_TILE_8X32 = 2, GBR_TILE_COUNT = 3 };

/* Bind n >= 1 grids and their states for batched stepping.
 * Every grid must be 2-D, inviscid, static, periodic, MEG6, without a
 * sponge, with limiter GBR_LIM_NONE or GBR_LIM_MP, and all must share precision, limiter, gamma, the MP
 * constants, the stream and the device; a grid may appear once. Metrics
 * must be computed (gbr_metrics) before gbr_batch_run.
 * Q[b]: device state of grid b, advanced in place by gbr_batch_run; it must
 * stay allocated until gbr_batch_destroy. The grids' own RK and residual
 * buffers serve as the two stage buffers, so no other step or RHS call may
 * run on these grids while the batch has work queued.
 * tile: GBR_TILE_* or GBR_TILE_AUTO, which times one stage launch of every
 * shape on this batch (writing only the stage buffers) and keeps the
 * fastest. Results do not depend on the tile shape up to floating-point
 * contraction; a caller that needs bitwise equality between batches fixes
 * the shape.
 * The library allocates a few bytes per grid and per tile on the device.
 * Errors: GBR_E_ARG, GBR_E_UNSUPPORTED (a grid outside the requirements),
 * GBR_E_NOMEM, GBR_E_DEVICE; message in gbr_last_error(g[0]).             */
gbr_status gbr_batch_create(const gbr_grid *g, int n, double *const *Q, int tile, gbr_batch *out);

/* Enqueue `steps` >= 0 SSP-RK3 steps of every grid of the batch: per grid,
 * dt from App. B (dt_mode GBR_DT_CFL, cfl_or_dt the CFL number) or dt =
 * cfl_or_dt (GBR_DT_FIXED), then the three stages. The batch runs on its own
 * stream, ordered after the work queued on the grids' stream before the
 * call; work queued there afterwards waits for it. use_graph != 0 captures
 * one step as a HIP graph on first use (again when cfl_or_dt or dt_mode
 * change) and replays it. Non-physical states set the grid's flag
 * (gbr_check_state). Errors: GBR_E_ARG, GBR_E_DEVICE; message in
 * gbr_last_error of the first grid.                                        */
gbr_status gbr_batch_run(gbr_batch b, int steps, double cfl_or_dt, int dt_mode, int use_graph);

/* Wait for the batch, then copy, per grid in creation order, the time
 * accumulated by all steps since creation into t[n] and the last step's dt
 * into dt[n] (host arrays, each may be NULL), and the tile shape in use
 * into *tile (may be NULL).                                                */
gbr_status gbr_batch_query(gbr_batch b, double *t, double *dt, int *tile);

/* Wait for the batch and release it (not the grids). NULL is accepted.     */
gbr_status gbr_batch_destroy(gbr_batch b);

/* Measurement probe, not part of the solver: the STREAM triad
 * a[i] = b[i] + s c[i], i < n, enqueued on hip_stream (a hipStream_t or
 * NULL). a, b, c are device arrays of n doubles, 16-byte aligned, a not
 * overlapping b or c. Its rate, 24 n bytes over the kernel time, is the
 * achievable HBM bandwidth the solver's kernels are reported against.
 * Errors: GBR_E_ARG (n < 0, null or misaligned pointer), GBR_E_DEVICE. */
gbr_status gbr_probe_triad(double *a, const double *b, const double *c, double s, long n,
                           void *hip_stream);

/* Message for the last error on g (static text for g == NULL). Valid until
 * the next call on g.                                                       */
const char *gbr_last_error(gbr_grid g);

#ifdef __cplusplus
}
#endif
#endif /* GBR_H */

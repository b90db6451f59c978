// Internal declarations of the HIP implementation of gbr.h (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "gbr.h"

// Library-owned state of one grid.
struct gbr_grid_s {
    gbr_config cfg;
    hipStream_t stream = nullptr;
    int device = 0;
    long ncell = 0;
    int nvar = 0;
    double *metrics = nullptr;   // GBR_SLOT_COUNT * ncell
    // FP32-bulk grids only, kFloatMetricSlots * ncell floats: the metric
    // slots the RHS kernels read in the compute type (every face slot and the
    // cell unhatted metrics, slots 0 .. 47), rounded once from `metrics`
    // after each metric evaluation
    float *metrics_f = nullptr;
    double *scratch = nullptr;   // 12 * ncell: coordinate derivatives (metrics) / gradients (rhs)
    unsigned char *lim_flag = nullptr;  // ncell: 1 where the Ducros sensor exceeds theta_c
    double *grad2 = nullptr;     // 6 * ncell, MIG4 only: IG4 gradients of rho and p, (d * 2 + s)
    double *prim = nullptr;      // 6 * ncell: rho, u, v, w, p, T of the state being differentiated
    double *prim2 = nullptr;     // 6 * ncell: second primitive buffer (gbr_step stages alternate)
    double *partial = nullptr;   // kReducePartials: per-block minima of the time-step reduction
    double *qn = nullptr;        // nvar * ncell: RK stage buffer (gbr_step) / batch stage buffer
    double *res = nullptr;       // nvar * ncell: RHS (gbr_step; float data in FP32-bulk)
    double *dt = nullptr;        // 1: time step of the last gbr_step / gbr_cfl
    unsigned long long *dtmin = nullptr;  // 1: min-reduction word (bit pattern of a positive double)
    int *flags = nullptr;        // [0] non-physical state, [1] non-positive Jacobian
    double *sigma = nullptr;     // ncell: sponge strength (gbr_set_sponge), or null
    double qref[5] = {0, 0, 0, 0, 0};  // sponge reference state, conserved
    bool bounded = false;        // some direction is non-periodic
    std::string err;
    // kernel timing (gbr_timing_enable): event pairs per launch
    bool timing = false;
    struct Rec { int cls; hipEvent_t a, b; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};

namespace gbr {

constexpr int kReducePartials = 4096;

// Ghost layers on each side of a non-periodic direction.
constexpr int kNg = GBR_NG;

// Dimensions and physics parameters passed by value to kernels. Cells with
// lo[d] <= index < hi[d] along every d are interior (advanced in time);
// lo = 0, hi = n along periodic directions.
struct Dims {
    int n[3];
    long ncell;
    int lo[3], hi[3];
};

__host__ __device__ inline bool in_box(const Dims &dm, int i, int j, int k)
{
    return i >= dm.lo[0] && i < dm.hi[0] && j >= dm.lo[1] && j < dm.hi[1] && k >= dm.lo[2] && k < dm.hi[2];
}

__host__ __device__ inline bool in_box(const Dims &dm, long idx)
{
    const int i = int(idx % dm.n[0]);
    const int j = int((idx / dm.n[0]) % dm.n[1]);
    const int k = int(idx / ((long)dm.n[0] * dm.n[1]));
    return in_box(dm, i, j, k);
}

struct Phys {
    double gamma;
    double gm1;       // gamma - 1
    double gM2;       // gamma Mref^2  (T = gM2 p / rho)
    double inv_gm1;   // 1 / (gamma - 1)
    double suth;      // Sutherland S / T_ref
    double re;        // Re: mu = Sutherland(T) / Re
    double kden;      // (gamma - 1) Mref^2 Pr: kappa = mu / kden
    double theta_c;
    double alpha_mp, beta_mp, alpha_d;
    int limiter;
};

// Metric slots kept in float for FP32-bulk grids (0 .. 47: the face slots
// and the cell unhatted metrics).
constexpr int kFloatMetricSlots = 48;

// Wide explicit stencils of the MIG4 gradient and of the metric derivative
// and interface interpolation built on it (gbr_stencil.hip).
constexpr int kIg4Half = 48;
constexpr int kIg4DHalf = kIg4Half + 2;
struct Ig4Stencil {
    double w[kIg4Half + 1];  // f'_i = sum_{j = 1..kIg4Half} w[j] (f_{i+j} - f_{i-j})
};
struct Ig4MetricStencil {
    double d[kIg4DHalf + 1];     // D f_i = sum_{j = 1..kIg4DHalf} d[j] (f_{i+j} - f_{i-j})
    double e[2 * kIg4Half + 4];  // I_{i+1/2} = sum_{m = -(H+1)..H+2} e[m + H + 1] f_{i+m}, H = kIg4Half
};
// Constants of the IG4 gradients as two first-order recurrences (k_ig4_rec):
// q and K of the factorised left-hand side, the right-hand-side weights a and
// b, and the powers pw[j] = (-q)^j.
struct Ig4Rec {
    double q, K, a, b;
    double pw[20];
};
const Ig4Stencil &ig4_stencil();
const Ig4Rec &ig4_rec();
const Ig4MetricStencil &ig4_metric_stencil();

Dims dims_of(const gbr_grid_s *g);
Phys phys_of(const gbr_grid_s *g);

// Brackets the launches of one kernel class with timing events when the
// grid's timing is enabled.
class Timed {
  public:
    Timed(gbr_grid_s *g, int cls);
    ~Timed();
    Timed(const Timed &) = delete;
    Timed &operator=(const Timed &) = delete;

  private:
    gbr_grid_s *g_;
    int cls_;
    hipEvent_t b_ = nullptr;
};

// Kernel launchers (enqueue on g->stream; return hipSuccess or the launch error).
hipError_t launch_metrics(gbr_grid_s *g, const double *xyz, const double *xyz_t);
hipError_t launch_metrics_nonfp(gbr_grid_s *g, const double *xyz);
// Refresh the float metric copy of an FP32-bulk grid (no-op otherwise).
hipError_t launch_metrics_float(gbr_grid_s *g);
hipError_t launch_rhs(gbr_grid_s *g, const double *Q, void *res);
hipError_t launch_rk_stage(gbr_grid_s *g, int stage, const double *dt, const double *Qn,
                           double *Q, const void *res);
// Diagnostics from the shared cell gradients (fields may be null, integrals
// may be null).
hipError_t launch_diagnostics(gbr_grid_s *g, const double *Q, double *fields, double *integrals);
// RHS and SSP-RK3 stage of gbr_step with the stage fused into the last sweep.
// Q: state at the start of the step, advanced in place; S: stage buffer.
// prims_ready: the first stage's primitives were formed by launch_cfl_prims.
hipError_t launch_step_stage(gbr_grid_s *g, int stage, const double *dt, double *Q, double *S,
                             bool prims_ready = false);
hipError_t launch_cfl(gbr_grid_s *g, const double *Q, double cfl, double *dt);
// launch_cfl with the per-block minima in `partial` (kReducePartials doubles)
// and no timing events.
hipError_t launch_cfl_into(gbr_grid_s *g, const double *Q, double cfl, double *dt, double *partial);
// launch_cfl plus the primitives of Q for the first stage of gbr_step.
hipError_t launch_cfl_prims(gbr_grid_s *g, const double *Q, double cfl, double *dt);
// Non-periodic boundaries (gbr_bounds.hip): App. C metrics of a static grid
// with ghost slots copied from the nearest interior ones; ghost primitives
// from the boundary types (Dirichlet ghosts from Q's own ghost cells); ghost
// states of Q after a step; ghost sensor values; sponge term added to Res.
hipError_t launch_metrics_bounded(gbr_grid_s *g, const double *xyz);
template <class R>
hipError_t launch_bc_prims(gbr_grid_s *g, R *prim, const double *Q);
hipError_t launch_bc_state(gbr_grid_s *g, double *Q);
hipError_t launch_flag_ghosts(gbr_grid_s *g, unsigned char *flag);
template <class R>
hipError_t launch_sponge(gbr_grid_s *g, const double *Q, R *res);
hipError_t launch_fill(gbr_grid_s *g, double *p, long n, double value);
hipError_t launch_copy(gbr_grid_s *g, double *dst, const double *src, long n);
// End of a gbr_step: dt_out = dt and t += dt (either may be null).
hipError_t launch_step_time(gbr_grid_s *g, const double *dt, double *dt_out, double *t);

}  // namespace gbr

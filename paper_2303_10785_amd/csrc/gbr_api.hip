// C ABI of libgbr (declared in include/gbr.h): argument checking, device
// buffer ownership and batching over grid handles. All arithmetic is in the
// kernels of gbr_metrics.hip and gbr_rhs.hip.
#include <cmath>
#include <cstdio>
#include <new>

#include "gbr_internal.hpp"

namespace gbr {

Dims dims_of(const gbr_grid_s *g)
{
    Dims d;
    for (int q = 0; q < 3; ++q) {
        d.n[q] = g->cfg.n[q];
        const bool b = g->cfg.bc[q][0] != GBR_BC_PERIODIC;
        d.lo[q] = b ? kNg : 0;
        d.hi[q] = b ? d.n[q] - kNg : d.n[q];
    }
    d.ncell = g->ncell;
    return d;
}

Phys phys_of(const gbr_grid_s *g)
{
    const gbr_config &c = g->cfg;
    Phys p;
    p.gamma = c.gamma;
    p.gm1 = c.gamma - 1.0;
    p.gM2 = c.gamma * c.Mref * c.Mref;
    p.inv_gm1 = 1.0 / (c.gamma - 1.0);
    p.suth = c.suth;
    p.re = c.Re;
    p.kden = (c.gamma - 1.0) * c.Mref * c.Mref * c.Pr;
    p.theta_c = c.theta_c;
    p.alpha_mp = c.alpha_mp;
    p.beta_mp = c.beta_mp;
    p.alpha_d = c.alpha_d;
    p.limiter = c.limiter;
    return p;
}

static hipEvent_t pooled_event(gbr_grid_s *g)
{
    if (!g->pool.empty()) {
        hipEvent_t e = g->pool.back();
        g->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

Timed::Timed(gbr_grid_s *g, int cls) : g_(g), cls_(cls)
{
    if (!g_->timing) return;
    b_ = pooled_event(g_);
    if (b_) (void)hipEventRecord(b_, g_->stream);
}

Timed::~Timed()
{
    if (!g_->timing || !b_) return;
    hipEvent_t e = pooled_event(g_);
    if (!e) {
        g_->pool.push_back(b_);
        return;
    }
    (void)hipEventRecord(e, g_->stream);
    g_->recs.push_back({cls_, b_, e});
}

}  // namespace gbr

namespace {

const char *kNullHandle = "null grid handle";

bool config_ok(const gbr_config *c, const char **why)
{
    if (!c) return *why = "null config", false;
    if (c->ndim != 2 && c->ndim != 3) return *why = "ndim must be 2 or 3", false;
    for (int q = 0; q < 3; ++q)
        if (c->n[q] < 1) return *why = "cell counts must be >= 1", false;
    if (c->ndim == 2 && c->n[2] != 1) return *why = "2-D grids need n[2] == 1", false;
    if ((long long)c->n[0] * c->n[1] * c->n[2] > (1ll << 31))
        return *why = "grid larger than 2^31 cells", false;
    if (c->limiter < GBR_LIM_NONE || c->limiter > GBR_LIM_DUCROS) return *why = "unknown limiter", false;
    if (c->precision != GBR_FP64 && c->precision != GBR_FP32_BULK) return *why = "unsupported precision", false;
    if (c->scheme != GBR_SCHEME_MEG6 && c->scheme != GBR_SCHEME_MIG4) return *why = "unknown scheme", false;
    if (!(c->gamma > 1.0) || !(c->Re > 0.0) || !(c->Pr > 0.0) || !(c->Mref > 0.0) || !(c->suth >= 0.0))
        return *why = "gamma must exceed 1 and Re, Pr, Mref be positive", false;
    for (int d = 0; d < 3; ++d) {
        for (int side = 0; side < 2; ++side)
            if (c->bc[d][side] < GBR_BC_PERIODIC || c->bc[d][side] > GBR_BC_WALL)
                return *why = "unknown boundary type", false;
        const bool lo = c->bc[d][0] != GBR_BC_PERIODIC, hi = c->bc[d][1] != GBR_BC_PERIODIC;
        if (lo != hi) return *why = "a direction is periodic on both sides or on neither", false;
        if (lo && (d >= c->ndim || c->n[d] < 2 * GBR_NG + 12))
            return *why = "a bounded direction needs d < ndim and n[d] >= 2 GBR_NG + 12", false;
    }
    return true;
}

bool any_bounded(const gbr_config *c)
{
    for (int d = 0; d < 3; ++d)
        if (c->bc[d][0] != GBR_BC_PERIODIC) return true;
    return false;
}

size_t bytes_for(const gbr_config *c)
{
    size_t N = (size_t)c->n[0] * c->n[1] * c->n[2];
    size_t nv = (size_t)c->ndim + 2;
    size_t doubles = N * (GBR_SLOT_COUNT + 12 + 12 + 2 * nv + (c->scheme == GBR_SCHEME_MIG4 ? 6 : 0)) + 1 +
                     gbr::kReducePartials;
    const size_t floats = (c->precision == GBR_FP32_BULK) ? N * gbr::kFloatMetricSlots : 0;
    return doubles * sizeof(double) + floats * sizeof(float) + N + sizeof(unsigned long long) + 2 * sizeof(int);
}

gbr_status fail(gbr_grid_s *g, gbr_status s, const char *msg)
{
    if (g) g->err = msg;
    return s;
}

gbr_status hip_fail(gbr_grid_s *g, hipError_t e, const char *where)
{
    if (g) {
        char buf[256];
        std::snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
        g->err = buf;
    }
    return e == hipErrorOutOfMemory ? GBR_E_NOMEM : GBR_E_DEVICE;
}

void drop_records(gbr_grid_s *g)
{
    for (auto &r : g->recs) {
        g->pool.push_back(r.a);
        g->pool.push_back(r.b);
    }
    g->recs.clear();
}

void release(gbr_grid_s *g)
{
    if (!g) return;
    drop_records(g);
    for (hipEvent_t e : g->pool) (void)hipEventDestroy(e);
    g->pool.clear();
    for (void *p : {(void *)g->metrics, (void *)g->metrics_f, (void *)g->scratch, (void *)g->lim_flag,
                    (void *)g->grad2, (void *)g->prim, (void *)g->prim2, (void *)g->sigma,
                    (void *)g->partial, (void *)g->qn,
                    (void *)g->res, (void *)g->dt, (void *)g->dtmin, (void *)g->flags})
        if (p) (void)hipFree(p);
    delete g;
}

// Check the batch arguments shared by every batched call.
gbr_status batch_ok(const gbr_grid *g, int n)
{
    if (n < 0) return GBR_E_ARG;
    if (n > 0 && !g) return GBR_E_ARG;
    for (int b = 0; b < n; ++b)
        if (!g[b]) return GBR_E_ARG;
    return GBR_OK;
}

}  // namespace

extern "C" {

size_t gbr_grid_bytes(const gbr_config *cfg)
{
    const char *why;
    return config_ok(cfg, &why) ? bytes_for(cfg) : 0;
}

gbr_status gbr_grid_create(const gbr_config *cfg, void *hip_stream, gbr_grid *out)
{
    if (!out) return GBR_E_ARG;
    *out = nullptr;
    const char *why = nullptr;
    if (!config_ok(cfg, &why)) return GBR_E_ARG;
    // App. C covers static grids; the IG4 line system has no boundary closure
    // in the paper
    if (any_bounded(cfg) && (cfg->moving || cfg->scheme != GBR_SCHEME_MEG6)) return GBR_E_UNSUPPORTED;
    gbr_grid_s *g = new (std::nothrow) gbr_grid_s;
    if (!g) return GBR_E_NOMEM;
    g->cfg = *cfg;
    g->bounded = any_bounded(cfg);
    g->stream = (hipStream_t)hip_stream;
    g->ncell = (long)cfg->n[0] * cfg->n[1] * cfg->n[2];
    g->nvar = cfg->ndim + 2;
    hipError_t e = hipGetDevice(&g->device);
    size_t N = (size_t)g->ncell;
    auto alloc = [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes);
    };
    alloc((void **)&g->metrics, N * GBR_SLOT_COUNT * sizeof(double));
    if (cfg->precision == GBR_FP32_BULK) alloc((void **)&g->metrics_f, N * gbr::kFloatMetricSlots * sizeof(float));
    alloc((void **)&g->scratch, N * 12 * sizeof(double));
    alloc((void **)&g->lim_flag, N);
    if (cfg->scheme == GBR_SCHEME_MIG4) alloc((void **)&g->grad2, N * 6 * sizeof(double));
    alloc((void **)&g->prim, N * 6 * sizeof(double));
    alloc((void **)&g->prim2, N * 6 * sizeof(double));
    alloc((void **)&g->partial, gbr::kReducePartials * sizeof(double));
    alloc((void **)&g->qn, N * g->nvar * sizeof(double));
    alloc((void **)&g->res, N * g->nvar * sizeof(double));
    alloc((void **)&g->dt, sizeof(double));
    alloc((void **)&g->dtmin, sizeof(unsigned long long));
    alloc((void **)&g->flags, 2 * sizeof(int));
    if (e == hipSuccess) e = hipMemsetAsync(g->flags, 0, 2 * sizeof(int), g->stream);
    if (e == hipSuccess) e = hipMemsetAsync(g->metrics, 0, N * GBR_SLOT_COUNT * sizeof(double), g->stream);
    if (e == hipSuccess && g->metrics_f)
        e = hipMemsetAsync(g->metrics_f, 0, N * gbr::kFloatMetricSlots * sizeof(float), g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) {
        gbr_status s = (e == hipErrorOutOfMemory) ? GBR_E_NOMEM : GBR_E_DEVICE;
        release(g);
        return s;
    }
    *out = g;
    return GBR_OK;
}

gbr_status gbr_grid_destroy(gbr_grid g)
{
    if (!g) return GBR_OK;
    (void)hipStreamSynchronize(g->stream);
    release(g);
    return GBR_OK;
}

gbr_status gbr_set_stream(gbr_grid g, void *hip_stream)
{
    if (!g) return GBR_E_ARG;
    g->stream = (hipStream_t)hip_stream;
    return GBR_OK;
}

gbr_status gbr_metrics(const gbr_grid *g, int n, const double *const *xyz, const double *const *xyz_t)
{
    gbr_status s = batch_ok(g, n);
    if (s != GBR_OK) return s;
    if (n == 0) return GBR_OK;
    if (!xyz) return fail(g[0], GBR_E_ARG, "null coordinate array");
    for (int b = 0; b < n; ++b) {
        gbr_grid_s *gg = g[b];
        if (!xyz[b]) return fail(gg, GBR_E_ARG, "null coordinates");
        const double *xt = xyz_t ? xyz_t[b] : nullptr;
        if (gg->cfg.moving && !xt) return fail(gg, GBR_E_ARG, "moving grid needs grid velocities");
        hipError_t e = hipMemsetAsync(gg->flags + 1, 0, sizeof(int), gg->stream);
        if (e == hipSuccess)
            e = gg->bounded ? gbr::launch_metrics_bounded(gg, xyz[b]) : gbr::launch_metrics(gg, xyz[b], xt);
        if (e != hipSuccess) return hip_fail(gg, e, "metrics launch");
    }
    for (int b = 0; b < n; ++b) {
        gbr_grid_s *gg = g[b];
        int flag = 0;
        hipError_t e = hipMemcpyAsync(&flag, gg->flags + 1, sizeof(int), hipMemcpyDeviceToHost, gg->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(gg->stream);
        if (e != hipSuccess) return hip_fail(gg, e, "metrics sync");
        if (flag) return fail(gg, GBR_E_JACOBIAN, "non-positive Jacobian (folded or left-handed grid)");
    }
    return GBR_OK;
}

gbr_status gbr_metrics_nonfp(const gbr_grid *g, int n, const double *const *xyz)
{
    gbr_status s = batch_ok(g, n);
    if (s != GBR_OK) return s;
    if (n == 0) return GBR_OK;
    if (!xyz) return fail(g[0], GBR_E_ARG, "null coordinate array");
    for (int b = 0; b < n; ++b) {
        gbr_grid_s *gg = g[b];
        if (!xyz[b]) return fail(gg, GBR_E_ARG, "null coordinates");
        if (gg->cfg.moving) return fail(gg, GBR_E_UNSUPPORTED, "non-conservative metrics are for static grids");
        if (gg->bounded) return fail(gg, GBR_E_UNSUPPORTED, "non-conservative metrics are for periodic grids");
        hipError_t e = hipMemsetAsync(gg->flags + 1, 0, sizeof(int), gg->stream);
        if (e == hipSuccess) e = gbr::launch_metrics_nonfp(gg, xyz[b]);
        if (e != hipSuccess) return hip_fail(gg, e, "metrics launch");
    }
    for (int b = 0; b < n; ++b) {
        gbr_grid_s *gg = g[b];
        int flag = 0;
        hipError_t e = hipMemcpyAsync(&flag, gg->flags + 1, sizeof(int), hipMemcpyDeviceToHost, gg->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(gg->stream);
        if (e != hipSuccess) return hip_fail(gg, e, "metrics sync");
        if (flag) return fail(gg, GBR_E_JACOBIAN, "non-positive Jacobian (folded or left-handed grid)");
    }
    return GBR_OK;
}

gbr_status gbr_rhs(const gbr_grid *g, int n, const double *const *Q, void *const *res)
{
    gbr_status s = batch_ok(g, n);
    if (s != GBR_OK) return s;
    if (n == 0) return GBR_OK;
    if (!Q || !res) return fail(g[0], GBR_E_ARG, "null state or residual array");
    for (int b = 0; b < n; ++b) {
        if (!Q[b] || !res[b]) return fail(g[b], GBR_E_ARG, "null state or residual");
        if ((const void *)Q[b] == res[b]) return fail(g[b], GBR_E_ARG, "residual aliases the state");
        hipError_t e = gbr::launch_rhs(g[b], Q[b], res[b]);
        if (e != hipSuccess) return hip_fail(g[b], e, "rhs launch");
    }
    return GBR_OK;
}

gbr_status gbr_rk_stage(const gbr_grid *g, int n, int stage, const double *const *dt,
                        const double *const *Qn, double *const *Q, const void *const *res)
{
    gbr_status s = batch_ok(g, n);
    if (s != GBR_OK) return s;
    if (n == 0) return GBR_OK;
    if (stage < 0 || stage > 2) return fail(g[0], GBR_E_ARG, "stage must be 0, 1 or 2");
    if (!dt || !Qn || !Q || !res) return fail(g[0], GBR_E_ARG, "null pointer array");
    for (int b = 0; b < n; ++b) {
        if (!dt[b] || !Qn[b] || !Q[b] || !res[b]) return fail(g[b], GBR_E_ARG, "null pointer");
        hipError_t e = gbr::launch_rk_stage(g[b], stage, dt[b], Qn[b], Q[b], res[b]);
        if (e != hipSuccess) return hip_fail(g[b], e, "rk stage launch");
    }
    return GBR_OK;
}

gbr_status gbr_cfl(const gbr_grid *g, int n, const double *const *Q, double cfl, double *const *dt)
{
    gbr_status s = batch_ok(g, n);
    if (s != GBR_OK) return s;
    if (n == 0) return GBR_OK;
    if (!Q || !dt) return fail(g[0], GBR_E_ARG, "null pointer array");
    if (!(cfl > 0.0)) return fail(g[0], GBR_E_ARG, "cfl must be positive");
    for (int b = 0; b < n; ++b) {
        if (!Q[b] || !dt[b]) return fail(g[b], GBR_E_ARG, "null pointer");
        hipError_t e = gbr::launch_cfl(g[b], Q[b], cfl, dt[b]);
        if (e != hipSuccess) return hip_fail(g[b], e, "cfl launch");
    }
    return GBR_OK;
}

gbr_status gbr_step(const gbr_grid *g, int n, double *const *Q, const double *const *xyz,
                    const double *const *xyz_t, double cfl_or_dt, int dt_mode, double *const *dt_out,
                    double *const *t)
{
    gbr_status s = batch_ok(g, n);
    if (s != GBR_OK) return s;
    if (n == 0) return GBR_OK;
    if (!Q) return fail(g[0], GBR_E_ARG, "null state array");
    if (dt_mode != GBR_DT_CFL && dt_mode != GBR_DT_FIXED) return fail(g[0], GBR_E_ARG, "unknown dt mode");
    if (!(cfl_or_dt > 0.0)) return fail(g[0], GBR_E_ARG, "cfl / dt must be positive");
    for (int b = 0; b < n; ++b) {
        gbr_grid_s *gg = g[b];
        if (!Q[b]) return fail(gg, GBR_E_ARG, "null state");
        double *dto = dt_out ? dt_out[b] : nullptr, *tb = t ? t[b] : nullptr;
        if (dto && dto == tb) return fail(gg, GBR_E_ARG, "time and time-step outputs alias");
        hipError_t e = hipSuccess;
        if (gg->cfg.moving) {
            const double *x = xyz ? xyz[b] : nullptr;
            const double *xt = xyz_t ? xyz_t[b] : nullptr;
            if (!x || !xt) return fail(gg, GBR_E_ARG, "moving grid needs coordinates and velocities");
            e = gbr::launch_metrics(gg, x, xt);
        }
        if (e == hipSuccess) {
            if (dt_mode == GBR_DT_CFL)
                e = gbr::launch_cfl_prims(gg, Q[b], cfl_or_dt, gg->dt);
            else
                e = gbr::launch_fill(gg, gg->dt, 1, cfl_or_dt);
        }
        const bool prims_ready = dt_mode == GBR_DT_CFL;
        for (int st = 0; st < 3 && e == hipSuccess; ++st)
            e = gbr::launch_step_stage(gg, st, gg->dt, Q[b], gg->qn, st == 0 && prims_ready);
        if (e == hipSuccess && gg->bounded) e = gbr::launch_bc_state(gg, Q[b]);
        if (e == hipSuccess && (dto || tb)) e = gbr::launch_step_time(gg, gg->dt, dto, tb);
        if (e != hipSuccess) return hip_fail(gg, e, "step launch");
    }
    return GBR_OK;
}

gbr_status gbr_diagnostics(const gbr_grid *g, int n, const double *const *Q, double *const *fields,
                           double *const *integrals)
{
    gbr_status s = batch_ok(g, n);
    if (s != GBR_OK) return s;
    if (n == 0) return GBR_OK;
    if (!Q) return fail(g[0], GBR_E_ARG, "null state array");
    for (int b = 0; b < n; ++b) {
        if (!Q[b]) return fail(g[b], GBR_E_ARG, "null state");
        if (g[b]->bounded) return fail(g[b], GBR_E_UNSUPPORTED, "diagnostics are for periodic grids");
        hipError_t e = gbr::launch_diagnostics(g[b], Q[b], fields ? fields[b] : nullptr,
                                               integrals ? integrals[b] : nullptr);
        if (e != hipSuccess) return hip_fail(g[b], e, "diagnostics launch");
    }
    return GBR_OK;
}

gbr_status gbr_check_state(gbr_grid g)
{
    if (!g) return GBR_E_ARG;
    int flags[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(flags, g->flags, sizeof flags, hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e == hipSuccess) e = hipMemsetAsync(g->flags, 0, sizeof flags, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "state check");
    if (flags[1]) return fail(g, GBR_E_JACOBIAN, "non-positive Jacobian in a metric update");
    if (flags[0]) return fail(g, GBR_E_STATE, "non-physical state (rho <= 0, p <= 0 or non-finite)");
    return GBR_OK;
}

gbr_status gbr_set_sponge(gbr_grid g, const double *sigma, const double *ref)
{
    if (!g) return GBR_E_ARG;
    if (!sigma) {
        hipError_t e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) return hip_fail(g, e, "sponge sync");
        if (g->sigma) (void)hipFree(g->sigma);
        g->sigma = nullptr;
        return GBR_OK;
    }
    if (!ref) return fail(g, GBR_E_ARG, "null sponge reference state");
    if (!(ref[0] > 0.0) || !(ref[4] > 0.0)) return fail(g, GBR_E_ARG, "sponge reference needs rho, p > 0");
    hipError_t e = hipSuccess;
    if (!g->sigma) e = hipMalloc((void **)&g->sigma, (size_t)g->ncell * sizeof(double));
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->sigma, sigma, (size_t)g->ncell * sizeof(double), hipMemcpyDeviceToDevice, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "sponge copy");
    const double w = g->cfg.ndim == 3 ? ref[3] : 0.0;
    g->qref[0] = ref[0];
    g->qref[1] = ref[0] * ref[1];
    g->qref[2] = ref[0] * ref[2];
    g->qref[3] = ref[0] * w;
    g->qref[4] = ref[4] / (g->cfg.gamma - 1.0) + 0.5 * ref[0] * (ref[1] * ref[1] + ref[2] * ref[2] + w * w);
    return GBR_OK;
}

const double *gbr_metric_ptr(gbr_grid g, int slot)
{
    if (!g || slot < 0 || slot >= GBR_SLOT_COUNT) return nullptr;
    return g->metrics + (long)slot * g->ncell;
}

gbr_status gbr_timing_enable(gbr_grid g, int on)
{
    if (!g) return GBR_E_ARG;
    if (!on) {
        (void)hipStreamSynchronize(g->stream);
        drop_records(g);
    }
    g->timing = on != 0;
    return GBR_OK;
}

gbr_status gbr_timing_collect(gbr_grid g, double *ms, long *launches)
{
    if (!g || !ms || !launches) return GBR_E_ARG;
    hipError_t e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return hip_fail(g, e, "timing sync");
    for (auto &r : g->recs) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess && r.cls >= 0 && r.cls < GBR_K_COUNT) {
            ms[r.cls] += t;
            launches[r.cls] += 1;
        }
    }
    drop_records(g);
    return GBR_OK;
}

const char *gbr_last_error(gbr_grid g)
{
    if (!g) return kNullHandle;
    return g->err.c_str();
}

}  // extern "C"

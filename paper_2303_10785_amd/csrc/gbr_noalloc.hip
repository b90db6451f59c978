// gbr_cfl_noalloc: the time step of gbr_cfl with its per-block partial minima
// in a static device array instead of the grid's allocated buffer, for
// callers that cannot allocate device memory (code under stream capture,
// tight serving loops). Nothing here calls hipMalloc or hipFree.
#include <mutex>

#include "gbr_internal.hpp"

namespace {

// One slice of per-block partial minima per grid of a call.
constexpr int kNoallocGrids = 32;
constexpr int kMaxDevices = 64;

}  // namespace

// Static scratch of gbr_cfl_noalloc (1 MiB on every device the library runs
// on, held until the process ends). In host code this name is only a handle
// for hipGetSymbolAddress: kernels receive the device address looked up per
// device below, never the name itself.
static __device__ __align__(256) double scratch[kNoallocGrids * gbr::kReducePartials];

namespace {

std::mutex scratch_mu;
double *scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current.
hipError_t scratch_on(int device, double **out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_ptr[device] = static_cast<double *>(p);
    }
    *out = scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

extern "C" gbr_status gbr_cfl_noalloc(const gbr_grid *g, int n, const double *const *Q, double cfl,
                                      double *const *dt)
{
    if (n < 0 || (n > 0 && !g)) return GBR_E_ARG;
    for (int b = 0; b < n; ++b)
        if (!g[b]) return GBR_E_ARG;
    if (n == 0) return GBR_OK;
    if (n > kNoallocGrids) {
        g[0]->err = "gbr_cfl_noalloc takes at most 32 grids per call (one static scratch slice each)";
        return GBR_E_ARG;
    }
    if (!Q || !dt) {
        g[0]->err = "null pointer array";
        return GBR_E_ARG;
    }
    if (!(cfl > 0.0)) {
        g[0]->err = "cfl must be positive";
        return GBR_E_ARG;
    }
    for (int b = 0; b < n; ++b)
        if (!Q[b] || !dt[b]) {
            g[b]->err = "null pointer";
            return GBR_E_ARG;
        }
    for (int b = 0; b < n; ++b) {
        double *base = nullptr;
        hipError_t e = scratch_on(g[b]->device, &base);
        if (e == hipSuccess)
            e = gbr::launch_cfl_into(g[b], Q[b], cfl, dt[b], base + (size_t)b * gbr::kReducePartials);
        if (e != hipSuccess) {
            g[b]->err = std::string("gbr_cfl_noalloc: ") + hipGetErrorString(e);
            return GBR_E_DEVICE;
        }
    }
    return GBR_OK;
}

// Measurement probe: the STREAM triad a = b + s c, a pure streaming kernel
// whose bandwidth is the achievable HBM rate against which the solver's
// kernels are reported. It is not part of the solver.
#include <hip/hip_runtime.h>

#include "gbr.h"

namespace {

constexpr int kBlock = 256;
constexpr int kPerThread = 4;  // double2 elements per thread, kBlock apart (coalesced)

__global__ void __launch_bounds__(kBlock) k_triad(double2 *__restrict__ a, const double2 *__restrict__ b,
                                                  const double2 *__restrict__ c, double s, long n2)
{
    const long base = (long)blockIdx.x * (kBlock * kPerThread) + threadIdx.x;
    double2 x[kPerThread], y[kPerThread];
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
        const long e = base + (long)q * kBlock;
        if (e < n2) {
            x[q] = b[e];
            y[q] = c[e];
        }
    }
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
        const long e = base + (long)q * kBlock;
        if (e < n2) a[e] = make_double2(x[q].x + s * y[q].x, x[q].y + s * y[q].y);
    }
}

__global__ void k_triad_tail(double *a, const double *b, const double *c, double s)
{
    if (threadIdx.x == 0) a[0] = b[0] + s * c[0];
}

}  // namespace

extern "C" gbr_status gbr_probe_triad(double *a, const double *b, const double *c, double s, long n,
                                      void *hip_stream)
{
    if (n < 0 || (n > 0 && (!a || !b || !c))) return GBR_E_ARG;
    if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) % 16 != 0) return GBR_E_ARG;
    if (n == 0) return GBR_OK;
    hipStream_t st = (hipStream_t)hip_stream;
    const long n2 = n / 2;
    if (n2 > 0) {
        const long per_block = (long)kBlock * kPerThread;
        const long blocks = (n2 + per_block - 1) / per_block;
        if (blocks > 0x7fffffffL) return GBR_E_ARG;
        hipLaunchKernelGGL(k_triad, dim3((unsigned)blocks), dim3(kBlock), 0, st, (double2 *)a,
                           (const double2 *)b, (const double2 *)c, s, n2);
    }
    if (n % 2) hipLaunchKernelGGL(k_triad_tail, dim3(1), dim3(64), 0, st, a + n - 1, b + n - 1, c + n - 1, s);
    return hipGetLastError() == hipSuccess ? GBR_OK : GBR_E_DEVICE;
}

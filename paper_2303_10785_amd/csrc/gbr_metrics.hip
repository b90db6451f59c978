// Metric kernels (Sec. 4.2, Sec. 7): conservative metrics, Jacobian,
// interface values and GCL terms. FP64 throughout.
//
// Data flow (each a grid-wide kernel; one thread per cell):
//   k_coord_deriv : D_d x_c of the periodic extension of the coordinates
//                   (9 values per cell, into the scratch buffer)
//   k_cell_metrics: hat(d)_c = D_d2[(c1)_d1 c2] - D_d1[(c1)_d2 c2] with the
//                   products formed from the coordinates extended around the
//                   cell, 1/J = det[D_d x_c], J, unhatted d_c = J hat(d)_c,
//                   temporal metrics on moving grids
//   k_face_metrics: interface values of the 3 hatted f-metrics, hat f_t and
//                   all 9 unhatted metrics for each family f (MEG6: from LDS
//                   tiles, k_face_metrics_xi and k_face_metrics_tiled)
//   k_gcl         : (1/J)_t = -sum_f [I_f hat f_t](+1/2) - [...](-1/2)
#include "gbr_device.hpp"
#include "gbr_internal.hpp"

namespace gbr {
namespace {

constexpr int kBlock = 256;

struct MetricArgs {
    Dims dm;
    int ndim;
    double off[3][3];
    const double *xyz;
    const double *xyz_t;
    double *dx;      // 9 * ncell
    double *m;       // GBR_SLOT_COUNT * ncell
    int *flags;
};

__device__ __forceinline__ void unpack(const Dims &dm, long idx, int ijk[3])
{
    ijk[0] = int(idx % dm.n[0]);
    ijk[1] = int((idx / dm.n[0]) % dm.n[1]);
    ijk[2] = int(idx / ((long)dm.n[0] * dm.n[1]));
}

__device__ __forceinline__ long pack(const Dims &dm, int i, int j, int k)
{
    return i + (long)dm.n[0] * (j + (long)dm.n[1] * k);
}

// Linear index of the neighbour q steps along d, and how many periods it crossed.
__device__ __forceinline__ long step_to(const Dims &dm, const int ijk[3], int d, int q, int *wraps)
{
    int t[3] = {ijk[0], ijk[1], ijk[2]};
    int a = t[d] + q;
    t[d] = wrap_index(a, dm.n[d]);
    if (wraps) *wraps = wrap_count(a, dm.n[d]);
    return pack(dm, t[0], t[1], t[2]);
}

// step_to for |q| <= n[d]: the neighbour then lies at most one period away,
// so one comparison gives the period count and the index follows from the
// cell's own (same results as step_to, without the integer divisions).
__device__ __forceinline__ long step_near(const Dims &dm, const int ijk[3], int d, int q, long idx, long sd,
                                         int *wraps)
{
    const int n = dm.n[d], a = ijk[d] + q;
    const int w = a < 0 ? -1 : (a >= n ? 1 : 0);
    if (wraps) *wraps = w;
    return idx + (long)(q - w * n) * sd;
}

// Coordinate c at linear index nb (z is the zeta index in 2-D).
__device__ __forceinline__ double coord(const MetricArgs &a, int c, long nb)
{
    if (c == 2 && a.ndim == 2) return 0.0;
    return a.xyz[c * a.dm.ncell + nb];
}

// Composite central derivative (Eq. FP-interp2) at the window centre of the
// extended values f(q), q = offset along the line: the closed 11-point form
// for MEG6, the wide IG4-based stencil for MIG4 (Sec. 7).
template <bool IG4, class F>
__device__ __forceinline__ double composite(const Ig4MetricStencil &s, F f)
{
    if (IG4) {
        double acc = 0.0;
        for (int j = 1; j <= kIg4DHalf; ++j) acc += s.d[j] * (f(j) - f(-j));
        return acc;
    }
    double v[11];
#pragma unroll
    for (int q = -5; q <= 5; ++q) v[q + 5] = f(q);
    return dcomp(v + 5);
}

// Interface value at +1/2 (Eq. FP-interp / interp-formulae) of f(q).
template <bool IG4, class F>
__device__ __forceinline__ double interface(const Ig4MetricStencil &s, F f)
{
    if (IG4) {
        double acc = 0.0;
        for (int m = -(kIg4Half + 1); m <= kIg4Half + 2; ++m) acc += s.e[m + kIg4Half + 1] * f(m);
        return acc;
    }
    double v[10];
#pragma unroll
    for (int q = -4; q <= 5; ++q) v[q + 4] = f(q);
    return face_interp(v + 4);
}

// Windows of the composite derivative: half-width along the line.
template <bool IG4>
constexpr int window_half() { return IG4 ? kIg4DHalf : 5; }

// Whether the window of cell ijk along d, or of another cell of the same
// wavefront, reaches across the periodic seam (then neighbours enter as
// periodic images); away from it a neighbour at offset q is the cell q
// strides along d. Decided per wavefront, so both window forms never run
// under one mask; image_rel gives the plain difference for cells whose
// window does not wrap.
template <bool IG4>
__device__ __forceinline__ bool near_seam(const Dims &dm, const int ijk[3], int d)
{
    return __any(ijk[d] < window_half<IG4>() || ijk[d] >= dm.n[d] - window_half<IG4>());
}

__device__ __forceinline__ long stride_of(const Dims &dm, int d)
{
    return d == 0 ? 1 : (d == 1 ? (long)dm.n[0] : (long)dm.n[0] * dm.n[1]);
}

// Neighbour q steps along d (and the periods crossed) for windows reaching
// at most `reach` cells: step_near when the line is at least that long
// (uniform over the grid), step_to otherwise.
__device__ __forceinline__ long neighbour(const Dims &dm, const int ijk[3], int d, int q, long idx, int reach,
                                         int *wraps)
{
    return dm.n[d] >= reach ? step_near(dm, ijk, d, q, idx, stride_of(dm, d), wraps)
                            : step_to(dm, ijk, d, q, wraps);
}

template <bool IG4>
__global__ void __launch_bounds__(kBlock) k_coord_deriv(MetricArgs a, Ig4MetricStencil st)
{
    long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx >= a.dm.ncell) return;
    int ijk[3];
    unpack(a.dm, idx, ijk);
    // Coordinates are measured from the cell's own centre: the metrics are
    // translation invariant and this avoids cancellation of O(|x| / dx).
    // Across the periodic seam the image is placed relative to the centre
    // with one rounding (image_rel).
    for (int d = 0; d < 3; ++d) {
        const bool seam = near_seam<IG4>(a.dm, ijk, d);
        const long sd = stride_of(a.dm, d);
        for (int c = 0; c < 3; ++c) {
            const double org = coord(a, c, idx);
            a.dx[(d * 3 + c) * a.dm.ncell + idx] =
                seam ? composite<IG4>(st, [&](int q) {
                    int wr;
                    long nb = neighbour(a.dm, ijk, d, q, idx, window_half<IG4>(), &wr);
                    return image_rel(coord(a, c, nb), wr, a.off[d][c], org);
                })
                     : composite<IG4>(st, [&](int q) { return coord(a, c, idx + q * sd) - org; });
        }
    }
}

template <bool IG4>
__global__ void __launch_bounds__(kBlock) k_cell_metrics(MetricArgs a, Ig4MetricStencil st)
{
    long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx >= a.dm.ncell) return;
    const long N = a.dm.ncell;
    int ijk[3];
    unpack(a.dm, idx, ijk);
    double hat[3][3];
    // D_e of (c1)_f * c2 along direction e at this cell, c2 measured from org
    auto dprod = [&](int e, int f, int c1, int c2, double org) {
        const double *fac = a.dx + (f * 3 + c1) * N;
        if (near_seam<IG4>(a.dm, ijk, e))
            return composite<IG4>(st, [&](int q) {
                int wr;
                long nb = neighbour(a.dm, ijk, e, q, idx, window_half<IG4>(), &wr);
                return fac[nb] * image_rel(coord(a, c2, nb), wr, a.off[e][c2], org);
            });
        const long se = stride_of(a.dm, e);
        return composite<IG4>(st, [&](int q) {
            const long nb = idx + q * se;
            return fac[nb] * (coord(a, c2, nb) - org);
        });
    };
    for (int d = 0; d < 3; ++d) {
        const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        for (int c = 0; c < 3; ++c) {
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            const double org = coord(a, c2, idx);
            hat[d][c] = dprod(d2, d1, c1, c2, org) - dprod(d1, d2, c1, c2, org);
        }
    }
    double x[3][3];
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) x[d][c] = a.dx[(d * 3 + c) * N + idx];
    double invj = x[0][0] * (x[1][1] * x[2][2] - x[1][2] * x[2][1]) -
                  x[0][1] * (x[1][0] * x[2][2] - x[1][2] * x[2][0]) +
                  x[0][2] * (x[1][0] * x[2][1] - x[1][1] * x[2][0]);
    if (!(invj > 0.0)) atomicOr(a.flags + 1, 1);
    double jac = 1.0 / invj;
    double *m = a.m;
    m[GBR_SLOT_CELL_INVJ * N + idx] = invj;
    m[GBR_SLOT_CELL_J * N + idx] = jac;
    for (int d = 0; d < 3; ++d) {
        for (int c = 0; c < 3; ++c) {
            m[GBR_SLOT_CELL_HAT(d, c) * N + idx] = hat[d][c];
            m[GBR_SLOT_CELL_UNHAT(d, c) * N + idx] = hat[d][c] / invj;
        }
        double ht = 0.0;
        if (a.xyz_t) {
            ht = -(a.xyz_t[idx] * hat[d][0] + a.xyz_t[N + idx] * hat[d][1] +
                   (a.ndim == 3 ? a.xyz_t[2 * N + idx] * hat[d][2] : 0.0));
        }
        m[GBR_SLOT_CELL_HATT(d) * N + idx] = ht;
        m[GBR_SLOT_CELL_UNHATT(d) * N + idx] = ht * jac;
    }
}

template <bool IG4>
__global__ void __launch_bounds__(kBlock) k_face_metrics(MetricArgs a, Ig4MetricStencil st, int fmask)
{
    long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx >= a.dm.ncell) return;
    const long N = a.dm.ncell;
    int ijk[3];
    unpack(a.dm, idx, ijk);
    double *m = a.m;
    for (int f = 0; f < 3; ++f) {
        if (!((fmask >> f) & 1)) continue;
        long nb[10];  // MEG6 window, reused by every slot
        if (!IG4)
            for (int q = -4; q <= 5; ++q) nb[q + 4] = neighbour(a.dm, ijk, f, q, idx, 5, nullptr);
        auto interp = [&](int slot) {
            const double *s = m + slot * N;
            // (the 100-point IG4 window keeps step_to: a per-point choice
            // inside that loop cost more than the modulos it saves)
            return interface<IG4>(st, [&](int q) { return IG4 ? s[step_to(a.dm, ijk, f, q, nullptr)] : s[nb[q + 4]]; });
        };
        for (int c = 0; c < 3; ++c) m[GBR_SLOT_FACE_HAT(f, c) * N + idx] = interp(GBR_SLOT_CELL_HAT(f, c));
        m[GBR_SLOT_FACE_HATT(f) * N + idx] = interp(GBR_SLOT_CELL_HATT(f));
        for (int e = 0; e < 3; ++e)
            for (int c = 0; c < 3; ++c)
                m[GBR_SLOT_FACE_UNHAT(f, e, c) * N + idx] = interp(GBR_SLOT_CELL_UNHAT(e, c));
    }
}

// MEG6 interface values of family F = 1 (eta) or 2 (zeta) from LDS tiles:
// a workgroup owns FT interfaces along F for FC consecutive cells along i
// and stages the 13 source slots of cells s0-4 .. s0+FT+4 once (each
// interface's 10-point window then reads LDS instead of L2). Same formula on
// the same values as k_face_metrics.
constexpr int FT = 16, FC = kBlock / FT, FNP = FT + 9;

template <int F>
__global__ void __launch_bounds__(kBlock) k_face_metrics_tiled(MetricArgs a)
{
    constexpr int OD = (F == 1) ? 2 : 1;  // the remaining direction
    __shared__ double sv[13][FNP * FC];
    const Dims &dm = a.dm;
    const long N = dm.ncell;
    const int ns = dm.n[F], nc = dm.n[0];
    const int tiles_s = (ns + FT - 1) / FT;
    const int s0 = (blockIdx.x % tiles_s) * FT;
    const int c0 = (blockIdx.x / tiles_s) * FC;
    const int o = blockIdx.y;
    int src[13];
    for (int c = 0; c < 3; ++c) src[c] = GBR_SLOT_CELL_HAT(F, c);
    src[3] = GBR_SLOT_CELL_HATT(F);
    for (int e = 0; e < 3; ++e)
        for (int c = 0; c < 3; ++c) src[4 + e * 3 + c] = GBR_SLOT_CELL_UNHAT(e, c);
    for (int e = threadIdx.x; e < FNP * FC; e += kBlock) {
        const int sl = e / FC, cl = e % FC;  // i fastest
        int t[3];
        t[0] = min(c0 + cl, nc - 1);
        t[F] = wrap_index(s0 - 4 + sl, ns);
        t[OD] = o;
        const long cell = pack(dm, t[0], t[1], t[2]);
#pragma unroll
        for (int q = 0; q < 13; ++q) sv[q][e] = a.m[(long)src[q] * N + cell];
    }
    __syncthreads();
    const int tl = threadIdx.x / FC, cl = threadIdx.x % FC;
    const int sg = s0 + tl, cg = c0 + cl;
    if (sg >= ns || cg >= nc) return;
    int t[3];
    t[0] = cg;
    t[F] = sg;
    t[OD] = o;
    const long idx = pack(dm, t[0], t[1], t[2]);
    int dst[13];
    for (int c = 0; c < 3; ++c) dst[c] = GBR_SLOT_FACE_HAT(F, c);
    dst[3] = GBR_SLOT_FACE_HATT(F);
    for (int e = 0; e < 3; ++e)
        for (int c = 0; c < 3; ++c) dst[4 + e * 3 + c] = GBR_SLOT_FACE_UNHAT(F, e, c);
#pragma unroll
    for (int q = 0; q < 13; ++q) {
        double v[10];
#pragma unroll
        for (int w = 0; w < 10; ++w) v[w] = sv[q][(tl + w) * FC + cl];  // cells sg-4 .. sg+5
        a.m[(long)dst[q] * N + idx] = face_interp(v + 4);
    }
}

// MEG6 interface values of the xi family from LDS tiles: a workgroup owns
// XT interfaces along i for XC lines along j and stages the same 13 source
// slots of cells s0-4 .. s0+XT+4 (i fastest, coalesced rows). Same formula on
// the same values as k_face_metrics.
constexpr int XT = 64, XC = kBlock / XT, XNP = XT + 9;

__global__ void __launch_bounds__(kBlock) k_face_metrics_xi(MetricArgs a)
{
    __shared__ double sv[13][XC * XNP];  // [slot][line][s]
    const Dims &dm = a.dm;
    const long N = dm.ncell;
    const int ns = dm.n[0], nc = dm.n[1];
    const int tiles_s = (ns + XT - 1) / XT;
    const int s0 = (blockIdx.x % tiles_s) * XT;
    const int c0 = (blockIdx.x / tiles_s) * XC;
    const int o = blockIdx.y;
    // cells s0-4 .. s0+XT+4 lie in [0, ns) unless the tile is at a line end
    const bool edge = s0 < 4 || s0 + XT + 5 > ns;
    int src[13];
    for (int c = 0; c < 3; ++c) src[c] = GBR_SLOT_CELL_HAT(0, c);
    src[3] = GBR_SLOT_CELL_HATT(0);
    for (int e = 0; e < 3; ++e)
        for (int c = 0; c < 3; ++c) src[4 + e * 3 + c] = GBR_SLOT_CELL_UNHAT(e, c);
    for (int e = threadIdx.x; e < XNP * XC; e += kBlock) {
        const int sl = e % XNP, cl = e / XNP;
        const int si = s0 - 4 + sl;
        const long cell = pack(dm, edge ? wrap_index(si, ns) : si, min(c0 + cl, nc - 1), o);
#pragma unroll
        for (int q = 0; q < 13; ++q) sv[q][e] = a.m[(long)src[q] * N + cell];
    }
    __syncthreads();
    const int tl = threadIdx.x % XT, cl = threadIdx.x / XT;
    const int sg = s0 + tl, cg = c0 + cl;
    if (sg >= ns || cg >= nc) return;
    const long idx = pack(dm, sg, cg, o);
    int dst[13];
    for (int c = 0; c < 3; ++c) dst[c] = GBR_SLOT_FACE_HAT(0, c);
    dst[3] = GBR_SLOT_FACE_HATT(0);
    for (int e = 0; e < 3; ++e)
        for (int c = 0; c < 3; ++c) dst[4 + e * 3 + c] = GBR_SLOT_FACE_UNHAT(0, e, c);
#pragma unroll
    for (int q = 0; q < 13; ++q) {
        double v[10];
#pragma unroll
        for (int w = 0; w < 10; ++w) v[w] = sv[q][cl * XNP + tl + w];  // cells sg-4 .. sg+5
        a.m[(long)dst[q] * N + idx] = face_interp(v + 4);
    }
}

__global__ void __launch_bounds__(kBlock) k_gcl(MetricArgs a)
{
    long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx >= a.dm.ncell) return;
    const long N = a.dm.ncell;
    int ijk[3];
    unpack(a.dm, idx, ijk);
    double s = 0.0;
    for (int f = 0; f < 3; ++f) {
        const double *ft = a.m + GBR_SLOT_FACE_HATT(f) * N;
        s += ft[idx] - ft[step_to(a.dm, ijk, f, -1, nullptr)];
    }
    a.m[GBR_SLOT_CELL_INVJT * N + idx] = -s;
}

// --- App. D (non-freestream-preserving metrics, negative control) ---------
// Fourth-order central derivative (Eq. 4thorder-grads) at the window centre.
__device__ __forceinline__ double c4(const double *v)
{
    return (2.0 / 3.0) * (v[1] - v[-1]) - (1.0 / 12.0) * (v[2] - v[-2]);
}

// Interface value at +1/2 of v[-3..4]: Eq. interp-formulae with the
// fourth-order derivative in place of E6 (derivatives at cells -1 .. 2, each
// reaching two cells further).
__device__ __forceinline__ double face_c4(const double *v)
{
    double gv[4];
#pragma unroll
    for (int q = -1; q <= 2; ++q) gv[q + 1] = c4(v + q);
    const double h0 = 2.0 * (v[1] - 2.0 * v[0] + v[-1]) - 0.5 * (gv[2] - gv[0]);
    const double h1 = 2.0 * (v[2] - 2.0 * v[1] + v[0]) - 0.5 * (gv[3] - gv[1]);
    return 0.5 * ((v[0] + 0.5 * gv[1] + h0 / 12.0) + (v[1] - 0.5 * gv[2] + h1 / 12.0));
}

__global__ void __launch_bounds__(kBlock) k_coord_deriv_c4(MetricArgs a)
{
    long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx >= a.dm.ncell) return;
    int ijk[3];
    unpack(a.dm, idx, ijk);
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) {
            double v[5];
            for (int q = -2; q <= 2; ++q) {
                int wr;
                long nb = step_to(a.dm, ijk, d, q, &wr);
                v[q + 2] = coord(a, c, nb) + wr * a.off[d][c];
            }
            a.dx[(d * 3 + c) * a.dm.ncell + idx] = c4(v + 2);
        }
}

// hat(d)_c = (c1)_d1 (c2)_d2 - (c1)_d2 (c2)_d1 (App. D, cyclic form), J and
// unhatted metrics; static grid.
__global__ void __launch_bounds__(kBlock) k_cell_metrics_nonfp(MetricArgs a)
{
    long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx >= a.dm.ncell) return;
    const long N = a.dm.ncell;
    double x[3][3];
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) x[d][c] = a.dx[(d * 3 + c) * N + idx];
    const double invj = x[0][0] * (x[1][1] * x[2][2] - x[1][2] * x[2][1]) -
                        x[0][1] * (x[1][0] * x[2][2] - x[1][2] * x[2][0]) +
                        x[0][2] * (x[1][0] * x[2][1] - x[1][1] * x[2][0]);
    if (!(invj > 0.0)) atomicOr(a.flags + 1, 1);
    double *m = a.m;
    m[GBR_SLOT_CELL_INVJ * N + idx] = invj;
    m[GBR_SLOT_CELL_J * N + idx] = 1.0 / invj;
    m[GBR_SLOT_CELL_INVJT * N + idx] = 0.0;
    for (int d = 0; d < 3; ++d) {
        const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        for (int c = 0; c < 3; ++c) {
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            const double hat = x[d1][c1] * x[d2][c2] - x[d2][c1] * x[d1][c2];
            m[GBR_SLOT_CELL_HAT(d, c) * N + idx] = hat;
            m[GBR_SLOT_CELL_UNHAT(d, c) * N + idx] = hat / invj;
        }
        m[GBR_SLOT_CELL_HATT(d) * N + idx] = 0.0;
        m[GBR_SLOT_CELL_UNHATT(d) * N + idx] = 0.0;
    }
}

__global__ void __launch_bounds__(kBlock) k_face_metrics_c4(MetricArgs a)
{
    long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx >= a.dm.ncell) return;
    const long N = a.dm.ncell;
    int ijk[3];
    unpack(a.dm, idx, ijk);
    double *m = a.m;
    for (int f = 0; f < 3; ++f) {
        long nb[8];
        for (int q = -3; q <= 4; ++q) nb[q + 3] = step_to(a.dm, ijk, f, q, nullptr);
        auto interp = [&](int slot) {
            double v[8];
            for (int q = 0; q < 8; ++q) v[q] = m[slot * N + nb[q]];
            return face_c4(v + 3);
        };
        for (int c = 0; c < 3; ++c) m[GBR_SLOT_FACE_HAT(f, c) * N + idx] = interp(GBR_SLOT_CELL_HAT(f, c));
        m[GBR_SLOT_FACE_HATT(f) * N + idx] = 0.0;
        for (int e = 0; e < 3; ++e)
            for (int c = 0; c < 3; ++c)
                m[GBR_SLOT_FACE_UNHAT(f, e, c) * N + idx] = interp(GBR_SLOT_CELL_UNHAT(e, c));
    }
}

// Float copy of the metric slots the FP32-bulk RHS kernels read: the 13
// interface slots of each family and the 9 cell unhatted metrics, which are
// slots 0 .. 47, each rounded to nearest as the kernels would round it on
// load.
static_assert(GBR_SLOT_FACE_UNHAT(2, 2, 2) == 38 && GBR_SLOT_CELL_UNHAT(0, 0) == 39 &&
                  GBR_SLOT_CELL_UNHAT(2, 2) == kFloatMetricSlots - 1,
              "float metric slots are the first 48");

__global__ void __launch_bounds__(kBlock) k_metrics_float(const double *m, float *mf, long n)
{
    const long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx < n) mf[idx] = float(m[idx]);
}

}  // namespace

hipError_t launch_metrics_float(gbr_grid_s *g)
{
    if (!g->metrics_f) return hipSuccess;
    const long N = g->ncell;
    const long n = N * kFloatMetricSlots;
    hipLaunchKernelGGL(k_metrics_float, dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, g->stream,
                       (const double *)g->metrics, g->metrics_f, n);
    return hipGetLastError();
}

hipError_t launch_metrics(gbr_grid_s *g, const double *xyz, const double *xyz_t)
{
    MetricArgs a;
    a.dm = dims_of(g);
    a.ndim = g->cfg.ndim;
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) a.off[d][c] = g->cfg.off[d][c];
    if (a.ndim == 2) {
        a.off[2][0] = 0.0;
        a.off[2][1] = 0.0;
        a.off[2][2] = 1.0;
        for (int d = 0; d < 2; ++d) a.off[d][2] = 0.0;
    }
    a.xyz = xyz;
    a.xyz_t = g->cfg.moving ? xyz_t : nullptr;
    a.dx = g->scratch;
    a.m = g->metrics;
    a.flags = g->flags;
    unsigned blocks = unsigned((a.dm.ncell + kBlock - 1) / kBlock);
    Timed timed(g, GBR_K_METRICS);
    const Ig4MetricStencil &st = ig4_metric_stencil();
    if (g->cfg.scheme == GBR_SCHEME_MIG4) {
        hipLaunchKernelGGL(k_coord_deriv<true>, dim3(blocks), dim3(kBlock), 0, g->stream, a, st);
        hipLaunchKernelGGL(k_cell_metrics<true>, dim3(blocks), dim3(kBlock), 0, g->stream, a, st);
    } else {
        hipLaunchKernelGGL(k_coord_deriv<false>, dim3(blocks), dim3(kBlock), 0, g->stream, a, st);
        hipLaunchKernelGGL(k_cell_metrics<false>, dim3(blocks), dim3(kBlock), 0, g->stream, a, st);
    }
    if (g->cfg.scheme == GBR_SCHEME_MIG4) {
        hipLaunchKernelGGL(k_face_metrics<true>, dim3(blocks), dim3(kBlock), 0, g->stream, a, st, 7);
    } else {
        // every family from LDS tiles (in 2-D the trivial zeta family per cell)
        const int n0 = a.dm.n[0];
        hipLaunchKernelGGL(k_face_metrics_xi,
                           dim3(unsigned(((n0 + XT - 1) / XT) * ((a.dm.n[1] + XC - 1) / XC)), unsigned(a.dm.n[2])),
                           dim3(kBlock), 0, g->stream, a);
        if (a.ndim == 2)
            hipLaunchKernelGGL(k_face_metrics<false>, dim3(blocks), dim3(kBlock), 0, g->stream, a, st, 4);
        hipLaunchKernelGGL(k_face_metrics_tiled<1>,
                           dim3(unsigned(((a.dm.n[1] + FT - 1) / FT) * ((n0 + FC - 1) / FC)), unsigned(a.dm.n[2])),
                           dim3(kBlock), 0, g->stream, a);
        if (a.ndim == 3)
            hipLaunchKernelGGL(k_face_metrics_tiled<2>,
                               dim3(unsigned(((a.dm.n[2] + FT - 1) / FT) * ((n0 + FC - 1) / FC)), unsigned(a.dm.n[1])),
                               dim3(kBlock), 0, g->stream, a);
    }
    hipLaunchKernelGGL(k_gcl, dim3(blocks), dim3(kBlock), 0, g->stream, a);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_metrics_float(g);
}

hipError_t launch_metrics_nonfp(gbr_grid_s *g, const double *xyz)
{
    MetricArgs a;
    a.dm = dims_of(g);
    a.ndim = g->cfg.ndim;
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) a.off[d][c] = g->cfg.off[d][c];
    if (a.ndim == 2) {
        a.off[2][0] = 0.0;
        a.off[2][1] = 0.0;
        a.off[2][2] = 1.0;
        for (int d = 0; d < 2; ++d) a.off[d][2] = 0.0;
    }
    a.xyz = xyz;
    a.xyz_t = nullptr;
    a.dx = g->scratch;
    a.m = g->metrics;
    a.flags = g->flags;
    unsigned blocks = unsigned((a.dm.ncell + kBlock - 1) / kBlock);
    Timed timed(g, GBR_K_METRICS);
    hipLaunchKernelGGL(k_coord_deriv_c4, dim3(blocks), dim3(kBlock), 0, g->stream, a);
    hipLaunchKernelGGL(k_cell_metrics_nonfp, dim3(blocks), dim3(kBlock), 0, g->stream, a);
    hipLaunchKernelGGL(k_face_metrics_c4, dim3(blocks), dim3(kBlock), 0, g->stream, a);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_metrics_float(g);
}

}  // namespace gbr

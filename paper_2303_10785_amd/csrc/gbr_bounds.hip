// Non-periodic boundaries (Sec. 6, App. C).
//
// A bounded direction d stores kNg ghost layers on each side inside every
// field array: interior cells are kNg .. n[d] - kNg - 1. Ghost cells have
// no metrics of their own (Sec. 6): the metrics of interior cells use the
// one-sided closures of App. C along bounded directions, and each ghost slot
// then holds the value of the nearest interior cell (face slots: the nearest
// interface between the two boundary faces), so that every kernel reading a
// ghost slot sees finite data. Ghost primitive states come from the boundary
// type before every RHS; interfaces and gradients of interior cells reach at
// most kNg cells into the ghost layers, so the interior flux formulae are
// unchanged at boundaries, as the paper states.
//
// Kernels:
//   k_coord_deriv_b, k_cell_metrics_b, k_face_metrics_b : the steps of the
//       periodic metric kernels, with App. C rows along bounded directions
//       (interior cells only)
//   k_metric_ghosts : ghost slots <- nearest interior slots
//   k_bc_prims      : ghost primitives of one direction (both sides)
//   k_bc_state      : ghost conserved states of one direction after a step
//   k_theta_ghosts  : ghost sensor values <- nearest interior cell
//   k_sponge        : Res += -sigma (Q - Q_ref) / J in interior cells
#include <cstring>

#include "gbr_device.hpp"
#include "gbr_internal.hpp"

namespace gbr {
namespace {

constexpr int kBlock = 256;
constexpr int kRows = 5;   // modified interfaces at each end (faces 0 .. 4)
constexpr int kTaps = 9;   // cells 0 .. 8 from the boundary that they read

// Interface rows of App. C at the low end: F[f] = sum_k w[f][k] v[k] for
// f = 0 .. kRows - 1. The high end is the mirror image: F[m - f] =
// sum_k w[f][k] v[m - 1 - k].
struct BoundRows {
    double w[kRows][kTaps];
};

// --- host: the App. C line procedure, applied to unit vectors -------------
// First derivatives: second-order one-sided at the boundary cell, the
// fourth-order partially one-sided formula on cells i-1 .. i+3 at the second
// cell, fourth-order central at the third, E6 inside; second derivatives:
// the same two closures applied to the first derivatives at the first two
// cells, the Hermite form of Sec. 5.1 Step-1 from the third cell inwards.
// Interfaces: the boundary face takes the boundary cell's state extrapolated
// to it, the next face the second cell's state alone, the others the
// central average (Eq. FP-interp). The high end mirrors the low end.
void appc_faces(const double *v, int m, double *F)
{
    double p[64], h[64];
    auto os2 = [](const double *x, int s) { return s * (-1.5 * x[0] + 2.0 * x[s] - 0.5 * x[2 * s]); };
    auto pos4 = [](const double *x, int s) {
        return s * (-0.25 * x[-s] - (5.0 / 6.0) * x[0] + 1.5 * x[s] - 0.5 * x[2 * s] + (1.0 / 12.0) * x[3 * s]);
    };
    auto c4 = [](const double *x) { return (2.0 / 3.0) * (x[1] - x[-1]) - (1.0 / 12.0) * (x[2] - x[-2]); };
    auto e6h = [](const double *x) {
        return 0.75 * (x[1] - x[-1]) - 0.15 * (x[2] - x[-2]) + (1.0 / 60.0) * (x[3] - x[-3]);
    };
    p[0] = os2(v, 1);
    p[1] = pos4(v + 1, 1);
    p[2] = c4(v + 2);
    for (int c = 3; c <= m - 4; ++c) p[c] = e6h(v + c);
    p[m - 3] = c4(v + m - 3);
    p[m - 2] = pos4(v + m - 2, -1);
    p[m - 1] = os2(v + m - 1, -1);
    h[0] = os2(p, 1);
    h[1] = pos4(p + 1, 1);
    for (int c = 2; c <= m - 3; ++c) h[c] = 2.0 * (v[c + 1] - 2.0 * v[c] + v[c - 1]) - 0.5 * (p[c + 1] - p[c - 1]);
    h[m - 2] = pos4(p + m - 2, -1);
    h[m - 1] = os2(p + m - 1, -1);
    auto up = [&](int c) { return v[c] + 0.5 * p[c] + h[c] / 12.0; };    // state at c + 1/2
    auto down = [&](int c) { return v[c] - 0.5 * p[c] + h[c] / 12.0; };  // state at c - 1/2
    F[0] = down(0);
    F[1] = down(1);
    for (int f = 2; f <= m - 2; ++f) F[f] = 0.5 * (up(f - 1) + down(f));
    F[m - 1] = up(m - 2);
    F[m] = up(m - 1);
}

const BoundRows &bound_rows()
{
    static const BoundRows rows = [] {
        BoundRows r;
        constexpr int m = 32;  // long enough that the two ends do not interact
        double v[m], F[m + 1];
        for (int k = 0; k < kTaps; ++k) {
            std::memset(v, 0, sizeof v);
            v[k] = 1.0;
            appc_faces(v, m, F);
            for (int f = 0; f < kRows; ++f) r.w[f][k] = F[f];
        }
        return r;
    }();
    return rows;
}

// --- device ----------------------------------------------------------------
struct BArgs {
    Dims dm;
    int ndim;
    int bounded[3];
    double off[3][3];
    const double *xyz;
    double *dx;   // 9 * ncell
    double *m;    // GBR_SLOT_COUNT * ncell
    int *flags;
};

__device__ __forceinline__ void unpack(const Dims &dm, long idx, int ijk[3])
{
    ijk[0] = int(idx % dm.n[0]);
    ijk[1] = int((idx / dm.n[0]) % dm.n[1]);
    ijk[2] = int(idx / ((long)dm.n[0] * dm.n[1]));
}

__device__ __forceinline__ long pack(const Dims &dm, const int t[3])
{
    return t[0] + (long)dm.n[0] * (t[1] + (long)dm.n[1] * t[2]);
}

__device__ __forceinline__ double coord(const BArgs &a, int c, long nb)
{
    if (c == 2 && a.ndim == 2) return 0.0;
    return a.xyz[c * a.dm.ncell + nb];
}

// Interface value F[f], f = 0 .. m, of a bounded line of m interior values
// val(k), k = 0 .. m - 1 (F[f] lies between cells f - 1 and f).
template <class V>
__device__ __forceinline__ double bface(const BoundRows &br, int f, int m, V val)
{
    if (f < kRows) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kTaps; ++k) s += br.w[f][k] * val(k);
        return s;
    }
    if (f > m - kRows) {
        const int r = m - f;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < kTaps; ++k) s += br.w[r][k] * val(m - 1 - k);
        return s;
    }
    double w[10];
#pragma unroll
    for (int q = -4; q <= 5; ++q) w[q + 4] = val(f - 1 + q);
    return face_interp(w + 4);
}

// Composite derivative (Eq. FP-interp2) at cell ijk along d of f(t), where
// f(t) is the value at the cell whose index tuple is t: App. C along a
// bounded direction, the periodic closed form (with the coordinate shift
// per wrap, supplied by f) otherwise.
template <class F>
__device__ __forceinline__ double deriv(const BArgs &a, const BoundRows &br, const int ijk[3], int d, F f)
{
    int t[3] = {ijk[0], ijk[1], ijk[2]};
    if (a.bounded[d]) {
        const int m = a.dm.n[d] - 2 * kNg, pos = ijk[d] - kNg;
        auto val = [&](int k) {
            t[d] = kNg + k;
            return f(t, 0);
        };
        return bface(br, pos + 1, m, val) - bface(br, pos, m, val);
    }
    double v[11];
#pragma unroll
    for (int q = -5; q <= 5; ++q) {
        const int s = ijk[d] + q;
        t[d] = wrap_index(s, a.dm.n[d]);
        v[q + 5] = f(t, wrap_count(s, a.dm.n[d]));
    }
    return dcomp(v + 5);
}

__global__ void __launch_bounds__(kBlock) k_coord_deriv_b(BArgs a, BoundRows br)
{
    const long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx >= a.dm.ncell) return;
    int ijk[3];
    unpack(a.dm, idx, ijk);
    if (!in_box(a.dm, ijk[0], ijk[1], ijk[2])) return;
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) {
            const double org = coord(a, c, idx);
            a.dx[(d * 3 + c) * a.dm.ncell + idx] = deriv(a, br, ijk, d, [&](const int t[3], int wr) {
                return image_rel(coord(a, c, pack(a.dm, t)), wr, a.off[d][c], org);
            });
        }
}

__global__ void __launch_bounds__(kBlock) k_cell_metrics_b(BArgs a, BoundRows br)
{
    const long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx >= a.dm.ncell) return;
    const long N = a.dm.ncell;
    int ijk[3];
    unpack(a.dm, idx, ijk);
    if (!in_box(a.dm, ijk[0], ijk[1], ijk[2])) return;
    double hat[3][3];
    for (int d = 0; d < 3; ++d) {
        const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
        for (int c = 0; c < 3; ++c) {
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            const double org = coord(a, c2, idx);
            const double ta = deriv(a, br, ijk, d2, [&](const int t[3], int wr) {
                const long nb = pack(a.dm, t);
                return a.dx[(d1 * 3 + c1) * N + nb] * image_rel(coord(a, c2, nb), wr, a.off[d2][c2], org);
            });
            const double tb = deriv(a, br, ijk, d1, [&](const int t[3], int wr) {
                const long nb = pack(a.dm, t);
                return a.dx[(d2 * 3 + c1) * N + nb] * image_rel(coord(a, c2, nb), wr, a.off[d1][c2], org);
            });
            hat[d][c] = ta - tb;
        }
    }
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
        for (int c = 0; c < 3; ++c) {
            m[GBR_SLOT_CELL_HAT(d, c) * N + idx] = hat[d][c];
            m[GBR_SLOT_CELL_UNHAT(d, c) * N + idx] = hat[d][c] / invj;
        }
        m[GBR_SLOT_CELL_HATT(d) * N + idx] = 0.0;
        m[GBR_SLOT_CELL_UNHATT(d) * N + idx] = 0.0;
    }
}

// Interface values of family f stored at cell idx (the interface between
// idx and its +1 neighbour along f): interfaces of interior cells only.
__global__ void __launch_bounds__(kBlock) k_face_metrics_b(BArgs a, BoundRows br)
{
    const long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx >= a.dm.ncell) return;
    const long N = a.dm.ncell;
    int ijk[3];
    unpack(a.dm, idx, ijk);
    double *m = a.m;
    for (int f = 0; f < 3; ++f) {
        bool ok = true;
        for (int e = 0; e < 3; ++e)
            if (e != f && (ijk[e] < a.dm.lo[e] || ijk[e] >= a.dm.hi[e])) ok = false;
        const int mm = a.dm.n[f] - 2 * kNg, F = ijk[f] - kNg + 1;
        if (a.bounded[f] && (F < 0 || F > mm)) ok = false;
        if (!ok) continue;
        auto interp = [&](int slot) {
            const double *s = m + (long)slot * N;
            int t[3] = {ijk[0], ijk[1], ijk[2]};
            if (a.bounded[f])
                return bface(br, F, mm, [&](int k) {
                    t[f] = kNg + k;
                    return s[pack(a.dm, t)];
                });
            double w[10];
            for (int q = -4; q <= 5; ++q) {
                t[f] = wrap_index(ijk[f] + q, a.dm.n[f]);
                w[q + 4] = s[pack(a.dm, t)];
            }
            return face_interp(w + 4);
        };
        for (int c = 0; c < 3; ++c) m[GBR_SLOT_FACE_HAT(f, c) * N + idx] = interp(GBR_SLOT_CELL_HAT(f, c));
        m[GBR_SLOT_FACE_HATT(f) * N + idx] = 0.0;
        for (int e = 0; e < 3; ++e)
            for (int c = 0; c < 3; ++c)
                m[GBR_SLOT_FACE_UNHAT(f, e, c) * N + idx] = interp(GBR_SLOT_CELL_UNHAT(e, c));
    }
}

// Nearest valid position: interior cells for cell slots, interfaces
// lo - 1 .. hi - 1 along the family direction for face slots.
__device__ __forceinline__ long clamp_to(const Dims &dm, const int ijk[3], int face_of)
{
    int t[3];
    for (int d = 0; d < 3; ++d) {
        const int lo = (d == face_of && dm.lo[d] > 0) ? dm.lo[d] - 1 : dm.lo[d];
        t[d] = min(max(ijk[d], lo), dm.hi[d] - 1);
    }
    return pack(dm, t);
}

__global__ void __launch_bounds__(kBlock) k_metric_ghosts(Dims dm, double *m)
{
    const long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx >= dm.ncell) return;
    const long N = dm.ncell;
    int ijk[3];
    unpack(dm, idx, ijk);
    const long cc = clamp_to(dm, ijk, -1);
    if (cc != idx)
        for (int s = GBR_SLOT_CELL_UNHAT(0, 0); s < GBR_SLOT_COUNT; ++s) m[s * N + idx] = m[s * N + cc];
    for (int f = 0; f < 3; ++f) {
        const long fc = clamp_to(dm, ijk, f);
        if (fc == idx) continue;
        for (int s = GBR_SLOT_FACE_HAT(f, 0); s < GBR_SLOT_FACE_HAT(f, 0) + 13; ++s) m[s * N + idx] = m[s * N + fc];
    }
}

// The ghost cells of direction d, one thread each: entry e = q + 2 kNg r with
// q < kNg the low side at depth q and q >= kNg the high side at depth
// q - kNg (depth 0 next to the boundary face); r runs over the two other
// directions' full extents.
struct Slab {
    int d, a, b;  // d and the two other directions
    long count;   // 2 kNg * n[a] * n[b]
};

__host__ __device__ inline Slab slab_of(const Dims &dm, int d)
{
    Slab s;
    s.d = d;
    s.a = (d + 1) % 3;
    s.b = (d + 2) % 3;
    s.count = 2L * kNg * dm.n[s.a] * dm.n[s.b];
    return s;
}

// Ghost cell (into t), its side (0 low, 1 high) and depth (0 next to the
// boundary face) for slab entry e.
__device__ __forceinline__ void slab_cell(const Dims &dm, const Slab &s, long e, int t[3], int *side, int *depth)
{
    const int q = int(e % (2 * kNg));
    const long r = e / (2 * kNg);
    t[s.a] = int(r % dm.n[s.a]);
    t[s.b] = int(r / dm.n[s.a]);
    *side = q >= kNg;
    *depth = q % kNg;
    t[s.d] = *side ? dm.n[s.d] - kNg + *depth : kNg - 1 - *depth;
}

// Unit normal of the boundary face on the ghost's line.
__device__ __forceinline__ void wall_normal(const Dims &dm, const double *m, int d, const int t[3], int side,
                                            double nr[3])
{
    int f[3] = {t[0], t[1], t[2]};
    f[d] = side ? dm.n[d] - kNg - 1 : kNg - 1;
    const long fc = pack(dm, f);
    double nn = 0.0;
    for (int c = 0; c < 3; ++c) {
        nr[c] = m[GBR_SLOT_FACE_HAT(d, c) * dm.ncell + fc];
        nn += nr[c] * nr[c];
    }
    nn = sqrt(nn);
    for (int c = 0; c < 3; ++c) nr[c] /= nn;
}

struct BcTypes {
    int t[2];  // GBR_BC_* of the low and high side
};

// Ghost primitives (rho, u, v, w, p, T) of direction d.
template <int NDIM, class R>
__global__ void __launch_bounds__(kBlock) k_bc_prims(Dims dm, Slab s, BcTypes bt, R *prim, const double *Q,
                                                      const double *m, double gm1, double gM2)
{
    const long e = blockIdx.x * (long)kBlock + threadIdx.x;
    if (e >= s.count) return;
    const long N = dm.ncell;
    int t[3], side, depth;
    slab_cell(dm, s, e, t, &side, &depth);
    const long gc = pack(dm, t);
    const int type = bt.t[side];
    if (type == GBR_BC_INFLOW) {
        // the caller's state in the ghost cell, as the primitives kernel forms it
        const double r = Q[gc];
        const double ir = 1.0 / r;
        const double u = Q[N + gc] * ir;
        const double v = Q[2 * N + gc] * ir;
        const double w = (NDIM == 3) ? Q[3 * N + gc] * ir : 0.0;
        const double E = Q[(NDIM + 1) * N + gc];
        const double p = gm1 * (E - 0.5 * r * (u * u + v * v + w * w));
        prim[gc] = R(r);
        prim[N + gc] = R(u);
        prim[2 * N + gc] = R(v);
        prim[3 * N + gc] = R(w);
        prim[4 * N + gc] = R(p);
        prim[5 * N + gc] = R(gM2 * p * ir);
        return;
    }
    int src[3] = {t[0], t[1], t[2]};
    if (type == GBR_BC_OUTFLOW)
        src[s.d] = side ? dm.n[s.d] - kNg - 1 : kNg;
    else
        src[s.d] = side ? dm.n[s.d] - kNg - 1 - depth : kNg + depth;
    const long sc = pack(dm, src);
    R pv[6];
#pragma unroll
    for (int v = 0; v < 6; ++v) pv[v] = prim[v * N + sc];
    if (type == GBR_BC_WALL) {
        double nr[3];
        wall_normal(dm, m, s.d, t, side, nr);
        if (NDIM == 2) nr[2] = 0.0;
        const double un = double(pv[1]) * nr[0] + double(pv[2]) * nr[1] + double(pv[3]) * nr[2];
        for (int c = 0; c < NDIM; ++c) pv[1 + c] = R(double(pv[1 + c]) - 2.0 * un * nr[c]);
    }
#pragma unroll
    for (int v = 0; v < 6; ++v) prim[v * N + gc] = pv[v];
}

// Ghost conserved states of direction d at the end of a step (outflow and
// wall sides; inflow ghosts keep the caller's state).
template <int NV>
__global__ void __launch_bounds__(kBlock) k_bc_state(Dims dm, Slab s, BcTypes bt, double *Q, const double *m)
{
    const long e = blockIdx.x * (long)kBlock + threadIdx.x;
    if (e >= s.count) return;
    const long N = dm.ncell;
    int t[3], side, depth;
    slab_cell(dm, s, e, t, &side, &depth);
    const int type = bt.t[side];
    if (type == GBR_BC_INFLOW) return;
    const long gc = pack(dm, t);
    int src[3] = {t[0], t[1], t[2]};
    if (type == GBR_BC_OUTFLOW)
        src[s.d] = side ? dm.n[s.d] - kNg - 1 : kNg;
    else
        src[s.d] = side ? dm.n[s.d] - kNg - 1 - depth : kNg + depth;
    const long sc = pack(dm, src);
    double q[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = Q[v * N + sc];
    if (type == GBR_BC_WALL) {
        constexpr int nd = NV - 2;
        double nr[3];
        wall_normal(dm, m, s.d, t, side, nr);
        double mn = 0.0;
        for (int c = 0; c < nd; ++c) mn += q[1 + c] * nr[c];
        for (int c = 0; c < nd; ++c) q[1 + c] -= 2.0 * mn * nr[c];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) Q[v * N + gc] = q[v];
}

// Ghost sensor flags of the slab of one bounded direction: the flag of the
// nearest interior cell (clamped along every bounded direction, so a
// corner ghost visited by two slabs gets the same value from both).
__global__ void __launch_bounds__(kBlock) k_flag_ghosts(Dims dm, Slab s, unsigned char *flag)
{
    const long e = blockIdx.x * (long)kBlock + threadIdx.x;
    if (e >= s.count) return;
    int t[3], side, depth;
    slab_cell(dm, s, e, t, &side, &depth);
    flag[pack(dm, t)] = flag[clamp_to(dm, t, -1)];
}

struct QRef {
    double q[5];
};

template <int NV, class R>
__global__ void __launch_bounds__(kBlock) k_sponge(Dims dm, const double *Q, R *res, const double *sigma,
                                                    const double *invj, QRef qr)
{
    const long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx >= dm.ncell || !in_box(dm, idx)) return;
    const long N = dm.ncell;
    const double sg = sigma[idx], vj = invj[idx];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int src = (NV == 4 && v == 3) ? 4 : v;
        const long e = v * N + idx;
        res[e] = R(double(res[e]) - sg * (Q[e] - qr.q[src]) * vj);
    }
}

}  // namespace

hipError_t launch_metrics_bounded(gbr_grid_s *g, const double *xyz)
{
    BArgs a;
    a.dm = dims_of(g);
    a.ndim = g->cfg.ndim;
    for (int d = 0; d < 3; ++d) {
        a.bounded[d] = g->cfg.bc[d][0] != GBR_BC_PERIODIC;
        for (int c = 0; c < 3; ++c) a.off[d][c] = g->cfg.off[d][c];
    }
    if (a.ndim == 2) {
        a.off[2][0] = 0.0;
        a.off[2][1] = 0.0;
        a.off[2][2] = 1.0;
        for (int d = 0; d < 2; ++d) a.off[d][2] = 0.0;
    }
    a.xyz = xyz;
    a.dx = g->scratch;
    a.m = g->metrics;
    a.flags = g->flags;
    const BoundRows &br = bound_rows();
    const unsigned blocks = unsigned((a.dm.ncell + kBlock - 1) / kBlock);
    Timed timed(g, GBR_K_METRICS);
    hipLaunchKernelGGL(k_coord_deriv_b, dim3(blocks), dim3(kBlock), 0, g->stream, a, br);
    hipLaunchKernelGGL(k_cell_metrics_b, dim3(blocks), dim3(kBlock), 0, g->stream, a, br);
    hipLaunchKernelGGL(k_face_metrics_b, dim3(blocks), dim3(kBlock), 0, g->stream, a, br);
    hipLaunchKernelGGL(k_metric_ghosts, dim3(blocks), dim3(kBlock), 0, g->stream, a.dm, a.m);
    hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_metrics_float(g);
}

template <class R>
hipError_t launch_bc_prims(gbr_grid_s *g, R *prim, const double *Q)
{
    const Dims dm = dims_of(g);
    const Phys ph = phys_of(g);
    Timed timed(g, GBR_K_PRIMS);
    for (int d = 0; d < g->cfg.ndim; ++d) {
        if (g->cfg.bc[d][0] == GBR_BC_PERIODIC) continue;
        const Slab s = slab_of(dm, d);
        const BcTypes bt{{g->cfg.bc[d][0], g->cfg.bc[d][1]}};
        const unsigned blocks = unsigned((s.count + kBlock - 1) / kBlock);
        if (g->cfg.ndim == 3)
            hipLaunchKernelGGL((k_bc_prims<3, R>), dim3(blocks), dim3(kBlock), 0, g->stream, dm, s, bt, prim, Q,
                               g->metrics, ph.gm1, ph.gM2);
        else
            hipLaunchKernelGGL((k_bc_prims<2, R>), dim3(blocks), dim3(kBlock), 0, g->stream, dm, s, bt, prim, Q,
                               g->metrics, ph.gm1, ph.gM2);
    }
    return hipGetLastError();
}

hipError_t launch_bc_state(gbr_grid_s *g, double *Q)
{
    const Dims dm = dims_of(g);
    Timed timed(g, GBR_K_COPY);
    for (int d = 0; d < g->cfg.ndim; ++d) {
        if (g->cfg.bc[d][0] == GBR_BC_PERIODIC) continue;
        const Slab s = slab_of(dm, d);
        const BcTypes bt{{g->cfg.bc[d][0], g->cfg.bc[d][1]}};
        const unsigned blocks = unsigned((s.count + kBlock - 1) / kBlock);
        if (g->nvar == 5)
            hipLaunchKernelGGL(k_bc_state<5>, dim3(blocks), dim3(kBlock), 0, g->stream, dm, s, bt, Q, g->metrics);
        else
            hipLaunchKernelGGL(k_bc_state<4>, dim3(blocks), dim3(kBlock), 0, g->stream, dm, s, bt, Q, g->metrics);
    }
    return hipGetLastError();
}

hipError_t launch_flag_ghosts(gbr_grid_s *g, unsigned char *flag)
{
    const Dims dm = dims_of(g);
    Timed timed(g, GBR_K_CELL_GRAD);
    for (int d = 0; d < g->cfg.ndim; ++d) {
        if (g->cfg.bc[d][0] == GBR_BC_PERIODIC) continue;
        const Slab s = slab_of(dm, d);
        const unsigned blocks = unsigned((s.count + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_flag_ghosts, dim3(blocks), dim3(kBlock), 0, g->stream, dm, s, flag);
    }
    return hipGetLastError();
}

template <class R>
hipError_t launch_sponge(gbr_grid_s *g, const double *Q, R *res)
{
    const Dims dm = dims_of(g);
    const unsigned blocks = unsigned((dm.ncell + kBlock - 1) / kBlock);
    QRef qr;
    for (int v = 0; v < 5; ++v) qr.q[v] = g->qref[v];
    const double *invj = g->metrics + (long)GBR_SLOT_CELL_INVJ * g->ncell;
    Timed timed(g, GBR_K_RK_STAGE);
    if (g->nvar == 5)
        hipLaunchKernelGGL((k_sponge<5, R>), dim3(blocks), dim3(kBlock), 0, g->stream, dm, Q, res, g->sigma, invj, qr);
    else
        hipLaunchKernelGGL((k_sponge<4, R>), dim3(blocks), dim3(kBlock), 0, g->stream, dm, Q, res, g->sigma, invj, qr);
    return hipGetLastError();
}

template hipError_t launch_bc_prims<double>(gbr_grid_s *, double *, const double *);
template hipError_t launch_bc_prims<float>(gbr_grid_s *, float *, const double *);
template hipError_t launch_sponge<double>(gbr_grid_s *, const double *, double *);
template hipError_t launch_sponge<float>(gbr_grid_s *, const double *, float *);

}  // namespace gbr

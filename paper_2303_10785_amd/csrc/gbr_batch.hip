// Batched SSP-RK3 stepping of many 2-D Euler grids (gbr_batch_* in gbr.h).
//
// One step of every grid in the batch is five launches, each covering all
// grids at once through a work list of (grid, tile) items:
//   k_batch_reset : per grid, the time-step reduction word <- +inf
//   k_batch_cfl   : per tile, the App. B bound of every cell, block minimum,
//                   one atomic minimum per tile into the grid's word (the
//                   minimum is exact, so the result does not depend on order)
//   k_batch_stage : one launch per RK stage. Per tile of TX x TY cells:
//                   primitives of the xi and eta pencils (6-cell halo) and
//                   their E6 derivatives in LDS, every xi and eta interface of
//                   the tile (Sec. 5.1 Steps 1-6: limited or direct states,
//                   HLLC), the flux differences (Step-7) and the SSP-RK3
//                   update (App. B) of the tile's own cells. The stage reads
//                   one state buffer and writes another (Q -> S1 -> S2 -> Q),
//                   so no tile waits for another within a launch.
//   k_batch_finish: per grid, dt and the accumulated time.
// The stage and time-step kernels are persistent: a launch of 8 * k
// workgroups walks the work list, which is cut into eight contiguous chunks,
// one per XCD (workgroups are dispatched to the XCDs round-robin), so the
// halo re-reads of neighbouring tiles of a grid hit the same L2.
#include <algorithm>
#include <cstdio>
#include <new>
#include <vector>

#include "gbr_device.hpp"
#include "gbr_internal.hpp"

namespace gbr {
namespace {

constexpr int kBlock = 256;
constexpr int kXcd = 8;

struct BatchGrid {
    int ni, nj;
    long N;
    const double *m;  // metrics (GBR_SLOT_*)
    double *Q;        // caller state: stage-0 input, RK base state, stage-2 output
    double *S1, *S2;  // stage buffers (the grid's Qn and Res storage)
    int *flags;
};

struct BatchArgs {
    const BatchGrid *grids;
    const int2 *items;  // (grid, tile within the grid)
    int nitems;
    int per;            // items per XCD chunk
    int ngrid;
    double gamma, gm1, alpha_mp, beta_mp;
    unsigned long long *dtmin;  // per grid: bit pattern of the minimum bound
    double *dt, *t;             // per grid
    double cfl_or_dt;
    int dt_mode;
};

// Walk this workgroup's share of the work list.
template <class F>
__device__ __forceinline__ void for_items(const BatchArgs &a, F &&f)
{
    const int x = blockIdx.x % kXcd, lb = blockIdx.x / kXcd, gx = gridDim.x / kXcd;
    const int lo = x * a.per;
    const int hi = min(lo + a.per, a.nitems);
    for (int k = lo + lb; k < hi; k += gx) f(a.items[k]);
}

__device__ __forceinline__ double step_of(const BatchArgs &a, int gi)
{
    return a.dt_mode == GBR_DT_CFL ? a.cfl_or_dt * __longlong_as_double((long long)a.dtmin[gi]) : a.cfl_or_dt;
}

__global__ void __launch_bounds__(kBlock) k_batch_reset(BatchArgs a)
{
    const int gi = blockIdx.x * kBlock + threadIdx.x;
    if (gi < a.ngrid) a.dtmin[gi] = 0x7ff0000000000000ull;  // +inf
}

__global__ void __launch_bounds__(kBlock) k_batch_finish(BatchArgs a)
{
    const int gi = blockIdx.x * kBlock + threadIdx.x;
    if (gi >= a.ngrid) return;
    const double dt = step_of(a, gi);
    a.dt[gi] = dt;
    a.t[gi] += dt;
}

template <int TX, int TY>
__global__ void __launch_bounds__(kBlock) k_batch_cfl(BatchArgs a)
{
    static_assert(TX * TY == kBlock, "one cell per thread");
    __shared__ double wmin[kBlock / 64];
    for_items(a, [&](int2 it) {
        const BatchGrid &G = a.grids[it.x];
        const int tiles_i = (G.ni + TX - 1) / TX;
        const int i = (it.y % tiles_i) * TX + threadIdx.x % TX;
        const int j = (it.y / tiles_i) * TY + threadIdx.x / TX;
        double best = __builtin_inf();
        if (i < G.ni && j < G.nj)
            best = cell_dt_bound<2, false>(G.Q, G.m, G.N, i + (long)G.ni * j, a.gamma, a.gm1, 0.0, 0.0, 1.0,
                                           1.0, false);  // batched grids are static
        for (int off = warpSize / 2; off > 0; off >>= 1) best = fmin(best, __shfl_xor(best, off));
        if (threadIdx.x % warpSize == 0) wmin[threadIdx.x / warpSize] = best;
        __syncthreads();
        if (threadIdx.x == 0) {
            double b = wmin[0];
            for (int q = 1; q < kBlock / warpSize; ++q) b = fmin(b, wmin[q]);
            // positive doubles (and +inf) order like their bit patterns; a NaN
            // bound is larger than +inf and never wins, as with fmin
            atomicMin(a.dtmin + it.x, (unsigned long long)__double_as_longlong(b));
        }
        __syncthreads();
    });
}

// Interface states and HLLC flux of one interface whose left cell sits at
// P (primitives) and G (first derivatives) in LDS, with stride st between
// cells along the interface normal; returns false for a non-physical state.
template <bool LIM, class R>
__device__ __forceinline__ bool face_flux_2d(const R *P, const R *G, int st, int vsP, int vsG, R nx, R ny,
                                             R gamma, R igm1, R alpha_mp, R beta_mp, R phi[5])
{
    R PL[5], PR[5];
    if (LIM) {
        // FP64: one characteristic field at a time, its curvatures formed
        // from its values and first derivatives (252 -> 168 VGPRs with the
        // 16 x 16 tile, a third wave per SIMD); FP32 keeps all fields
        // together, which its registers allow
        if constexpr (sizeof(R) == 8)
            limited_states_pre<4, true, false>(P, G, P, st, vsP, vsG, 0, nx, ny, R(0), gamma, alpha_mp, beta_mp, PL,
                                               PR);
        else
            limited_states<4>(P, G, st, vsP, vsG, nx, ny, R(0), gamma, alpha_mp, beta_mp, PL, PR);
    } else
        direct_states<4>(P, G, st, vsP, vsG, PL, PR);
    PL[3] = R(0);
    PR[3] = R(0);
    hllc(PL, PR, R(0), nx, ny, R(0), gamma, igm1, phi);
    return PL[0] > R(0) && PL[4] > R(0) && PR[0] > R(0) && PR[4] > R(0) && isfinite(phi[0]) &&
           isfinite(phi[4]);
}

// FP64 16 x 16 tiles: at least three workgroups per CU (168 VGPRs with an
// 8-byte spill); the FP64 32 x 8 and 8 x 32 tiles are held at two by their
// LDS either way
template <int TX, int TY, bool LIM, class R>
__global__ void __launch_bounds__(kBlock, (sizeof(R) == 8 && TX == TY) ? 3 : 1)
    k_batch_stage(BatchArgs a, int stage, double ca, double cb)
{
    static_assert(TX * TY == kBlock, "one cell per thread");
    constexpr int PXS = TX + 12, PYS = TY + 12;  // pencil lengths (6-cell halo)
    constexpr int GXS = TX + 6, GYS = TY + 6;    // first-derivative lengths
    constexpr int VPX = TY * PXS, VPY = PYS * TX, VGX = TY * GXS, VGY = GYS * TX;
    constexpr int FX = TY * (TX + 1), FY = (TY + 1) * TX, NF = FX + FY;
    constexpr int NFT = (NF + kBlock - 1) / kBlock;  // faces per thread
    static_assert(4 * (FX + FY) <= 4 * (VPX + VPY), "fluxes alias the pencils");
    __shared__ R sP[4 * (VPX + VPY)];  // xi pencils [v][y][x], then eta pencils [v][y][x]
    __shared__ R sG[4 * (VGX + VGY)];
    // periodic indices of the cells i0-6 .. i0+TX+5 and j0-6 .. j0+TY+5, formed
    // once per tile (one modulo each) for every phase of the tile
    __shared__ int s_wi[TX + 12], s_wj[TY + 12];
    R *Px = sP, *Py = sP + 4 * VPX;
    R *Gx = sG, *Gy = sG + 4 * VGX;
    R *Fx = sP, *Fy = sP + 4 * FX;  // fluxes, after the pencils are consumed

    const R gamma = R(a.gamma), igm1 = R(1.0 / a.gm1), amp = R(a.alpha_mp), bmp = R(a.beta_mp);
    const int tid = threadIdx.x;

    for_items(a, [&](int2 it) {
        const BatchGrid &G = a.grids[it.x];
        const int ni = G.ni, nj = G.nj;
        const long N = G.N;
        const int tiles_i = (ni + TX - 1) / TX;
        const int i0 = (it.y % tiles_i) * TX, j0 = (it.y / tiles_i) * TY;
        const double *in = stage == 0 ? G.Q : (stage == 1 ? G.S1 : G.S2);
        double *out = stage == 0 ? G.S1 : (stage == 1 ? G.S2 : G.Q);

        for (int q = tid; q < TX + 12; q += kBlock) s_wi[q] = wrap_index(i0 - 6 + q, ni);
        for (int q = tid; q < TY + 12; q += kBlock) s_wj[q] = wrap_index(j0 - 6 + q, nj);
        __syncthreads();
        auto wi = [&](int i) { return s_wi[i - i0 + 6]; };  // i0-6 <= i < i0+TX+6
        auto wj = [&](int j) { return s_wj[j - j0 + 6]; };
        auto prim = [&](long c, R *dst, int vs) {
            double r = in[c];
            double ir = 1.0 / r;  // as the single-grid primitives kernel
            double u = in[N + c] * ir;
            double v = in[2 * N + c] * ir;
            double w = 0.0;
            double p = a.gm1 * (in[3 * N + c] - 0.5 * r * (u * u + v * v + w * w));
            dst[0] = R(r);
            dst[vs] = R(u);
            dst[2 * vs] = R(v);
            dst[3 * vs] = R(p);
        };
        // Phase 1: primitives of the xi pencils (rows j0.., cells i0-6 ..
        // i0+TX+5) and the eta pencils (columns i0.., cells j0-6 .. j0+TY+5)
        for (int e = tid; e < VPX; e += kBlock) {
            const int x = e % PXS, y = e / PXS;
            prim(wi(i0 - 6 + x) + (long)ni * wj(j0 + y), Px + e, VPX);
        }
        for (int e = tid; e < VPY; e += kBlock) {
            const int x = e % TX, y = e / TX;
            prim(wi(i0 + x) + (long)ni * wj(j0 - 6 + y), Py + e, VPY);
        }
        __syncthreads();
        // Phase 2: E6 first derivatives of cells i0-3 .. i0+TX+2 (xi) and
        // j0-3 .. j0+TY+2 (eta)
        for (int e = tid; e < VGX; e += kBlock) {
            const int x = e % GXS, y = e / GXS;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const R *p = Px + v * VPX + y * PXS + x + 3;
                Gx[v * VGX + e] = e6(p[-3], p[-2], p[-1], p[1], p[2], p[3]);
            }
        }
        for (int e = tid; e < VGY; e += kBlock) {
            const int x = e % TX, y = e / TX;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const R *p = Py + v * VPY + (y + 3) * TX + x;
                Gy[v * VGY + e] = e6(p[-3 * TX], p[-2 * TX], p[-TX], p[TX], p[2 * TX], p[3 * TX]);
            }
        }
        __syncthreads();
        // Phase 3: every interface of the tile. Face f < FX is the xi face
        // left of cell (i0 + fi, j0 + fj), fi = 0..TX; the others are eta
        // faces below cell (i0 + fi, j0 + fj), fj = 0..TY.
        R phi[NFT][4];
        bool ok = true;
#pragma unroll
        for (int q = 0; q < NFT; ++q) {
            const int f = tid + q * kBlock;
            if (f >= NF) break;
            const bool xi = f < FX;
            const int fi = xi ? f % (TX + 1) : (f - FX) % TX;
            const int fj = xi ? f / (TX + 1) : (f - FX) / TX;
            // left cell of the face and its position in the pencils
            const int ia = xi ? wi(i0 + fi - 1) : wi(i0 + fi);
            const int ja = xi ? wj(j0 + fj) : wj(j0 + fj - 1);
            const long ca = ia + (long)ni * ja;
            const R *P = xi ? Px + fj * PXS + fi + 5 : Py + (fj + 5) * TX + fi;
            const R *Gd = xi ? Gx + fj * GXS + fi + 2 : Gy + (fj + 2) * TX + fi;
            const int st = xi ? 1 : TX;
            const int vsP = xi ? VPX : VPY, vsG = xi ? VGX : VGY;
            const int fam = xi ? 0 : 1;
            const R nx = R(G.m[GBR_SLOT_FACE_HAT(fam, 0) * N + ca]);
            const R ny = R(G.m[GBR_SLOT_FACE_HAT(fam, 1) * N + ca]);
            R ph[5];
            const bool good = face_flux_2d<LIM>(P, Gd, st, vsP, vsG, nx, ny, gamma, igm1, amp, bmp, ph);
            // only interfaces of cells inside the grid count
            const bool real = xi ? (j0 + fj < nj && i0 + fi - 1 < ni) : (i0 + fi < ni && j0 + fj - 1 < nj);
            ok = ok && (good || !real);
            phi[q][0] = ph[0];
            phi[q][1] = ph[1];
            phi[q][2] = ph[2];
            phi[q][3] = ph[4];
        }
        if (!ok) atomicOr(G.flags, 1);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NFT; ++q) {
            const int f = tid + q * kBlock;
            if (f >= NF) break;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (f < FX)
                    Fx[v * FX + f] = phi[q][v];
                else
                    Fy[v * FY + (f - FX)] = phi[q][v];
            }
        }
        __syncthreads();
        // Phase 4: Res = -(xi difference) - (eta difference), then the RK
        // stage of the tile's own cells in double
        const int ti = tid % TX, tj = tid / TX;
        const int i = i0 + ti, j = j0 + tj;
        if (i < ni && j < nj) {
            const long c = i + (long)ni * j;
            const double dt = step_of(a, it.x);
            const double J = G.m[GBR_SLOT_CELL_J * N + c];
            double q[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) q[v] = in[v * N + c];
            {
                double r = q[0], ir = 1.0 / r, u = q[1] * ir, v = q[2] * ir;
                double p = a.gm1 * (q[3] - 0.5 * r * (u * u + v * v));
                if (!(r > 0.0 && p > 0.0 && isfinite(r) && isfinite(p) && isfinite(u) && isfinite(v)))
                    atomicOr(G.flags, 1);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                R res = -(Fx[v * FX + tj * (TX + 1) + ti + 1] - Fx[v * FX + tj * (TX + 1) + ti]);
                res = res - (Fy[v * FY + (tj + 1) * TX + ti] - Fy[v * FY + tj * TX + ti]);
                const double L = J * double(res);
                out[v * N + c] = ca * G.Q[v * N + c] + cb * (q[v] + dt * L);
            }
        }
        __syncthreads();
    });
}

// Tile shapes (GBR_TILE_*).
constexpr int kTiles[3][2] = {{16, 16}, {32, 8}, {8, 32}};

}  // namespace
}  // namespace gbr

struct gbr_batch_s {
    std::vector<gbr_grid_s *> grids;
    hipStream_t stream = nullptr;    // the batch's own stream (capturable)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    int tile = 0;
    int precision = GBR_FP64;
    bool limited = false;
    int blocks = 8;
    gbr::BatchGrid *d_grids = nullptr;
    int2 *d_items = nullptr;
    int nitems = 0;
    unsigned long long *d_dtmin = nullptr;
    double *d_dt = nullptr, *d_t = nullptr;
    gbr::Phys ph{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double g_cfl = 0.0;
    int g_mode = -1;
};

namespace gbr {
namespace {

template <int TX, int TY, class R>
void stage_kernel(bool lim, void (**k)(BatchArgs, int, double, double))
{
    *k = lim ? k_batch_stage<TX, TY, true, R> : k_batch_stage<TX, TY, false, R>;
}

using StageFn = void (*)(BatchArgs, int, double, double);
using CflFn = void (*)(BatchArgs);

StageFn stage_fn(int tile, int precision, bool lim)
{
    StageFn k = nullptr;
    const bool f32 = precision == GBR_FP32_BULK;
    switch (tile) {
    case 0: f32 ? stage_kernel<16, 16, float>(lim, &k) : stage_kernel<16, 16, double>(lim, &k); break;
    case 1: f32 ? stage_kernel<32, 8, float>(lim, &k) : stage_kernel<32, 8, double>(lim, &k); break;
    default: f32 ? stage_kernel<8, 32, float>(lim, &k) : stage_kernel<8, 32, double>(lim, &k); break;
    }
    return k;
}

CflFn cfl_fn(int tile)
{
    switch (tile) {
    case 0: return k_batch_cfl<16, 16>;
    case 1: return k_batch_cfl<32, 8>;
    default: return k_batch_cfl<8, 32>;
    }
}

// Work list for a tile shape: grids in order of decreasing size, each
// grid's tiles contiguous.
std::vector<int2> make_items(const gbr_batch_s *b, int tile)
{
    const int TX = kTiles[tile][0], TY = kTiles[tile][1];
    std::vector<int> order(b->grids.size());
    for (size_t q = 0; q < order.size(); ++q) order[q] = int(q);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return b->grids[x]->ncell > b->grids[y]->ncell; });
    std::vector<int2> items;
    for (int gi : order) {
        const gbr_grid_s *g = b->grids[gi];
        const int ti = (g->cfg.n[0] + TX - 1) / TX, tj = (g->cfg.n[1] + TY - 1) / TY;
        for (int t = 0; t < ti * tj; ++t) items.push_back(make_int2(gi, t));
    }
    return items;
}

BatchArgs args_of(const gbr_batch_s *b, double cfl_or_dt, int dt_mode)
{
    BatchArgs a;
    a.grids = b->d_grids;
    a.items = b->d_items;
    a.nitems = b->nitems;
    a.per = (b->nitems + kXcd - 1) / kXcd;
    a.ngrid = int(b->grids.size());
    a.gamma = b->ph.gamma;
    a.gm1 = b->ph.gm1;
    a.alpha_mp = b->ph.alpha_mp;
    a.beta_mp = b->ph.beta_mp;
    a.dtmin = b->d_dtmin;
    a.dt = b->d_dt;
    a.t = b->d_t;
    a.cfl_or_dt = cfl_or_dt;
    a.dt_mode = dt_mode;
    return a;
}

// Persistent launch size: a multiple of 8 workgroups, at most what the
// device keeps resident at once and at most one per work item.
int persistent_blocks(int nitems, const void *kernel)
{
    int dev = 0, cus = 0, occ = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, kBlock, 0) != hipSuccess || occ < 1) occ = 1;
    const int per = (nitems + kXcd - 1) / kXcd;
    const int resident = std::max(kXcd, (cus * occ) / kXcd * kXcd);
    return std::max(kXcd, std::min(resident, per * kXcd));
}

hipError_t enqueue_step(gbr_batch_s *b, double cfl_or_dt, int dt_mode)
{
    static const double A[3] = {0.0, 0.75, 1.0 / 3.0};
    static const double B[3] = {1.0, 0.25, 2.0 / 3.0};
    const BatchArgs a = args_of(b, cfl_or_dt, dt_mode);
    const unsigned gblocks = unsigned((a.ngrid + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_batch_reset, dim3(gblocks), dim3(kBlock), 0, b->stream, a);
    if (dt_mode == GBR_DT_CFL)
        hipLaunchKernelGGL(cfl_fn(b->tile), dim3(unsigned(b->blocks)), dim3(kBlock), 0, b->stream, a);
    StageFn k = stage_fn(b->tile, b->precision, b->limited);
    for (int s = 0; s < 3; ++s)
        hipLaunchKernelGGL(k, dim3(unsigned(b->blocks)), dim3(kBlock), 0, b->stream, a, s, A[s], B[s]);
    hipLaunchKernelGGL(k_batch_finish, dim3(gblocks), dim3(kBlock), 0, b->stream, a);
    return hipGetLastError();
}

hipError_t upload_items(gbr_batch_s *b, int tile)
{
    std::vector<int2> items = make_items(b, tile);
    if (b->d_items) (void)hipFree(b->d_items);
    b->d_items = nullptr;
    hipError_t e = hipMalloc((void **)&b->d_items, items.size() * sizeof(int2));
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    b->nitems = int(items.size());
    b->tile = tile;
    b->blocks = persistent_blocks(b->nitems, (const void *)stage_fn(tile, b->precision, b->limited));
    return e;
}

// Time one stage-0 launch of each tile shape on the batch (it writes only
// the S1 stage buffers) and keep the fastest.
hipError_t autotune(gbr_batch_s *b)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = 1e30f;
    int best_tile = 0;
    for (int t = 0; t < 3 && e == hipSuccess; ++t) {
        e = upload_items(b, t);
        if (e != hipSuccess) break;
        const BatchArgs a = args_of(b, 0.1, GBR_DT_CFL);
        const unsigned gblocks = unsigned((a.ngrid + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_batch_reset, dim3(gblocks), dim3(kBlock), 0, b->stream, a);
        hipLaunchKernelGGL(cfl_fn(t), dim3(unsigned(b->blocks)), dim3(kBlock), 0, b->stream, a);
        StageFn k = stage_fn(t, b->precision, b->limited);
        float ms = 1e30f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            e = hipEventRecord(e0, b->stream);
            hipLaunchKernelGGL(k, dim3(unsigned(b->blocks)), dim3(kBlock), 0, b->stream, a, 0, 0.0, 1.0);
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float x = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&x, e0, e1);
            if (rep > 0) ms = std::min(ms, x);  // first launch warms the caches
        }
        if (e == hipSuccess && ms < best) {
            best = ms;
            best_tile = t;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e == hipSuccess) e = upload_items(b, best_tile);
    return e;
}

void release_batch(gbr_batch_s *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void *p : {(void *)b->d_grids, (void *)b->d_items, (void *)b->d_dtmin, (void *)b->d_dt, (void *)b->d_t})
        if (p) (void)hipFree(p);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

__global__ void k_zero(double *p, int n)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e < n) p[e] = 0.0;
}

}  // namespace
}  // namespace gbr

extern "C" {

gbr_status gbr_batch_create(const gbr_grid *g, int n, double *const *Q, int tile, gbr_batch *out)
{
    using namespace gbr;
    if (!out) return GBR_E_ARG;
    *out = nullptr;
    if (n < 1 || !g || !Q) return GBR_E_ARG;
    for (int b = 0; b < n; ++b)
        if (!g[b]) return GBR_E_ARG;
    gbr_grid_s *g0 = g[0];
    if (tile < GBR_TILE_AUTO || tile >= GBR_TILE_COUNT) return g0->err = "unknown tile shape", GBR_E_ARG;
    for (int b = 0; b < n; ++b) {
        const gbr_config &c = g[b]->cfg;
        if (!Q[b]) return g0->err = "null state", GBR_E_ARG;
        if (c.ndim != 2 || c.viscous || c.moving || c.scheme != GBR_SCHEME_MEG6 || g[b]->bounded || g[b]->sigma ||
            (c.limiter != GBR_LIM_NONE && c.limiter != GBR_LIM_MP))
            return g0->err = "batched stepping needs static periodic 2-D Euler MEG6 grids without a sponge, "
                             "with limiter NONE or MP",
                   GBR_E_UNSUPPORTED;
        const gbr_config &c0 = g0->cfg;
        if (c.precision != c0.precision || c.limiter != c0.limiter || c.gamma != c0.gamma ||
            c.alpha_mp != c0.alpha_mp || c.beta_mp != c0.beta_mp)
            return g0->err = "batched grids must share precision, limiter, gamma and MP constants", GBR_E_ARG;
        if (g[b]->stream != g0->stream) return g0->err = "batched grids must share one stream", GBR_E_ARG;
        if (g[b]->device != g0->device) return g0->err = "batched grids must share one device", GBR_E_ARG;
        for (int q = 0; q < b; ++q)
            if (g[q] == g[b]) return g0->err = "a grid appears twice in the batch", GBR_E_ARG;
    }
    gbr_batch_s *bt = new (std::nothrow) gbr_batch_s;
    if (!bt) return GBR_E_NOMEM;
    bt->grids.assign(g, g + n);
    bt->precision = g0->cfg.precision;
    bt->limited = g0->cfg.limiter == GBR_LIM_MP;
    bt->ph = phys_of(g0);
    hipError_t e = hipStreamCreateWithFlags(&bt->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->ev_out, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc((void **)&bt->d_grids, n * sizeof(BatchGrid));
    if (e == hipSuccess) e = hipMalloc((void **)&bt->d_dtmin, n * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc((void **)&bt->d_dt, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&bt->d_t, n * sizeof(double));
    std::vector<BatchGrid> host(n);
    for (int b = 0; b < n; ++b) {
        gbr_grid_s *gg = g[b];
        host[b] = BatchGrid{gg->cfg.n[0], gg->cfg.n[1], gg->ncell, gg->metrics, Q[b], gg->qn, gg->res, gg->flags};
    }
    // the batch stream starts after the work already queued on the grids' stream
    if (e == hipSuccess) e = hipEventRecord(bt->ev_in, g0->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(bt->stream, bt->ev_in, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(bt->d_grids, host.data(), n * sizeof(BatchGrid), hipMemcpyHostToDevice, bt->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_zero, dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, bt->stream, bt->d_t, n);
        hipLaunchKernelGGL(k_zero, dim3(unsigned((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, bt->stream, bt->d_dt, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = (tile == GBR_TILE_AUTO) ? autotune(bt) : upload_items(bt, tile);
    if (e == hipSuccess) e = hipStreamSynchronize(bt->stream);
    if (e != hipSuccess) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "batch create: %s", hipGetErrorString(e));
        g0->err = buf;
        release_batch(bt);
        return e == hipErrorOutOfMemory ? GBR_E_NOMEM : GBR_E_DEVICE;
    }
    *out = bt;
    return GBR_OK;
}

gbr_status gbr_batch_run(gbr_batch b, int steps, double cfl_or_dt, int dt_mode, int use_graph)
{
    using namespace gbr;
    if (!b) return GBR_E_ARG;
    gbr_grid_s *g0 = b->grids[0];
    if (steps < 0) return g0->err = "steps must be >= 0", GBR_E_ARG;
    if (dt_mode != GBR_DT_CFL && dt_mode != GBR_DT_FIXED) return g0->err = "unknown dt mode", GBR_E_ARG;
    if (!(cfl_or_dt > 0.0)) return g0->err = "cfl / dt must be positive", GBR_E_ARG;
    if (steps == 0) return GBR_OK;
    hipError_t e = hipEventRecord(b->ev_in, g0->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_in, 0);
    if (e == hipSuccess && use_graph && (!b->exec || b->g_cfl != cfl_or_dt || b->g_mode != dt_mode)) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = enqueue_step(b, cfl_or_dt, dt_mode);
            e = hipStreamEndCapture(b->stream, &b->graph);
            if (e == hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e == hipSuccess) {
            b->g_cfl = cfl_or_dt;
            b->g_mode = dt_mode;
        }
    }
    for (int s = 0; s < steps && e == hipSuccess; ++s)
        e = use_graph ? hipGraphLaunch(b->exec, b->stream) : enqueue_step(b, cfl_or_dt, dt_mode);
    // later work on the grids' stream waits for the batch
    if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(g0->stream, b->ev_out, 0);
    if (e != hipSuccess) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "batch run: %s", hipGetErrorString(e));
        g0->err = buf;
        return e == hipErrorOutOfMemory ? GBR_E_NOMEM : GBR_E_DEVICE;
    }
    return GBR_OK;
}

gbr_status gbr_batch_query(gbr_batch b, double *t, double *dt, int *tile)
{
    if (!b) return GBR_E_ARG;
    const size_t n = b->grids.size();
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess && t) e = hipMemcpy(t, b->d_t, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess && dt) e = hipMemcpy(dt, b->d_dt, n * sizeof(double), hipMemcpyDeviceToHost);
    if (tile) *tile = b->tile;
    if (e != hipSuccess) {
        b->grids[0]->err = std::string("batch query: ") + hipGetErrorString(e);
        return GBR_E_DEVICE;
    }
    return GBR_OK;
}

gbr_status gbr_batch_destroy(gbr_batch b)
{
    gbr::release_batch(b);
    return GBR_OK;
}

}  // extern "C"

// Right-hand-side kernels (Sec. 3, Sec. 5.1 Steps 1-7, Sec. 5.2 Steps 1-5),
// SSP-RK3 stage (App. B) and time step (App. B).
//
// One RHS evaluation is 2 + ndim launches:
//   k_prims       : per cell, primitives (rho, u, v, w, p) and T from Q into
//                   structure-of-arrays scratch (the only divisions by rho),
//                   and the positivity / finiteness check of the state.
//   k_cell_grad   : per cell, E6 gradients of (u, v, w, T) along xi, eta,
//                   zeta (kept for the tangential viscous terms) and the
//                   Ducros sensor flag; LDS-tiled in (i, j) with a register window
//                   along k.
//   k_sweep<D>    : per direction D, a tile of interfaces along D: primitive
//                   pencils staged in LDS with a 6-cell halo, E6 first
//                   derivatives and (see kCurvLds) the Hermite second
//                   derivatives formed once per cell in LDS; one thread per
//                   interface forms the characteristic (limited) or direct
//                   van Leer states, HLLC and the alpha-damping viscous
//                   flux. The fluxes go
//                   back to LDS and each cell accumulates
//                   -(Phi(+1/2) - Phi(-1/2)) into Res (written by the first
//                   sweep, zeta in 3-D and eta in 2-D, updated by the others;
//                   in gbr_step the xi sweep comes last and applies the
//                   SSP-RK3 stage).
// Tiles along D overlap by one interface, so no cell needs a flux computed by
// another workgroup.
//
// Precision: the RHS kernels are templated on the compute type R. FP64 runs
// everything in double. FP32-bulk (R = float) keeps primitives, gradients,
// the sensor, the reconstruction, limiter, HLLC, viscous flux and Res in
// float and reads the metrics from a float copy of the double ones, while
// Q, J and (1/J)_t stay in double and the RK stage accumulates in double.
#include <algorithm>
#include <type_traits>

#include "gbr_device.hpp"
#include "gbr_internal.hpp"

namespace gbr {
namespace {

constexpr int kBlock = 256;
#ifndef GBR_TS_CROSS
#define GBR_TS_CROSS 16
#endif
#ifndef GBR_TS_XI
#define GBR_TS_XI 128
#endif
#ifndef GBR_COMPACT_DIRS
#define GBR_COMPACT_DIRS 7  // bit D: gather the sensor-flagged interfaces of sweep D (FP64)
#endif
// Where the sweep keeps the Hermite second derivatives of its cells in an
// LDS array (formed once per cell) and where each interface forms the
// curvatures of its characteristic fields from their values and first
// derivatives instead (limited_states_pre). The FP64 eta / zeta sweeps do
// the latter: without the array their LDS drops from 43.9 to 31.8 KB and,
// with the limiter's per-field pencil reads, their registers from 162 to
// 108, a fourth wave per SIMD (eta -3 %, MIG4 eta / zeta -5 / -2 % on the
// 13 M jet). The FP64 xi sweep, already at four waves, and the FP32-bulk
// sweeps keep the array: for them the extra arithmetic costs more.
template <int D, class R>
constexpr bool kCurvLds = sizeof(R) == 4 || D == 0;

// Workgroups are handed to the eight XCDs in turn, and each XCD has its own
// L2. Neighbouring tiles of a line share halo cells, and with them whole
// 128-byte lines; in launch order they land on different XCDs, whose L2s
// each fetch those lines. The tiled kernels therefore take their tile from
// a permuted block index: within each run of 8 x GBR_XCD_GROUP consecutive
// blocks, block 8a + x (on XCD x) takes tile GBR_XCD_GROUP x + a, so
// GBR_XCD_GROUP consecutive tiles run on one XCD at about the same time and
// the shared lines are fetched once into its L2. The order across the grid
// is unchanged, and blocks past the last full run keep their own tile.
// Groups of 32 also hold the neighbours across the lines of a tile in the
// eta / zeta sweeps, whose FP32 rows (16 floats) are half a 128-byte line.
// (On the 13 M jet: FP64 sweeps and gradients read about 150 B per
// cell-RHS less; FP32-bulk step 7.4 -> 6.55 ms, FP64 11.2 -> 11.1 ms.)
#ifndef GBR_XCD_GROUP
#define GBR_XCD_GROUP 32
#endif
__device__ __forceinline__ void tile_of_block(int &bx, int &by)
{
    constexpr unsigned run = 8u * GBR_XCD_GROUP;
    const unsigned nx = gridDim.x, total = nx * gridDim.y;
    unsigned b = blockIdx.x + nx * blockIdx.y;
    if (b / run < total / run) b = run * (b / run) + GBR_XCD_GROUP * (b % 8u) + (b % run) / 8u;
    bx = int(b % nx);
    by = int(b / nx);
}

template <class R>
struct PhysR {
    R gamma, igm1, gM2, suth, re, ikden, theta_c, alpha_mp, beta_mp, alpha_d;  // igm1 = 1 / gm1, ikden = 1 / kden
    int limiter;
};

template <class R>
struct RhsArgs {
    Dims dm;
    Phys ph;       // double parameters (time step, RK)
    PhysR<R> pr;   // the same in the compute type
    const double *Q;
    R *res;
    R *grad;       // 12 * ncell: (d * 4 + s), s = u, v, w, T
    R *grad2;      // 6 * ncell (MIG4): (d * 2 + s), s = rho, p
    unsigned char *flag;  // ncell: 1 where the Ducros sensor exceeds theta_c
    R *prim;       // 6 * ncell: rho, u, v, w, p, T
    const double *m;  // metrics (always double)
    const R *mr;      // the metrics the flux kernels read in the compute type:
                      // m itself (FP64), or its float copy (FP32-bulk: slots
                      // 0 .. 47, the face slots and cell unhatted metrics)
    int *flags;
    // SSP-RK3 stage fused into the last sweep (gbr_step only)
    const double *Qin; // stage input state
    double *Qout;      // stage output state (may equal Qin or Qn: each cell is read before it is written)
    const double *Qn;  // stage-0 state
    const double *dt;  // time step (device)
    double ca, cb;     // stage coefficients
    R *prim_out;       // primitives of the updated state for the next stage, or null
    const double *sigma;  // sponge strength per cell (fused stage), or null
    double qref[5];       // sponge reference state, conserved
    int moving;           // grid velocities present (temporal metrics non-zero)
};

__device__ __forceinline__ long pack(const Dims &dm, int i, int j, int k)
{
    return i + (long)dm.n[0] * (j + (long)dm.n[1] * k);
}

// Linear index of the cell at position s along direction sd, c along cd and
// o along the remaining direction.
__device__ __forceinline__ long cell_of(const Dims &dm, int sd, int cd, int s, int c, int o)
{
    int t[3];
    t[sd] = s;
    t[cd] = c;
    t[3 - sd - cd] = o;
    return pack(dm, t[0], t[1], t[2]);
}

// ----------------------------------------------------------------------------
// primitives, cell gradients and sensor
// ----------------------------------------------------------------------------
template <int NDIM, class R>
__device__ __forceinline__ void prims_cell(const RhsArgs<R> &a, long idx)
{
    const long N = a.dm.ncell;
    double r = a.Q[idx];
    double ir = 1.0 / r;
    double u = a.Q[N + idx] * ir;
    double v = a.Q[2 * N + idx] * ir;
    double w = (NDIM == 3) ? a.Q[3 * N + idx] * ir : 0.0;
    double E = a.Q[(NDIM + 1) * N + idx];
    double p = a.ph.gm1 * (E - 0.5 * r * (u * u + v * v + w * w));
    double T = a.ph.gM2 * p * ir;
    a.prim[idx] = R(r);
    a.prim[N + idx] = R(u);
    a.prim[2 * N + idx] = R(v);
    a.prim[3 * N + idx] = R(w);
    a.prim[4 * N + idx] = R(p);
    a.prim[5 * N + idx] = R(T);
    // ghost cells of bounded directions take their states from the boundary
    // types afterwards; only interior states are checked
    if (!(r > 0.0 && p > 0.0 && isfinite(r) && isfinite(p) && isfinite(u) && isfinite(v) && isfinite(w)) &&
        in_box(a.dm, idx))
        atomicOr(a.flags, 1);
}

template <int NDIM, class R>
__global__ void __launch_bounds__(kBlock) k_prims(RhsArgs<R> a)
{
    long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    if (idx < a.dm.ncell) prims_cell<NDIM, R>(a, idx);
}

// Ducros sensor (a gate of the limiter added by this implementation, not in
// the paper): theta = div^2 /
// (div^2 + |curl|^2 + 1e-30) of the physical velocity gradient
// G[a][b] = sum_d (d_{x_b}) du_a/dd from the computational gradients gd[d][a].
// The kernels keep one byte per cell, theta > theta_c, in the compute type;
// an interface is limited when either of its cells is flagged, which is the
// same decision as max(theta_a, theta_b) > theta_c.
template <class R>
__device__ __forceinline__ void load_unhat(const R *m, long N, long idx, R mt[3][3])
{
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int d = 0; d < 3; ++d) mt[b][d] = R(m[GBR_SLOT_CELL_UNHAT(d, b) * N + idx]);
}

template <class R>
__device__ __forceinline__ R ducros_theta(const R gd[3][4], const R mt[3][3])
{
    R G[3][3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
#pragma unroll
        for (int aa = 0; aa < 3; ++aa) G[aa][b] = mt[b][0] * gd[0][aa] + mt[b][1] * gd[1][aa] + mt[b][2] * gd[2][aa];
    }
    R div = G[0][0] + G[1][1] + G[2][2];
    R wx = G[2][1] - G[1][2], wy = G[0][2] - G[2][0], wz = G[1][0] - G[0][1];
    R d2 = div * div;
    return cdiv(d2, d2 + (wx * wx + wy * wy + wz * wz) + R(1e-30));
}

// MIG4 gradients (Eq. IG4_grads, read as differences, alpha = 5/14) from the
// factorisation of the tridiagonal left-hand side: with
// q = (1 - sqrt(1 - 4 alpha^2)) / (2 alpha), alpha E^-1 + 1 + alpha E equals
// (alpha / q)(1 + q E^-1)(1 + q E), whose inverse on the infinite (or
// periodically extended) line is K sum_m (-q)^|m| E^m, K = 1 / sqrt(1 - 4 alpha^2).
// So f' = K (L + R) with two first-order recurrences over the right-hand
// side r_k = a (f_{k+1} - f_{k-1}) + b (f_{k+2} - f_{k-2}):
//   L_k = r_k - q L_{k-1}          (= sum_{m >= 0} (-q)^m r_{k-m}),
//   R_k = -q (r_{k+1} + R_{k+1})   (= sum_{m >= 1} (-q)^m r_{k+m}).
// Started 46 cells away (q^46 < 5e-18) they give the cyclic solution to FP64
// rounding, like the explicit stencil of gbr_stencil.hip, at a few
// operations per cell instead of a 97-point sum.
// A workgroup stages a tile of TS cells along D plus a 48-cell halo on each
// side for TC lines in LDS, one variable at a time. Each line of LEN = TS +
// 96 positions is cut into NSEG segments of S positions, one per thread:
// every thread runs both recurrences over its segment from zero, the
// segments' end values meet in LDS, and each thread adds the carries of the
// segments before it (L) and after it (R), weighted by powers of (-q)^S,
// over the segments that reach it above 1e-18. Long tiles keep the halo
// share small: along xi 8 lines of 416 cells (32 segments of 16), along
// eta / zeta 16 lines (i fastest, coalesced) of 192 cells (16 segments of
// 18); lines shorter than a tile are staged around their period.
template <int D>
struct Ig4RecTile {
    static constexpr int H = kIg4Half;
    static constexpr int TS = (D == 0) ? 416 : 192;
    static constexpr int TC = (D == 0) ? 8 : 16;
    static constexpr int LEN = TS + 2 * H;
    static constexpr int S = (D == 0) ? 16 : 18;
    static constexpr int NSEG = LEN / S;
    static_assert(NSEG * S == LEN && NSEG * TC == 256, "one segment per thread");
    static constexpr int SD = D;
    static constexpr int CD = (D == 0) ? 1 : 0;
    static constexpr int OD = (D == 2) ? 1 : 2;
    // Along xi the threads of a line walk their segments side by side, so a
    // row keeps one spare word after every segment (segment starts then fall
    // into different LDS banks), and four spare words before and after the
    // rows take the window's reach two positions past the line ends (the
    // values read there only enter right-hand sides that are zero). Eta /
    // zeta rows are c fastest and their end segments clamp the window
    // instead, which keeps the workgroup within 40 KB of LDS.
    static constexpr int ROW = LEN + NSEG;
    static constexpr int BUF = (D == 0) ? ROW * TC + 8 : LEN * TC;
    // LDS position of (s, c), 0 <= s < LEN
    __device__ static constexpr int at(int sl, int cl)
    {
        return D == 0 ? 4 + cl * ROW + sl + sl / S : sl * TC + cl;
    }
    // offset of position p0 + t from at(p0, c) for a segment start p0,
    // -2 <= t <= S + 2 (along eta / zeta only inside the staged line)
    __device__ static constexpr int rel(int t) { return D == 0 ? t + (t < 0 ? -1 : t / S) : t * TC; }
    // segment end values: along xi [line][segment] with a spare word per
    // line, along eta / zeta [segment][line]; L of the last segment and R of
    // the first are never read and not stored there
    static constexpr int NEND = (D == 0) ? TC * (NSEG + 1) : (NSEG - 1) * TC;
    __device__ static constexpr int endl_at(int sg, int cl) { return D == 0 ? cl * (NSEG + 1) + sg : sg * TC + cl; }
    __device__ static constexpr int endr_at(int sg, int cl)
    {
        return D == 0 ? cl * (NSEG + 1) + sg : (sg - 1) * TC + cl;
    }
    // thread -> (line, segment)
    __device__ static constexpr int line_of(int tid) { return D == 0 ? tid / NSEG : tid % TC; }
    __device__ static constexpr int seg_of(int tid) { return D == 0 ? tid % NSEG : tid / TC; }
};

template <int D, int NDIM, class R>
__global__ void __launch_bounds__(kBlock) k_ig4_rec(RhsArgs<R> a, Ig4Rec rc)
{
    using T = Ig4RecTile<D>;
    constexpr int H = T::H, TS = T::TS, TC = T::TC, LEN = T::LEN, S = T::S, NSEG = T::NSEG;
    constexpr int CARRY = (H - 2 + S - 1) / S;  // segments whose end values reach a segment above q^46
    __shared__ R buf[T::BUF];
    __shared__ R endL[T::NEND], endR[T::NEND];
    const Dims &dm = a.dm;
    const long N = dm.ncell;
    const int ns = dm.n[T::SD], nc = dm.n[T::CD];
    const int tiles_s = (ns + TS - 1) / TS;
    int bx, o;
    tile_of_block(bx, o);
    const int s0 = (bx % tiles_s) * TS;
    const int c0 = (bx / tiles_s) * TC;
    const int tid = threadIdx.x;
    const int cl = T::line_of(tid), sg = T::seg_of(tid);
    const int p0 = sg * S;  // first position of this thread's segment
    if constexpr (D == 0) {
        // clear the spare words before and after the rows (read, never used)
        if (tid < 4) buf[tid] = R(0);
        if (tid < 4) buf[T::BUF - 4 + tid] = R(0);
    }
    const R q = R(rc.q), K = R(rc.K), ca = R(rc.a), cb = R(rc.b), rho = R(rc.pw[S]);
    R *outs[6] = {a.grad2 + (D * 2 + 0) * N, a.grad + (D * 4 + 0) * N, a.grad + (D * 4 + 1) * N,
                  a.grad + (D * 4 + 2) * N, a.grad2 + (D * 2 + 1) * N, a.grad + (D * 4 + 3) * N};
    // Staging with light index arithmetic: element e = tid + q kBlock of the
    // tile. Along eta / zeta its cross lane is fixed (tid % TC) and its
    // position along the line advances by kBlock / TC per q; along xi a line
    // of LEN = 2 kBlock positions takes two q per line, so each thread has
    // two positions along s and one line per pair of q. The periodic wrap is
    // applied once and then advanced by subtraction.
    static_assert(D != 0 || LEN == 2 * kBlock, "xi rows of two blocks");
    const long sd_stride = (T::SD == 0) ? 1 : (T::SD == 1 ? (long)dm.n[0] : (long)dm.n[0] * dm.n[1]);
    auto stage = [&](const R *f) {
        if constexpr (D == 0) {
            const int s_a = wrap_index(s0 - H + tid, ns);
            const int s_b = wrap_index(s0 - H + tid + kBlock, ns);
            R va[TC], vb[TC];
#pragma unroll
            for (int cc = 0; cc < TC; ++cc) {
                const long base = cell_of(dm, T::SD, T::CD, 0, min(c0 + cc, nc - 1), o);
                va[cc] = f[base + s_a];
                vb[cc] = f[base + s_b];
            }
#pragma unroll
            for (int cc = 0; cc < TC; ++cc) {
                buf[T::at(tid, cc)] = va[cc];
                buf[T::at(tid + kBlock, cc)] = vb[cc];
            }
        } else {
            constexpr int STEP = kBlock / TC;
            constexpr int NE = LEN / STEP;
            static_assert(NE * STEP == LEN, "whole staging rounds");
            const int cc = tid % TC;
            const long base = cell_of(dm, T::SD, T::CD, 0, min(c0 + cc, nc - 1), o);
            const int sl0 = tid / TC;
            int sg_ = wrap_index(s0 - H + sl0, ns);
            if (ns >= STEP) {
                // one conditional subtraction keeps the position in [0, ns),
                // so the loop unrolls and all NE loads are in flight at once
                // (the empty asm keeps the compiler from hoisting the offset
                // sequence out of the loop over variables, which would hold
                // NE addresses in registers for the kernel's lifetime)
                __asm__ volatile("" : "+v"(sg_));
                long off = sg_ * sd_stride;
                const long step_off = STEP * sd_stride, wrap_off = ns * sd_stride;
                R v[NE];
#pragma unroll
                for (int k = 0; k < NE; ++k) {
                    v[k] = f[base + off];
                    sg_ += STEP;
                    off += step_off;
                    if (sg_ >= ns) {
                        sg_ -= ns;
                        off -= wrap_off;
                    }
                }
#pragma unroll
                for (int k = 0; k < NE; ++k) buf[T::at(sl0 + k * STEP, cc)] = v[k];
            } else {
                for (int sl = sl0; sl < LEN; sl += STEP) {
                    buf[T::at(sl, cc)] = f[base + sg_ * sd_stride];
                    sg_ += STEP;
                    while (sg_ >= ns) sg_ -= ns;
                }
            }
        }
    };
    // window of the segment: positions p0 - 2 .. p0 + S + 2; along eta /
    // zeta the first segment reads position 0 for the two before it and the
    // last reads position LEN - 1 for the three after it
    const R *seg = buf + T::at(p0, cl);
    auto win = [&](int t) -> const R * {
        if constexpr (D == 0) {
            return seg + T::rel(t);
        } else {
            if (t < 0) return sg == 0 ? seg : seg + T::rel(t);
            if (t >= S) return sg == NSEG - 1 ? seg + T::rel(S - 1) : seg + T::rel(t);
            return seg + T::rel(t);
        }
    };
    // along eta / zeta each thread stores its own outputs (16 lanes of a
    // line row are 128 contiguous bytes); along xi they go back through LDS
    const int cgl = c0 + cl;
    const long out_base = cell_of(dm, T::SD, T::CD, 0, min(cgl, nc - 1), o);
#pragma unroll 1
    for (int v = 0; v < 6; ++v) {
        if (NDIM == 2 && v == 3) {  // w is identically zero in 2-D
            for (int e = tid; e < TS * TC; e += kBlock) {
                const int sl = (D == 0) ? e % TS : e / TC;
                const int cc = (D == 0) ? e / TS : e % TC;
                if (s0 + sl < ns && c0 + cc < nc) outs[v][cell_of(dm, T::SD, T::CD, s0 + sl, c0 + cc, o)] = R(0);
            }
            continue;
        }
        const R *f = a.prim + (long)v * N;
        stage(f);
        __syncthreads();
        // forward recurrence over the segment from zero, the right-hand sides
        // from a sliding window (positions within two of the staged ends have
        // none); only L is kept: r_k = L_k + q L_{k-1} recovers the
        // right-hand sides for the backward passes
        R Ll[S];
        R fm2 = *win(-2), fm1 = *win(-1), f0 = *win(0), fp1 = *win(1);
        R L = R(0), rnext = R(0);
#pragma unroll
        for (int t = 0; t <= S; ++t) {
            const int p = p0 + t;
            const R fp2 = *win(t + 2);
            const R r = (p >= 2 && p <= LEN - 3) ? ca * (fp1 - fm1) + cb * (fp2 - fm2) : R(0);
            if (t < S) {
                L = r - q * L;
                Ll[t] = L;
            } else {
                rnext = r;
            }
            fm2 = fm1;
            fm1 = f0;
            f0 = fp1;
            fp1 = fp2;
        }
        auto rhs_at = [&](int t) { return t == 0 ? Ll[0] : Ll[t] + q * Ll[t - 1]; };
        // backward recurrence from zero: only its value at the segment start
        R Rr = R(0);
#pragma unroll
        for (int t = S - 1; t >= 0; --t) Rr = -q * ((t == S - 1 ? rnext : rhs_at(t + 1)) + Rr);
        // L at the segment's last position and R at its first, from zero
        if (D == 0 || sg < NSEG - 1) endL[T::endl_at(sg, cl)] = L;
        if (D == 0 || sg > 0) endR[T::endr_at(sg, cl)] = Rr;
        __syncthreads();
        // carries: true L before the segment, true R after it
        R cin = R(0), cout = R(0);
#pragma unroll
        for (int m = CARRY; m >= 1; --m) {
            cin = rho * cin + ((sg - m >= 0) ? endL[T::endl_at(sg - m, cl)] : R(0));
            cout = rho * cout + ((sg + m < NSEG) ? endR[T::endr_at(sg + m, cl)] : R(0));
        }
        // true R backwards from the carry, true L in closed form from the carry
        Rr = cout;
        if constexpr (D == 0) {
#pragma unroll
            for (int t = S - 1; t >= 0; --t) {
                Rr = -q * ((t == S - 1 ? rnext : rhs_at(t + 1)) + Rr);
                buf[T::at(p0, cl) + T::rel(t)] = K * ((Ll[t] + R(rc.pw[t + 1]) * cin) + Rr);
            }
            __syncthreads();
            for (int e = tid; e < TS * TC; e += kBlock) {
                const int sl = e % TS;
                const int cc = e / TS;
                if (s0 + sl < ns && c0 + cc < nc)
                    outs[v][cell_of(dm, T::SD, T::CD, s0 + sl, c0 + cc, o)] = buf[T::at(H + sl, cc)];
            }
            __syncthreads();
        } else {
            // positions H .. H + TS - 1 of the line are the tile's cells
            // s0 .. s0 + TS - 1; the next variable's staging may overwrite
            // buf at once, since every thread has passed its window reads
            // (cell of the segment's last position, made opaque so that the
            // store addresses are formed here rather than held across the
            // loop over variables)
            int sp = s0 + p0 - H + S - 1;
            __asm__ volatile("" : "+v"(sp));
            R *dst = outs[v] + out_base + (long)sp * sd_stride;
#pragma unroll
            for (int t = S - 1; t >= 0; --t) {
                Rr = -q * ((t == S - 1 ? rnext : rhs_at(t + 1)) + Rr);
                if (p0 + t >= H && p0 + t < H + TS && sp < ns && cgl < nc)
                    *dst = K * ((Ll[t] + R(rc.pw[t + 1]) * cin) + Rr);
                --sp;
                dst -= sd_stride;
            }
        }
    }
}

// Sensor from the stored cell gradients (MIG4).
template <int NDIM, class R>
__global__ void __launch_bounds__(kBlock) k_sensor(RhsArgs<R> a)
{
    long idx = blockIdx.x * (long)kBlock + threadIdx.x;
    const long N = a.dm.ncell;
    if (idx >= N) return;
    R gd[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < 4; ++q) gd[d][q] = (d < NDIM) ? a.grad[(d * 4 + q) * N + idx] : R(0);
    R mt[3][3];
    load_unhat(a.mr, N, idx, mt);
    a.flag[idx] = ducros_theta(gd, mt) > a.pr.theta_c;
}

// Gradient tile: GI x GJ cells in the (i, j) plane, marching KC planes along
// k. Each k plane of (u, v, w, T) is staged in LDS with a 3-cell i/j halo for
// the xi and eta derivatives; the zeta derivative comes from a 7-deep register
// window along the thread's own column, which also supplies the tile's own
// cells of the LDS plane, so only the halo is read a second time.
// 16 x 16 tiles in FP64, where the smaller halo pays; 32 x 8 in FP32-bulk,
// where the wider rows do (both measured on the 13 M jet workload).
#ifndef GBR_GRAD_GI64
#define GBR_GRAD_GI64 16
#endif
#ifndef GBR_GRAD_GI32
#define GBR_GRAD_GI32 32
#endif
// Planes per tile along k: 8 re-reads more window planes than 16 (14 / 8
// against 22 / 16 per plane) but doubles the workgroups, which hides more
// latency (13 M jet: 0.575 -> 0.555 ms in FP64; 4 and 12 measured between).
#ifndef GBR_GRAD_KC
#define GBR_GRAD_KC 8
#endif
template <class R>
struct GradTile {
    static constexpr int GI = sizeof(R) == 8 ? GBR_GRAD_GI64 : GBR_GRAD_GI32;
    static constexpr int GJ = kBlock / GI, KC = GBR_GRAD_KC, HI = GI + 6, HJ = GJ + 6;
};

template <int NDIM, bool SENSOR, class R>
__global__ void __launch_bounds__(kBlock) k_cell_grad(RhsArgs<R> a)
{
    constexpr int GI = GradTile<R>::GI, GJ = GradTile<R>::GJ, KC = GradTile<R>::KC;
    constexpr int HI = GradTile<R>::HI, HJ = GradTile<R>::HJ;
    __shared__ R sp[4][HJ][HI];
    const Dims &dm = a.dm;
    const long N = dm.ncell;
    const int ni = dm.n[0], nj = dm.n[1], nk = dm.n[2];
    const int tiles_i = (ni + GI - 1) / GI;
    int bx, bz;
    tile_of_block(bx, bz);
    const int i0 = (bx % tiles_i) * GI, j0 = (bx / tiles_i) * GJ;
    const int k0 = bz * KC;
    const int ti = threadIdx.x % GI, tj = threadIdx.x / GI;
    const int i = i0 + ti, j = j0 + tj;
    const bool inside = i < ni && j < nj;
    const int ic = min(i, ni - 1), jc = min(j, nj - 1);
    const R *f[4] = {a.prim + N, a.prim + 2 * N, a.prim + 3 * N, a.prim + 5 * N};
    // halos leave the grid only for tiles at the ends of their lines
    const bool edge_ij = i0 < 3 || i0 + GI + 3 > ni || j0 < 3 || j0 + GJ + 3 > nj;
    const bool edge_k = k0 < 3 || k0 + KC + 3 > nk;
    R win[7][4];
    if (NDIM == 3) {
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const long c = pack(dm, ic, jc, wrap_if(edge_k, k0 - 3 + q, nk));
#pragma unroll
            for (int s = 0; s < 4; ++s) win[q][s] = f[s][c];
        }
    }
    const int kend = min(k0 + KC, nk);
    for (int k = k0; k < kend; ++k) {
        // the sensor's metrics are requested before the halo loads and the
        // barrier, so their latency overlaps that work
        R mt[3][3];
        if (SENSOR) load_unhat(a.mr, N, pack(dm, ic, jc, k), mt);
        if (NDIM == 3) {
            const long c = pack(dm, ic, jc, wrap_if(edge_k, k + 3, nk));
#pragma unroll
            for (int s = 0; s < 4; ++s) win[6][s] = f[s][c];
            // the tile's own cells of plane k are already in the register
            // window (read three planes ago, long evicted from L2 by the
            // other resident tiles): only the halo comes from memory
            if (inside) {
#pragma unroll
                for (int s = 0; s < 4; ++s) sp[s][tj + 3][ti + 3] = win[3][s];
            }
        }
        for (int e = threadIdx.x; e < HI * HJ; e += kBlock) {
            const int x = e % HI, y = e / HI;
            const int gi = i0 - 3 + x, gj = j0 - 3 + y;
            if (NDIM == 3 && x >= 3 && x < GI + 3 && y >= 3 && y < GJ + 3 && gi < ni && gj < nj) continue;
            const long c = pack(dm, wrap_if(edge_ij, gi, ni), wrap_if(edge_ij, gj, nj), k);
#pragma unroll
            for (int s = 0; s < 4; ++s) sp[s][y][x] = f[s][c];
        }
        __syncthreads();
        if (inside) {
            const long idx = pack(dm, i, j, k);
            R gd[3][4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const R *r = &sp[s][tj + 3][ti + 3];
                gd[0][s] = e6(r[-3], r[-2], r[-1], r[1], r[2], r[3]);
                gd[1][s] = e6(r[-3 * HI], r[-2 * HI], r[-HI], r[HI], r[2 * HI], r[3 * HI]);
                gd[2][s] = (NDIM == 3) ? e6(win[0][s], win[1][s], win[2][s], win[4][s], win[5][s], win[6][s])
                                       : R(0);
            }
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int s = 0; s < 4; ++s) a.grad[(d * 4 + s) * N + idx] = gd[d][s];
            if (SENSOR) a.flag[idx] = ducros_theta(gd, mt) > a.pr.theta_c;
        }
        __syncthreads();
        if (NDIM == 3) {
#pragma unroll
            for (int q = 0; q < 6; ++q)
#pragma unroll
                for (int s = 0; s < 4; ++s) win[q][s] = win[q + 1][s];
        }
    }
}

// ----------------------------------------------------------------------------
// per-direction interface sweep
// ----------------------------------------------------------------------------
template <int D, int TSO = 0>
struct Tile {
    // faces per tile along D (TSO overrides the default), lanes across, and
    // index roles: s = sweep direction D, c = cross direction, o = outer direction.
    static constexpr int TS = TSO ? TSO : ((D == 0) ? GBR_TS_XI : GBR_TS_CROSS);
    static constexpr int TC = kBlock / TS;
    static constexpr int SD = D;
    static constexpr int CD = (D == 0) ? 1 : 0;
    static constexpr int OD = (D == 2) ? 1 : 2;
    static constexpr int NP = TS + 11;  // primitive cells s0-6 .. s0+TS+4
    static constexpr int N1 = TS + 5;   // first derivatives s0-3 .. s0+TS+1
    static constexpr int N2 = TS + 3;   // second derivatives s0-2 .. s0+TS
    static constexpr int ST = (D == 0) ? 1 : TC;  // LDS stride between cells along D
    // LDS offset of (s, c) in an array with ns entries along s: s fastest for
    // the xi sweep (lanes run along s), c fastest otherwise (lanes run along c).
    __device__ static constexpr int at(int s, int c, int ns) { return D == 0 ? c * ns + s : s * TC + c; }
    // thread id -> (interface index along D, cross lane)
    __device__ static constexpr int t_of(int tid) { return D == 0 ? tid % TS : tid / TC; }
    __device__ static constexpr int c_of(int tid) { return D == 0 ? tid / TS : tid % TC; }
};


// At least three 256-thread workgroups per CU (3 waves per SIMD, at most 168
// VGPRs): the FP64 sweeps sit at 160-168 registers, and one more register
// (the MIG4 sweep with the fused RK stage reached 170) would cost a third of
// the occupancy; the bound trades that for a 4-register spill there.
#ifndef GBR_SWEEP_MINWAVES
#define GBR_SWEEP_MINWAVES 3
#endif
#define GBR_SWEEP_BOUNDS __launch_bounds__(kBlock, GBR_SWEEP_MINWAVES)
// MODE: 0 writes Res, 1 adds to Res, 2 adds to Res and applies the SSP-RK3
// stage to the tile's own cells (the last sweep of a gbr_step stage).
// One tile of TS - 1 cells along D: tile bx of a set of tiles_s tiles per
// line, the first starting at cell s_begin. The LDS arrays come from the
// kernel, sized for the largest tile shape it runs.
template <int D, int NDIM, bool VISC, int MODE, bool IG4, class R, int TSO>
__device__ __forceinline__ void sweep_tile(const RhsArgs<R> &a, int s_begin, int tiles_s, int bx, int o, R *sP, R *s1,
                                           R *s2, int *s_order, int *s_count)
{
    using T = Tile<D, TSO>;
    constexpr int TS = T::TS, TC = T::TC, NP = T::NP, N1 = T::N1, N2 = T::N2, st = T::ST;
    constexpr int VP = NP * TC, V1 = N1 * TC, V2 = N2 * TC;

    const Dims &dm = a.dm;
    const PhysR<R> &ph = a.pr;
    const long N = dm.ncell;
    const int ns = dm.n[T::SD], nc = dm.n[T::CD];
    const int ts = bx % tiles_s;
    const int tcb = bx / tiles_s;
    const int s0 = s_begin + ts * (TS - 1);
    const int c0 = tcb * TC;
    const int tid = threadIdx.x;
    // every cell this tile touches along D (s0 - 6 .. s0 + TS + 4) lies in
    // [0, ns) unless the tile sits at an end of its line
    const bool edge = s0 < 6 || s0 + TS + 5 > ns;

    // Phase 1: primitives of cells s0-6 .. s0+TS+4 into LDS. The wave's issue
    // priority is raised while it requests them, so that a new tile's loads
    // go out ahead of the arithmetic of the other tiles on the SIMD.
    __builtin_amdgcn_s_setprio(2);
    for (int e = tid; e < VP; e += kBlock) {
        int sl = (D == 0) ? e % NP : e / TC;
        int cl = (D == 0) ? e / NP : e % TC;
        int sg = wrap_if(edge, s0 - 6 + sl, ns);
        int cg = min(c0 + cl, nc - 1);
        long c = cell_of(dm, T::SD, T::CD, sg, cg, o);
        int at = T::at(sl, cl, NP);
#pragma unroll
        for (int v = 0; v < 5; ++v) sP[v * VP + at] = a.prim[v * N + c];
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    // Phase 2: first derivatives of cells s0-3 .. s0+TS+1: E6 from the LDS
    // pencils (MEG6), or the stored IG4 gradients (MIG4)
    for (int e = tid; e < V1; e += kBlock) {
        int sl = (D == 0) ? e % N1 : e / TC;
        int cl = (D == 0) ? e / N1 : e % TC;
        int at = T::at(sl, cl, N1);
        if (IG4) {
            const long c = cell_of(dm, T::SD, T::CD, wrap_if(edge, s0 - 3 + sl, ns), min(c0 + cl, nc - 1), o);
            s1[0 * V1 + at] = a.grad2[(D * 2 + 0) * N + c];
            s1[1 * V1 + at] = a.grad[(D * 4 + 0) * N + c];
            s1[2 * V1 + at] = a.grad[(D * 4 + 1) * N + c];
            s1[3 * V1 + at] = a.grad[(D * 4 + 2) * N + c];
            s1[4 * V1 + at] = a.grad2[(D * 2 + 1) * N + c];
        } else {
            int pc = T::at(sl + 3, cl, NP);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const R *x = sP + v * VP + pc;
                s1[v * V1 + at] = e6(x[-3 * st], x[-2 * st], x[-st], x[st], x[2 * st], x[3 * st]);
            }
        }
    }
    __syncthreads();
    // Hermite second derivatives (Step-1) of cells s0-2 .. s0+TS, once per
    // cell, where the sweep keeps them in LDS
    if constexpr (kCurvLds<D, R>) {
        for (int e = tid; e < V2; e += kBlock) {
            int sl = (D == 0) ? e % N2 : e / TC;
            int cl = (D == 0) ? e / N2 : e % TC;
            int pc = T::at(sl + 4, cl, NP);
            int gc = T::at(sl + 1, cl, N1);
            int at = T::at(sl, cl, N2);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const R *x = sP + v * VP + pc;
                const R *g = s1 + v * V1 + gc;
                s2[v * V2 + at] = hermite2(x[-st], x[0], x[st], g[-st], g[st]);
            }
        }
        __syncthreads();
    }

    // Phase 3: one interface per thread. Interface f (f = thread id of its
    // home lane) lies between cells a = s0+t-1 and a+1 with t = t_of(f).
    // With the Ducros gate the flagged interfaces of the tile are gathered
    // onto the first lanes, so whole wavefronts run either the limited or
    // the direct states instead of both under a mask.
    int f = tid;
    bool limited = ph.limiter == GBR_LIM_MP;
    // (FP64 only: in FP32 the scattered LDS reads cost more than the
    // divergence they remove)
    constexpr bool compact = sizeof(R) == 8 && ((GBR_COMPACT_DIRS >> D) & 1);
    // raised issue priority for the sensor loads of the gather, as in phase 1
    __builtin_amdgcn_s_setprio(2);
    if (compact && ph.limiter == GBR_LIM_DUCROS) {
        const int t0 = T::t_of(tid), cl0 = T::c_of(tid);
        const int cg0 = min(c0 + cl0, nc - 1);
        const long a0 = cell_of(dm, T::SD, T::CD, wrap_if(edge, s0 + t0 - 1, ns), cg0, o);
        const long b0 = cell_of(dm, T::SD, T::CD, wrap_if(edge, s0 + t0, ns), cg0, o);
        const bool mine = (a.flag[a0] | a.flag[b0]) != 0;
        const unsigned long long bal = __ballot(mine);
        const int lane = tid % 64, wave = tid / 64;
        const int below = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) s_count[wave] = __popcll(bal);
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            before += (w < wave) ? s_count[w] : 0;
            total += s_count[w];
        }
        const int lim_rank = before + below;  // flagged interfaces on lower lanes
        s_order[mine ? lim_rank : total + (tid - lim_rank)] = tid;
        __syncthreads();
        f = s_order[tid];
        limited = tid < total;
    }
    __builtin_amdgcn_s_setprio(0);
    const int t = T::t_of(f);
    const int cl = T::c_of(f);
    const int cg = c0 + cl;
    const int cgc = min(cg, nc - 1);
    const long ca = cell_of(dm, T::SD, T::CD, wrap_if(edge, s0 + t - 1, ns), cgc, o);
    const long cb = cell_of(dm, T::SD, T::CD, wrap_if(edge, s0 + t, ns), cgc, o);
    const R *Pa = sP + T::at(t + 5, cl, NP);
    const R *Ga = s1 + T::at(t + 2, cl, N1);
    const R *Ha = kCurvLds<D, R> ? s2 + T::at(t + 1, cl, N2) : Pa;
    const R *m = a.mr;
    if (!compact && ph.limiter == GBR_LIM_DUCROS) limited = (a.flag[ca] | a.flag[cb]) != 0;
    // In the eta and zeta sweeps the interface metrics are requested before
    // the unlimited states are formed, so their latency overlaps that work
    // (the limited path reads them after the limiter, whose register peak
    // they would raise). The xi sweep, which carries the RK stage, has no
    // registers to spare for that and reads them after both paths.
    constexpr bool pre = D != 0;
    const R *gr = a.grad;
    const R *Tc = a.prim + 5 * N;
    R nt, nx, ny, nz;
    auto load_face = [&]() {
        nt = a.moving ? R(m[GBR_SLOT_FACE_HATT(D) * N + ca]) : R(0);
        nx = R(m[GBR_SLOT_FACE_HAT(D, 0) * N + ca]);
        ny = R(m[GBR_SLOT_FACE_HAT(D, 1) * N + ca]);
        nz = (NDIM == 3) ? R(m[GBR_SLOT_FACE_HAT(D, 2) * N + ca]) : R(0);
    };
    R PL[5], PR[5];
    if (limited) {
        {
            // the normal is read here and again for the flux: keeping it live
            // across the limiter costs a wave of occupancy in FP64
            R lx = R(m[GBR_SLOT_FACE_HAT(D, 0) * N + ca]);
            R ly = R(m[GBR_SLOT_FACE_HAT(D, 1) * N + ca]);
            R lz = (NDIM == 3) ? R(m[GBR_SLOT_FACE_HAT(D, 2) * N + ca]) : R(0);
            limited_states_pre<5, sizeof(R) == 8, kCurvLds<D, R>>(Pa, Ga, Ha, st, VP, V1, V2, lx, ly, lz,
                                                                             ph.gamma, ph.alpha_mp, ph.beta_mp, PL, PR);
        }
        if (pre) load_face();
    } else {
        if (pre) load_face();
        if constexpr (kCurvLds<D, R>)
            direct_states_pre<5>(Pa, Ga, Ha, st, VP, V1, V2, PL, PR);
        else
            direct_states<5>(Pa, Ga, st, VP, V1, PL, PR);
    }
    if (!pre) load_face();
    if (NDIM == 2) {
        PL[3] = R(0);
        PR[3] = R(0);
    }
    bool ok = PL[0] > R(0) && PL[4] > R(0) && PR[0] > R(0) && PR[4] > R(0);

    // HLLC (Step-6) and the alpha-damping viscous flux (Sec. 5.2); the
    // temporal metric is zero on static grids and not read there
    R phi[5];
    hllc(PL, PR, nt, nx, ny, nz, ph.gamma, ph.igm1, phi);
    if (VISC) {
        // Step-1: interface gradients of (u, v, w, T) along each computational
        // direction; the normal one from Eq. AD-eqn1 (beta_D = 0), tangential
        // ones from the average of the two cell gradients.
        // T of the two cells: in FP64 from their density and pressure in LDS
        // (T = gM2 p / rho, as the primitives kernel forms it) rather than
        // read, 8 bytes per cell less; FP32-bulk reads the float T stored
        // from the double evaluation
        R ta, tb;
        if constexpr (sizeof(R) == 8) {
            ta = ph.gM2 * Pa[4 * VP] * (R(1) / Pa[0]);
            tb = ph.gM2 * Pa[4 * VP + st] * (R(1) / Pa[st]);
        } else {
            ta = Tc[ca];
            tb = Tc[cb];
        }
        R c0v[4] = {Pa[VP], Pa[2 * VP], Pa[3 * VP], ta};
        R c1v[4] = {Pa[VP + st], Pa[2 * VP + st], Pa[3 * VP + st], tb};
        R g0[4] = {Ga[V1], Ga[2 * V1], Ga[3 * V1], gr[(D * 4 + 3) * N + ca]};
        R g1[4] = {Ga[V1 + st], Ga[2 * V1 + st], Ga[3 * V1 + st], gr[(D * 4 + 3) * N + cb]};
        R sL[4], sR[4], gf[3][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            sL[s] = c0v[s] + R(0.5) * g0[s];
            sR[s] = c1v[s] - R(0.5) * g1[s];
            gf[D][s] = R(0.5) * (g0[s] + g1[s]) + R(0.5) * ph.alpha_d * (sR[s] - sL[s]);
        }
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            if (e == D) continue;
#pragma unroll
            for (int s = 0; s < 4; ++s)
                gf[e][s] = (e < NDIM) ? R(0.5) * (gr[(e * 4 + s) * N + ca] + gr[(e * 4 + s) * N + cb]) : R(0);
        }
        // Step-2: chain rule with the interface unhatted metrics
        R Dx[4][3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            R mb[3];
#pragma unroll
            for (int e = 0; e < 3; ++e)
                mb[e] = (e < NDIM && b < NDIM) ? R(m[GBR_SLOT_FACE_UNHAT(D, e, b) * N + ca]) : R(0);
#pragma unroll
            for (int s = 0; s < 4; ++s) Dx[s][b] = mb[0] * gf[0][s] + mb[1] * gf[1][s] + mb[2] * gf[2][s];
        }
        // Step-3: stresses and heat flux at the interface
        R Tf = R(0.5) * (sL[3] + sR[3]);
        R mu = viscosity(Tf, ph.suth, ph.re);
        R lam = R(-2.0 / 3.0) * mu;
        R kap = mu * ph.ikden;
        R uf = R(0.5) * (sL[0] + sR[0]), vf = R(0.5) * (sL[1] + sR[1]), wf = R(0.5) * (sL[2] + sR[2]);
        R div = Dx[0][0] + Dx[1][1] + Dx[2][2];
        R txx = R(2) * mu * Dx[0][0] + lam * div;
        R tyy = R(2) * mu * Dx[1][1] + lam * div;
        R tzz = R(2) * mu * Dx[2][2] + lam * div;
        R txy = mu * (Dx[0][1] + Dx[1][0]);
        R txz = mu * (Dx[0][2] + Dx[2][0]);
        R tyz = mu * (Dx[1][2] + Dx[2][1]);
        R bx = uf * txx + vf * txy + wf * txz + kap * Dx[3][0];
        R by = uf * txy + vf * tyy + wf * tyz + kap * Dx[3][1];
        R bz = uf * txz + vf * tyz + wf * tzz + kap * Dx[3][2];
        // Step-4: viscous interface flux with the hatted interface metrics
        phi[1] -= nx * txx + ny * txy + nz * txz;
        phi[2] -= nx * txy + ny * tyy + nz * tyz;
        phi[3] -= nx * txz + ny * tyz + nz * tzz;
        phi[4] -= nx * bx + ny * by + nz * bz;
    }
    ok = ok && isfinite(phi[0]) && isfinite(phi[4]);
    if (!ok && cg < nc) {
        // only interfaces of interior cells count (ghost interfaces of
        // bounded directions are computed but never used)
        int lo3[3], hi3[3];
        lo3[T::SD] = s0 + t - 1;
        hi3[T::SD] = s0 + t;
        lo3[T::CD] = hi3[T::CD] = cg;
        lo3[3 - T::SD - T::CD] = hi3[3 - T::SD - T::CD] = o;
        if (in_box(dm, lo3[0], lo3[1], lo3[2]) || in_box(dm, hi3[0], hi3[1], hi3[2])) atomicOr(a.flags, 1);
    }
    // Phase-4 operands of the home cell s0+t (t and the cross lane of this
    // thread's own position), issued before the flux exchange so that their
    // latency overlaps it
    const int th = T::t_of(tid), clh = T::c_of(tid);
    const int cgh = c0 + clh;
    int h3[3];
    h3[T::SD] = s0 + th;
    h3[T::CD] = cgh;
    h3[3 - T::SD - T::CD] = o;
    const bool interior = in_box(dm, h3[0], h3[1], h3[2]);
    const bool own = th < TS - 1 && s0 + th < ns && cgh < nc && (interior || MODE == 0);
    const long ch = own ? cell_of(dm, T::SD, T::CD, s0 + th, cgh, o) : 0;
    constexpr int NV = NDIM + 2;
    R rold[NV];
    double qin[NV], qn[NV];
    double dt = 0.0, J = 0.0, it = 0.0, sg = 0.0, vj = 0.0;
    if (own && MODE >= 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) rold[v] = a.res[(long)v * N + ch];
    }
    if (own && MODE == 2) {
        dt = *a.dt;
        J = a.m[GBR_SLOT_CELL_J * N + ch];
        // (1/J)_t is zero on static grids and not read there
        it = a.moving ? a.m[GBR_SLOT_CELL_INVJT * N + ch] : 0.0;
        if (a.sigma) {
            sg = a.sigma[ch];
            vj = a.m[GBR_SLOT_CELL_INVJ * N + ch];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            qin[v] = a.Qin[(long)v * N + ch];
            qn[v] = a.Qn[(long)v * N + ch];
        }
    }
    __syncthreads();
    // interface fluxes back to LDS (reusing the primitive buffer)
#pragma unroll
    for (int v = 0; v < 5; ++v) sP[v * kBlock + T::at(t, cl, TS)] = phi[v];
    __syncthreads();
    // Phase 4: Res of cell s0+t from its two interfaces (Sec. 3, Step-7)
    if (own) {
        double qnew[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            if (NDIM == 2 && v == 3) continue;
            const int ov = (NDIM == 2 && v == 4) ? 3 : v;
            const R d = sP[v * kBlock + T::at(th + 1, clh, TS)] - sP[v * kBlock + T::at(th, clh, TS)];
            R *r = a.res + (long)ov * N + ch;
            if (MODE == 0) {
                *r = interior ? -d : R(0);  // Res is zero in ghost cells
            } else if (MODE == 1) {
                *r = rold[ov] - d;
            } else {
                // App. B with Eq. time-split: Q <- a Qn + b (Q + dt J (Res - (1/J)_t Q)),
                // Res with the sponge term -sigma (Q - Q_ref) / J (Sec. 8.3)
                const R res = rold[ov] - d;
                const long e = (long)ov * N + ch;
                const double q = qin[ov];
                double rt = double(res);
                if (a.sigma) rt -= sg * (q - a.qref[v]) * vj;
                const double L = J * (rt - it * q);
                qnew[ov] = a.ca * qn[ov] + a.cb * (q + dt * L);
                a.Qout[e] = qnew[ov];
            }
        }
        if (MODE == 2 && a.prim_out) {
            // primitives of the new state for the next stage (as k_prims)
            const double r = qnew[0];
            const double ir = 1.0 / r;
            const double u = qnew[1] * ir;
            const double v = qnew[2] * ir;
            const double w = (NDIM == 3) ? qnew[3] * ir : 0.0;
            const double E = qnew[NDIM + 1];
            const double p = a.ph.gm1 * (E - 0.5 * r * (u * u + v * v + w * w));
            const double T = a.ph.gM2 * p * ir;
            a.prim_out[ch] = R(r);
            a.prim_out[N + ch] = R(u);
            a.prim_out[2 * N + ch] = R(v);
            a.prim_out[3 * N + ch] = R(w);
            a.prim_out[4 * N + ch] = R(p);
            a.prim_out[5 * N + ch] = R(T);
            if (!(r > 0.0 && p > 0.0 && isfinite(r) && isfinite(p) && isfinite(u) && isfinite(v) && isfinite(w)))
                atomicOr(a.flags, 1);
        }
    }
}

constexpr int cmax(int x, int y) { return x > y ? x : y; }

// A sweep launch: in each row of the grid (one outer index), tiles
// [0, main_blocks) have the default shape, tiles_s per line starting at
// cell 0; with TAIL > 0 the remaining tiles of the row are one TAIL-face
// tile per line starting at cell s_tail (the remainder of each line), so
// the narrow tiles run in the same launch as the full ones.
template <int D, int NDIM, bool VISC, int MODE, bool IG4, class R, int TAIL>
__global__ void GBR_SWEEP_BOUNDS k_sweep(RhsArgs<R> a, int tiles_s, int main_blocks, int s_tail)
{
    using T0 = Tile<D>;
    using T1 = Tile<D, TAIL ? TAIL : T0::TS>;
    __shared__ R sP[5 * cmax(T0::NP * T0::TC, T1::NP * T1::TC)];
    __shared__ R s1[5 * cmax(T0::N1 * T0::TC, T1::N1 * T1::TC)];
    __shared__ R s2[kCurvLds<D, R> ? 5 * cmax(T0::N2 * T0::TC, T1::N2 * T1::TC) : 1];
    __shared__ int s_order[kBlock];
    __shared__ int s_count[kBlock / 64];
    int bx, o;
    tile_of_block(bx, o);
    if (TAIL == 0 || bx < main_blocks)
        sweep_tile<D, NDIM, VISC, MODE, IG4, R, 0>(a, 0, tiles_s, bx, o, sP, s1, s2, s_order, s_count);
    else
        sweep_tile<D, NDIM, VISC, MODE, IG4, R, TAIL>(a, s_tail, 1, bx - main_blocks, o, sP, s1, s2, s_order,
                                                      s_count);
}

// ----------------------------------------------------------------------------
// SSP-RK3 stage (double accumulation) and time step
// ----------------------------------------------------------------------------
template <int NV, class R>
__global__ void __launch_bounds__(kBlock) k_rk_stage(Dims dm, long ncell, double ca, double cb,
                                                       const double *__restrict__ dtp,
                                                       const double *__restrict__ Qn,
                                                       double *__restrict__ Q,
                                                       const R *__restrict__ res,
                                                       const double *__restrict__ jac,
                                                       const double *__restrict__ invjt)
{
    long c = blockIdx.x * (long)kBlock + threadIdx.x;
    if (c >= ncell || !in_box(dm, c)) return;  // ghost cells are not advanced
    const double dt = *dtp;
    const double J = jac[c], it = invjt[c];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const long e = c + v * ncell;
        const double q = Q[e];
        const double L = J * (double(res[e]) - it * q);
        Q[e] = ca * Qn[e] + cb * (q + dt * L);
    }
}

// Minimum of best over the block (wavefronts first) into partial[blockIdx.x].
__device__ __forceinline__ void block_min_to(double best, double *partial)
{
    for (int off = warpSize / 2; off > 0; off >>= 1) best = fmin(best, __shfl_xor(best, off));
    __shared__ double wmin[kBlock / 32];
    const int lane = threadIdx.x % warpSize, wave = threadIdx.x / warpSize;
    if (lane == 0) wmin[wave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = wmin[0];
        for (int q = 1; q < kBlock / warpSize; ++q) b = fmin(b, wmin[q]);
        partial[blockIdx.x] = b;
    }
}

// Per-block minimum of the admissible step over a grid-stride range of cells.
template <int NDIM, bool VISC>
__global__ void __launch_bounds__(kBlock) k_cfl_partial(Dims dm, Phys ph, const double *Q, const double *m,
                                                          int moving, double *partial)
{
    const long N = dm.ncell;
    double best = __builtin_inf();
    for (long idx = blockIdx.x * (long)kBlock + threadIdx.x; idx < N; idx += (long)gridDim.x * kBlock) {
        if (!in_box(dm, idx)) continue;  // ghost cells are not advanced
        best = fmin(best, cell_dt_bound<NDIM, VISC>(Q, m, N, idx, ph.gamma, ph.gm1, ph.gM2, ph.suth, ph.re,
                                                        ph.alpha_d, moving != 0));
    }
    block_min_to(best, partial);
}

// The same minimum fused with the primitives of the step's first stage
// (k_prims): both read Q at the start of a step, so one pass serves both.
template <int NDIM, bool VISC, class R>
__global__ void __launch_bounds__(kBlock) k_prims_cfl(RhsArgs<R> a, int moving, double *partial)
{
    const long N = a.dm.ncell;
    const Phys &ph = a.ph;
    double best = __builtin_inf();
    for (long idx = blockIdx.x * (long)kBlock + threadIdx.x; idx < N; idx += (long)gridDim.x * kBlock) {
        prims_cell<NDIM, R>(a, idx);
        if (!in_box(a.dm, idx)) continue;  // ghost cells are not advanced
        best = fmin(best, cell_dt_bound<NDIM, VISC>(a.Q, a.m, N, idx, ph.gamma, ph.gm1, ph.gM2, ph.suth, ph.re,
                                                        ph.alpha_d, moving != 0));
    }
    block_min_to(best, partial);
}

// Minimum of the per-block values; dt = cfl * min.
__global__ void __launch_bounds__(1024) k_cfl_final(const double *partial, int n, double cfl, double *dt)
{
    double best = __builtin_inf();
    for (int q = threadIdx.x; q < n; q += blockDim.x) best = fmin(best, partial[q]);
    for (int off = warpSize / 2; off > 0; off >>= 1) best = fmin(best, __shfl_xor(best, off));
    __shared__ double wmin[1024 / 32];
    const int lane = threadIdx.x % warpSize, wave = threadIdx.x / warpSize;
    if (lane == 0) wmin[wave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = wmin[0];
        for (int q = 1; q < (int)blockDim.x / warpSize; ++q) b = fmin(b, wmin[q]);
        dt[0] = cfl * b;
    }
}

__global__ void __launch_bounds__(kBlock) k_fill(double *p, long n, double v)
{
    long e = blockIdx.x * (long)kBlock + threadIdx.x;
    if (e < n) p[e] = v;
}

__global__ void __launch_bounds__(kBlock) k_copy(double *__restrict__ d, const double *__restrict__ s, long n)
{
    long e = blockIdx.x * (long)kBlock + threadIdx.x;
    if (e < n) d[e] = s[e];
}

// The step's time step to the caller and the grid's time advanced by it
// (t^{n+1} = t^n + dt).
__global__ void k_step_time(const double *dt, double *dt_out, double *t)
{
    if (threadIdx.x != 0) return;
    const double d = dt[0];
    if (dt_out) dt_out[0] = d;
    if (t) t[0] += d;
}

template <int D, int NDIM, bool VISC, class R, bool IG4, int TAIL>
void launch_sweep(gbr_grid_s *g, const RhsArgs<R> &a, int mode, int tiles_s, int s_tail)
{
    using T0 = Tile<D>;
    using T1 = Tile<D, TAIL ? TAIL : T0::TS>;
    const int nc = a.dm.n[T0::CD], no = a.dm.n[T0::OD];
    const int main_blocks = tiles_s * ((nc + T0::TC - 1) / T0::TC);
    const int tail_blocks = TAIL ? (nc + T1::TC - 1) / T1::TC : 0;
    dim3 grid(unsigned(main_blocks + tail_blocks), unsigned(no));
    if (mode == 0)
        hipLaunchKernelGGL((k_sweep<D, NDIM, VISC, 0, IG4, R, TAIL>), grid, dim3(kBlock), 0, g->stream, a, tiles_s,
                           main_blocks, s_tail);
    else if (mode == 1)
        hipLaunchKernelGGL((k_sweep<D, NDIM, VISC, 1, IG4, R, TAIL>), grid, dim3(kBlock), 0, g->stream, a, tiles_s,
                           main_blocks, s_tail);
    else
        hipLaunchKernelGGL((k_sweep<D, NDIM, VISC, 2, IG4, R, TAIL>), grid, dim3(kBlock), 0, g->stream, a, tiles_s,
                           main_blocks, s_tail);
}

// xi lines are cut into tiles of GBR_TS_XI - 1 = 127 cells; a remainder of
// fewer than GBR_TS_XI_TAIL cells goes to one narrow tile per line
// (GBR_TS_XI_TAIL faces, kBlock / GBR_TS_XI_TAIL lines per workgroup) in the
// same launch, so that few lanes idle (a 400-cell line: 3 tiles and 19 cells
// in a 32-face tile, instead of 4 tiles with 108 idle lanes).
#ifndef GBR_TS_XI_TAIL
#define GBR_TS_XI_TAIL 32
#endif
template <int D, int NDIM, bool VISC, class R, bool IG4>
hipError_t sweep(gbr_grid_s *g, const RhsArgs<R> &a, int mode)
{
    using T = Tile<D>;
    const int ns = a.dm.n[T::SD];
    const int own = T::TS - 1, full = ns / own, rest = ns - full * own;
    Timed timed(g, GBR_K_SWEEP_XI + D);
    if constexpr (D == 0 && GBR_TS_XI_TAIL > 0) {
        if (rest > 0 && rest < GBR_TS_XI_TAIL) {
            launch_sweep<D, NDIM, VISC, R, IG4, GBR_TS_XI_TAIL>(g, a, mode, full, full * own);
            return hipGetLastError();
        }
    }
    launch_sweep<D, NDIM, VISC, R, IG4, 0>(g, a, mode, full + (rest > 0 ? 1 : 0), 0);
    return hipGetLastError();
}

// The sweeps of one RHS in the order zeta, eta, xi (eta, xi in 2-D): the
// first writes Res, the others add to it, and with fuse_rk the xi sweep
// applies the SSP-RK3 stage. The stage's extra traffic (Q, Qn, J, (1/J)_t
// in, Q and the next primitives out) coalesces best in the xi tiles, whose
// rows are 128 cells (1 KiB) long against 16 in the eta / zeta tiles.
template <int NDIM, bool VISC, class R, bool IG4>
hipError_t sweeps(gbr_grid_s *g, const RhsArgs<R> &a, bool fuse_rk)
{
    hipError_t e;
    if (NDIM == 3 && (e = sweep<NDIM == 3 ? 2 : 1, NDIM, VISC, R, IG4>(g, a, 0)) != hipSuccess) return e;
    if ((e = sweep<1, NDIM, VISC, R, IG4>(g, a, NDIM == 3 ? 1 : 0)) != hipSuccess) return e;
    return sweep<0, NDIM, VISC, R, IG4>(g, a, fuse_rk ? 2 : 1);
}

// ----------------------------------------------------------------------------
// diagnostics from the shared cell gradients (vorticity, Q-criterion,
// |grad rho|; kinetic-energy and enstrophy averages of Eq. KE-Ens)
// ----------------------------------------------------------------------------
constexpr int kDiagBlocks = 1024;

template <int NDIM, bool IG4, class R>
__global__ void __launch_bounds__(kBlock) k_diag(RhsArgs<R> a, double *fields, double *partial)
{
    const Dims &dm = a.dm;
    const long N = dm.ncell;
    double ke = 0.0, ens = 0.0, vol = 0.0;
    for (long idx = blockIdx.x * (long)kBlock + threadIdx.x; idx < N; idx += (long)gridDim.x * kBlock) {
        int ijk[3];
        ijk[0] = int(idx % dm.n[0]);
        ijk[1] = int((idx / dm.n[0]) % dm.n[1]);
        ijk[2] = int(idx / ((long)dm.n[0] * dm.n[1]));
        double gr[3], G[3][3];
        double rd[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int d = 0; d < NDIM; ++d) {
            if (IG4) {
                rd[d] = double(a.grad2[(d * 2 + 0) * N + idx]);
            } else {
                // E6 derivative of rho along d (Eq. E6_grads)
                const long stride = (d == 0) ? 1 : (d == 1) ? dm.n[0] : (long)dm.n[0] * dm.n[1];
                const long base = idx - (long)ijk[d] * stride;
                R f[7];
#pragma unroll
                for (int q = -3; q <= 3; ++q) f[q + 3] = a.prim[base + (long)wrap_index(ijk[d] + q, dm.n[d]) * stride];
                rd[d] = double(e6(f[0], f[1], f[2], f[4], f[5], f[6]));
            }
        }
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            double mb[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) mb[d] = (d < NDIM) ? a.m[GBR_SLOT_CELL_UNHAT(d, b) * N + idx] : 0.0;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                double sum = 0.0;
#pragma unroll
                for (int d = 0; d < NDIM; ++d) sum += mb[d] * double(a.grad[(d * 4 + q) * N + idx]);
                G[q][b] = sum;
            }
            double sum = 0.0;
#pragma unroll
            for (int d = 0; d < NDIM; ++d) sum += mb[d] * rd[d];
            gr[b] = sum;
        }
        const double om[3] = {G[2][1] - G[1][2], G[0][2] - G[2][0], G[1][0] - G[0][1]};
        double s2 = 0.0, w2 = 0.0;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double sab = 0.5 * (G[p][q] + G[q][p]), wab = 0.5 * (G[p][q] - G[q][p]);
                s2 += sab * sab;
                w2 += wab * wab;
            }
        if (fields) {
            fields[idx] = om[0];
            fields[N + idx] = om[1];
            fields[2 * N + idx] = om[2];
            fields[3 * N + idx] = 0.5 * (w2 - s2);
            fields[4 * N + idx] = sqrt(gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]);
        }
        const double rho = double(a.prim[idx]), u = double(a.prim[N + idx]), v = double(a.prim[2 * N + idx]),
                     w = double(a.prim[3 * N + idx]);
        const double dv = a.m[GBR_SLOT_CELL_INVJ * N + idx];
        ke += 0.5 * rho * (u * u + v * v + w * w) * dv;
        ens += 0.5 * rho * (om[0] * om[0] + om[1] * om[1] + om[2] * om[2]) * dv;
        vol += dv;
    }
    // block sums in a fixed order (wavefront shuffles, then the waves)
    __shared__ double part[3][kBlock / 64];
    double vals[3] = {ke, ens, vol};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double x = vals[q];
        for (int off = warpSize / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (threadIdx.x % warpSize == 0) part[q][threadIdx.x / warpSize] = x;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double x = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) x += part[threadIdx.x][w];
        partial[threadIdx.x * kDiagBlocks + blockIdx.x] = x;
    }
}

__global__ void __launch_bounds__(64) k_diag_final(const double *partial, int nb, double *out)
{
    if (threadIdx.x != 0) return;
    double t[3];
    for (int q = 0; q < 3; ++q) {
        double x = 0.0;
        for (int b = 0; b < nb; ++b) x += partial[q * kDiagBlocks + b];
        t[q] = x;
    }
    out[0] = t[0] / t[2];
    out[1] = t[1] / t[2];
    out[2] = t[2];
}

template <int D, int NDIM, class R>
void ig4_grad(gbr_grid_s *g, const RhsArgs<R> &a)
{
    using T = Ig4RecTile<D>;
    const int ns = a.dm.n[T::SD], nc = a.dm.n[T::CD], no = a.dm.n[T::OD];
    dim3 grid(unsigned(((ns + T::TS - 1) / T::TS) * ((nc + T::TC - 1) / T::TC)), unsigned(no));
    hipLaunchKernelGGL((k_ig4_rec<D, NDIM, R>), grid, dim3(kBlock), 0, g->stream, a, ig4_rec());
}

// One RHS: primitives of Q (unless given), cell gradients and sensor, the
// sweeps; with fuse_rk the last sweep applies the SSP-RK3 stage.
template <int NDIM, bool VISC, class R>
hipError_t rhs_all(gbr_grid_s *g, const RhsArgs<R> &a, bool prims = true, bool fuse_rk = false)
{
    unsigned blocks = unsigned((a.dm.ncell + kBlock - 1) / kBlock);
    hipError_t e;
    if (prims) {
        Timed timed(g, GBR_K_PRIMS);
        hipLaunchKernelGGL((k_prims<NDIM, R>), dim3(blocks), dim3(kBlock), 0, g->stream, a);
    }
    // ghost primitives of bounded directions (Sec. 6); Dirichlet ghosts from
    // the caller's state a.Q, which the stages never write in ghost cells
    if (g->bounded && (e = launch_bc_prims<R>(g, a.prim, a.Q)) != hipSuccess) return e;
    if (g->cfg.scheme == GBR_SCHEME_MIG4) {
        // IG4 gradients of all primitives along every direction (they feed the
        // reconstruction as well), then the sensor from them
        {
            Timed timed(g, GBR_K_CELL_GRAD);
            ig4_grad<0, NDIM, R>(g, a);
            ig4_grad<1, NDIM, R>(g, a);
            if (NDIM == 3) ig4_grad<NDIM == 3 ? 2 : 1, NDIM, R>(g, a);
            if (a.pr.limiter == GBR_LIM_DUCROS)
                hipLaunchKernelGGL((k_sensor<NDIM, R>), dim3(blocks), dim3(kBlock), 0, g->stream, a);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        return sweeps<NDIM, VISC, R, true>(g, a, fuse_rk);
    }
    // cell gradients feed only the tangential viscous terms and the sensor
    if (VISC || a.pr.limiter == GBR_LIM_DUCROS) {
        Timed timed(g, GBR_K_CELL_GRAD);
        using GT = GradTile<R>;
        dim3 gg(unsigned(((a.dm.n[0] + GT::GI - 1) / GT::GI) * ((a.dm.n[1] + GT::GJ - 1) / GT::GJ)),
                unsigned((a.dm.n[2] + GT::KC - 1) / GT::KC));
        if (a.pr.limiter == GBR_LIM_DUCROS)
            hipLaunchKernelGGL((k_cell_grad<NDIM, true, R>), gg, dim3(kBlock), 0, g->stream, a);
        else
            hipLaunchKernelGGL((k_cell_grad<NDIM, false, R>), gg, dim3(kBlock), 0, g->stream, a);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (g->bounded && a.pr.limiter == GBR_LIM_DUCROS && (e = launch_flag_ghosts(g, a.flag)) != hipSuccess)
        return e;
    if ((e = sweeps<NDIM, VISC, R, false>(g, a, fuse_rk)) != hipSuccess) return e;
    // the sponge of a plain RHS (the fused stage applies it itself)
    if (!fuse_rk && g->sigma) e = launch_sponge<R>(g, a.Q, a.res);
    return e;
}

template <class R>
RhsArgs<R> make_args(gbr_grid_s *g, const double *Q, R *res)
{
    RhsArgs<R> a;
    a.dm = dims_of(g);
    a.ph = phys_of(g);
    const Phys &p = a.ph;
    a.pr = PhysR<R>{R(p.gamma), R(1.0 / p.gm1), R(p.gM2), R(p.suth), R(p.re), R(1.0 / p.kden),
                    R(p.theta_c), R(p.alpha_mp), R(p.beta_mp), R(p.alpha_d), p.limiter};
    a.Q = Q;
    a.res = res;
    a.grad = reinterpret_cast<R *>(g->scratch);
    a.grad2 = reinterpret_cast<R *>(g->grad2);
    a.flag = g->lim_flag;
    a.prim = reinterpret_cast<R *>(g->prim);
    a.m = g->metrics;
    if constexpr (std::is_same<R, float>::value)
        a.mr = g->metrics_f;
    else
        a.mr = g->metrics;
    a.flags = g->flags;
    a.Qin = nullptr;
    a.Qout = nullptr;
    a.Qn = nullptr;
    a.dt = nullptr;
    a.ca = a.cb = 0.0;
    a.prim_out = nullptr;
    a.sigma = g->sigma;
    for (int v = 0; v < 5; ++v) a.qref[v] = g->qref[v];
    a.moving = g->cfg.moving;
    return a;
}

template <class R>
hipError_t rhs_typed(gbr_grid_s *g, const double *Q, R *res)
{
    RhsArgs<R> a = make_args<R>(g, Q, res);
    const bool visc = g->cfg.viscous != 0;
    if (g->cfg.ndim == 3)
        return visc ? rhs_all<3, true, R>(g, a) : rhs_all<3, false, R>(g, a);
    return visc ? rhs_all<2, true, R>(g, a) : rhs_all<2, false, R>(g, a);
}

template <class R>
hipError_t diag_typed(gbr_grid_s *g, const double *Q, double *fields, double *integrals)
{
    RhsArgs<R> a = make_args<R>(g, Q, nullptr);
    const long N = g->ncell;
    const unsigned blocks = unsigned((N + kBlock - 1) / kBlock);
    const bool ig4 = g->cfg.scheme == GBR_SCHEME_MIG4;
    Timed timed(g, GBR_K_DIAG);
    const int nd = g->cfg.ndim;
    if (nd == 3)
        hipLaunchKernelGGL((k_prims<3, R>), dim3(blocks), dim3(kBlock), 0, g->stream, a);
    else
        hipLaunchKernelGGL((k_prims<2, R>), dim3(blocks), dim3(kBlock), 0, g->stream, a);
    if (ig4) {
        if (nd == 3) {
            ig4_grad<0, 3, R>(g, a);
            ig4_grad<1, 3, R>(g, a);
            ig4_grad<2, 3, R>(g, a);
        } else {
            ig4_grad<0, 2, R>(g, a);
            ig4_grad<1, 2, R>(g, a);
        }
    } else {
        using GT = GradTile<R>;
        dim3 gg(unsigned(((a.dm.n[0] + GT::GI - 1) / GT::GI) * ((a.dm.n[1] + GT::GJ - 1) / GT::GJ)),
                unsigned((a.dm.n[2] + GT::KC - 1) / GT::KC));
        if (nd == 3)
            hipLaunchKernelGGL((k_cell_grad<3, false, R>), gg, dim3(kBlock), 0, g->stream, a);
        else
            hipLaunchKernelGGL((k_cell_grad<2, false, R>), gg, dim3(kBlock), 0, g->stream, a);
    }
    const int nb = int(std::min<long>(kDiagBlocks, (N + kBlock - 1) / kBlock));
    if (nd == 3) {
        if (ig4)
            hipLaunchKernelGGL((k_diag<3, true, R>), dim3(nb), dim3(kBlock), 0, g->stream, a, fields, g->partial);
        else
            hipLaunchKernelGGL((k_diag<3, false, R>), dim3(nb), dim3(kBlock), 0, g->stream, a, fields, g->partial);
    } else {
        if (ig4)
            hipLaunchKernelGGL((k_diag<2, true, R>), dim3(nb), dim3(kBlock), 0, g->stream, a, fields, g->partial);
        else
            hipLaunchKernelGGL((k_diag<2, false, R>), dim3(nb), dim3(kBlock), 0, g->stream, a, fields, g->partial);
    }
    if (integrals) hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, g->stream, g->partial, nb, integrals);
    return hipGetLastError();
}

static const double kRkA[3] = {0.0, 0.75, 1.0 / 3.0};
static const double kRkB[3] = {1.0, 0.25, 2.0 / 3.0};

// One gbr_step stage. Q is the state at the start of the step (Qn of every
// stage) and S a stage buffer: stage 0 maps Q to S, stage 1 updates S in
// place and stage 2 maps S back into Q, so Q needs no copy. Stage 0 forms
// the primitives of Q into the first primitive buffer; each stage reads the
// buffer of its index parity and the fused last sweep writes the next
// stage's primitives into the other one.
template <class R>
hipError_t step_stage_typed(gbr_grid_s *g, int stage, const double *dt, double *Q, double *S, bool prims_ready)
{
    RhsArgs<R> a = make_args<R>(g, Q, static_cast<R *>(static_cast<void *>(g->res)));
    R *buf[2] = {reinterpret_cast<R *>(g->prim), reinterpret_cast<R *>(g->prim2)};
    a.prim = buf[stage % 2];
    a.prim_out = stage < 2 ? buf[(stage + 1) % 2] : nullptr;
    a.Qin = stage == 0 ? Q : S;
    a.Qout = stage == 2 ? Q : S;
    a.Qn = Q;
    a.dt = dt;
    a.ca = kRkA[stage];
    a.cb = kRkB[stage];
    const bool visc = g->cfg.viscous != 0, first = stage == 0 && !prims_ready;
    if (g->cfg.ndim == 3)
        return visc ? rhs_all<3, true, R>(g, a, first, true) : rhs_all<3, false, R>(g, a, first, true);
    return visc ? rhs_all<2, true, R>(g, a, first, true) : rhs_all<2, false, R>(g, a, first, true);
}

template <class R>
hipError_t rk_typed(gbr_grid_s *g, int stage, const double *dt, const double *Qn, double *Q, const R *res)
{
    const double *A = kRkA, *B = kRkB;
    dim3 grid(unsigned((g->ncell + kBlock - 1) / kBlock));
    const double *jac = g->metrics + (long)GBR_SLOT_CELL_J * g->ncell;
    const double *ijt = g->metrics + (long)GBR_SLOT_CELL_INVJT * g->ncell;
    Timed timed(g, GBR_K_RK_STAGE);
    const Dims dm = dims_of(g);
    if (g->nvar == 5)
        hipLaunchKernelGGL((k_rk_stage<5, R>), grid, dim3(kBlock), 0, g->stream, dm, g->ncell, A[stage], B[stage],
                           dt, Qn, Q, res, jac, ijt);
    else
        hipLaunchKernelGGL((k_rk_stage<4, R>), grid, dim3(kBlock), 0, g->stream, dm, g->ncell, A[stage], B[stage],
                           dt, Qn, Q, res, jac, ijt);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_rhs(gbr_grid_s *g, const double *Q, void *res)
{
    if (g->cfg.precision == GBR_FP32_BULK) return rhs_typed<float>(g, Q, static_cast<float *>(res));
    return rhs_typed<double>(g, Q, static_cast<double *>(res));
}

hipError_t launch_diagnostics(gbr_grid_s *g, const double *Q, double *fields, double *integrals)
{
    if (g->cfg.precision == GBR_FP32_BULK) return diag_typed<float>(g, Q, fields, integrals);
    return diag_typed<double>(g, Q, fields, integrals);
}

hipError_t launch_step_stage(gbr_grid_s *g, int stage, const double *dt, double *Q, double *S, bool prims_ready)
{
    if (g->cfg.precision == GBR_FP32_BULK) return step_stage_typed<float>(g, stage, dt, Q, S, prims_ready);
    return step_stage_typed<double>(g, stage, dt, Q, S, prims_ready);
}

hipError_t launch_rk_stage(gbr_grid_s *g, int stage, const double *dt, const double *Qn, double *Q,
                           const void *res)
{
    if (g->cfg.precision == GBR_FP32_BULK)
        return rk_typed<float>(g, stage, dt, Qn, Q, static_cast<const float *>(res));
    return rk_typed<double>(g, stage, dt, Qn, Q, static_cast<const double *>(res));
}

hipError_t launch_cfl_into(gbr_grid_s *g, const double *Q, double cfl, double *dt, double *partial)
{
    const Dims dm = dims_of(g);
    const Phys ph = phys_of(g);
    long want = (g->ncell + kBlock - 1) / kBlock;
    int blocks = int(want < kReducePartials ? want : kReducePartials);
    const bool visc = g->cfg.viscous != 0;
    if (g->cfg.ndim == 3) {
        if (visc)
            hipLaunchKernelGGL((k_cfl_partial<3, true>), dim3(blocks), dim3(kBlock), 0, g->stream, dm, ph, Q,
                               g->metrics, g->cfg.moving, partial);
        else
            hipLaunchKernelGGL((k_cfl_partial<3, false>), dim3(blocks), dim3(kBlock), 0, g->stream, dm, ph, Q,
                               g->metrics, g->cfg.moving, partial);
    } else {
        if (visc)
            hipLaunchKernelGGL((k_cfl_partial<2, true>), dim3(blocks), dim3(kBlock), 0, g->stream, dm, ph, Q,
                               g->metrics, g->cfg.moving, partial);
        else
            hipLaunchKernelGGL((k_cfl_partial<2, false>), dim3(blocks), dim3(kBlock), 0, g->stream, dm, ph, Q,
                               g->metrics, g->cfg.moving, partial);
    }
    hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(1024), 0, g->stream, partial, blocks, cfl, dt);
    return hipGetLastError();
}

hipError_t launch_cfl(gbr_grid_s *g, const double *Q, double cfl, double *dt)
{
    Timed timed(g, GBR_K_CFL);
    return launch_cfl_into(g, Q, cfl, dt, g->partial);
}

namespace {
template <class R>
hipError_t cfl_prims_typed(gbr_grid_s *g, const double *Q, double cfl, double *dt)
{
    RhsArgs<R> a = make_args<R>(g, Q, nullptr);  // a.prim: the first stage's buffer
    long want = (g->ncell + kBlock - 1) / kBlock;
    int blocks = int(want < kReducePartials ? want : kReducePartials);
    const int mv = g->cfg.moving;
    Timed timed(g, GBR_K_CFL);
    if (g->cfg.ndim == 3) {
        if (g->cfg.viscous)
            hipLaunchKernelGGL((k_prims_cfl<3, true, R>), dim3(blocks), dim3(kBlock), 0, g->stream, a, mv, g->partial);
        else
            hipLaunchKernelGGL((k_prims_cfl<3, false, R>), dim3(blocks), dim3(kBlock), 0, g->stream, a, mv, g->partial);
    } else {
        if (g->cfg.viscous)
            hipLaunchKernelGGL((k_prims_cfl<2, true, R>), dim3(blocks), dim3(kBlock), 0, g->stream, a, mv, g->partial);
        else
            hipLaunchKernelGGL((k_prims_cfl<2, false, R>), dim3(blocks), dim3(kBlock), 0, g->stream, a, mv, g->partial);
    }
    hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(1024), 0, g->stream, g->partial, blocks, cfl, dt);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_cfl_prims(gbr_grid_s *g, const double *Q, double cfl, double *dt)
{
    if (g->cfg.precision == GBR_FP32_BULK) return cfl_prims_typed<float>(g, Q, cfl, dt);
    return cfl_prims_typed<double>(g, Q, cfl, dt);
}

hipError_t launch_fill(gbr_grid_s *g, double *p, long n, double value)
{
    unsigned blocks = unsigned((n + kBlock - 1) / kBlock);
    Timed timed(g, GBR_K_COPY);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(kBlock), 0, g->stream, p, n, value);
    return hipGetLastError();
}

hipError_t launch_copy(gbr_grid_s *g, double *dst, const double *src, long n)
{
    unsigned blocks = unsigned((n + kBlock - 1) / kBlock);
    Timed timed(g, GBR_K_COPY);
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(kBlock), 0, g->stream, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_step_time(gbr_grid_s *g, const double *dt, double *dt_out, double *t)
{
    Timed timed(g, GBR_K_COPY);
    hipLaunchKernelGGL(k_step_time, dim3(1), dim3(64), 0, g->stream, dt, dt_out, t);
    return hipGetLastError();
}

}  // namespace gbr

// hog_kernels.h -- gfx950 kernels of the ADER-WENO zone update (FP64 path).
//
// Data layout in HBM (all structure-of-arrays, x fastest, one array per
// (mode, variable) so consecutive lanes touch consecutive zones):
//   U[2]  padded state, ghost width 3 on every active axis (double buffer);
//   A     x-sweep output   [a][v]        over box AX = x:[-1,n] y:[-3,n+2] z:[-3,n+2]
//   B     y-sweep output   [(a,b)][v]    over box BY = x:[-1,n] y:[-1,n]   z:[-3,n+2]
//   W     spatial modes    [m][v]        over box R  = x:[-1,n] y:[-1,n]   z:[-1,n]
//                          (in 2D the y-sweep output is W)
//   FP    face-point states [d][side][pt][v] over R (predictor output)
//   F[d]  face fluxes [v] over the faces f+1/2, f in [-1, n-1] along d
// Boxes use interior zone numbering (0..n-1 are interior zones).
#pragma once
#include <type_traits>
#include <hip/hip_runtime.h>
#include <climits>
#include "hog_tables.h"
#include "hog_physics.h"

namespace hog {

constexpr int kGhostZones = 3;   // WENO radius 2 plus one face neighbour

struct Box {
    int lo[3];
    int n[3];
};
struct Pad {
    int np[3];
    int off[3];
    long long vs;   // stride between variables
};

__host__ __device__ inline long long box_size(const Box& b) { return (long long)b.n[0] * b.n[1] * b.n[2]; }
__device__ __forceinline__ void box_ijk(const Box& b, long long idx, int& i, int& j, int& k)
{
    i = (int)(idx % b.n[0]) + b.lo[0];
    long long r = idx / b.n[0];
    j = (int)(r % b.n[1]) + b.lo[1];
    k = (int)(r / b.n[1]) + b.lo[2];
}
__device__ __forceinline__ long long box_index(const Box& b, int i, int j, int k)
{
    return ((long long)(k - b.lo[2]) * b.n[1] + (j - b.lo[1])) * b.n[0] + (i - b.lo[0]);
}
__device__ __forceinline__ long long pad_index(const Pad& p, int i, int j, int k)
{
    return ((long long)(k + p.off[2]) * p.np[1] + (j + p.off[1])) * p.np[0] + (i + p.off[0]);
}

// Per-step scalars kept on the device so a run of steps needs no host round trip.
struct StepInfo {
    double dt;                      // time step of the current step
    double t;                       // time advanced since the last reset
    double t_end;                   // > 0: clip dt so that t does not pass t_end
    double lam[3];                  // dt / dx_d
    unsigned long long smax_bits;   // bits of max_zones sum_d (|u_d| + c) / dx_d (>= 0)
    unsigned long long bad;         // first non-physical zone, ULLONG_MAX if none
    unsigned long long fallback;    // predictor zones that used the positivity fallback
    unsigned long long nstep;       // steps begun since the last arm (k_arm), not counting halted ones
    int sticky;                     // 1 inside a device-side run of steps: a non-physical state halts it
    int halted;                     // 1: a step of this run produced a non-physical state; later steps
                                    //    of the run write no new state
    double pad_[5];
};

// ------------------------------------------------------------------------
// Step bookkeeping
// ------------------------------------------------------------------------
__global__ void k_begin_step(StepInfo* info, double dt_user, double cfl, double h0, double h1, double h2)
{
    if (info->sticky && info->bad != ULLONG_MAX) {   // keep the first failure and the state before it
        info->halted = 1;
        return;
    }
    info->nstep += 1;
    double dt = dt_user;
    if (!(dt > 0.0)) dt = cfl / __longlong_as_double((long long)info->smax_bits);
    if (info->t_end > 0.0) {
        double rem = info->t_end - info->t;
        if (dt > rem) dt = rem > 0.0 ? rem : 0.0;
    }
    info->dt = dt;
    info->lam[0] = dt / h0;
    info->lam[1] = dt / h1;
    info->lam[2] = dt / h2;
    info->t += dt;
    info->smax_bits = 0ull;
    info->bad = ULLONG_MAX;
    info->fallback = 0ull;
}

__global__ void k_reset(StepInfo* info, double t_end, int reset_time)
{
    if (reset_time) {
        info->t = 0.0;
        info->t_end = t_end;
        info->nstep = 0ull;
        info->sticky = 0;
        info->halted = 0;
    }
    info->smax_bits = 0ull;
    info->bad = ULLONG_MAX;
}

// Start (sticky = 1) or end (sticky = 0) a device-side run of steps.
__global__ void k_arm(StepInfo* info, int sticky)
{
    info->sticky = sticky;
    info->halted = 0;
    info->nstep = 0ull;
}

// ------------------------------------------------------------------------
// a1: ghost zones (periodic wrap or zero-gradient clamp per axis; fills
// edges and corners too).  One thread per padded zone; interior threads exit.
// ------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_ghost(double* __restrict__ U, Pad p, int n0, int n1, int n2,
                                               int bc0, int bc1, int bc2)
{
    constexpr int NV = D + 2;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)p.np[0] * p.np[1] * p.np[2];
    if (idx >= tot) return;
    int i = (int)(idx % p.np[0]) - p.off[0];
    long long r = idx / p.np[0];
    int j = (int)(r % p.np[1]) - p.off[1];
    int k = (int)(r / p.np[1]) - p.off[2];
    // an external axis (bc 2) keeps the ghost layers the caller supplied: a
    // zone inside the interior or on the supplied layers of every axis is left
    // alone; the others are filled along the remaining axes from the supplied
    // values (the source keeps the external coordinates)
    const bool k0 = (i >= 0 && i < n0) || bc0 == 2;
    const bool k1 = (j >= 0 && j < n1) || bc1 == 2;
    const bool k2 = (D == 3) ? ((k >= 0 && k < n2) || bc2 == 2) : true;
    if (k0 && k1 && k2) return;
    auto src = [](int x, int n, int bc) {
        if (bc == 2) return x;
        if (bc == 0) { x %= n; return x < 0 ? x + n : x; }
        return x < 0 ? 0 : (x >= n ? n - 1 : x);
    };
    const int si = src(i, n0, bc0), sj = src(j, n1, bc1), sk = (D == 3) ? src(k, n2, bc2) : 0;
    const long long s = pad_index(p, si, sj, sk);
#pragma unroll
    for (int v = 0; v < NV; ++v) U[v * p.vs + idx] = U[v * p.vs + s];
}

// ------------------------------------------------------------------------
// a7: CFL signal speed and non-physical check of a state (block max, then
// one 64-bit atomic max on the bit pattern: exact, hence deterministic).
// ------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void cfl_reduce(double s, bool ok, long long zone, StepInfo* info)
{
    __shared__ double red[4];
    if (!ok) atomicMin(&info->bad, (unsigned long long)zone);
    double m = ok ? s : 0.0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = red[0];
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q) b = fmax(b, red[q]);
        atomicMax(&info->smax_bits, (unsigned long long)__double_as_longlong(b));
    }
}

template <int D>
__device__ __forceinline__ double signal_speed(const double* u, double gamma, double ih0, double ih1, double ih2,
                                               bool& ok)
{
    const double rho = u[0];
    const double ir = 1.0 / rho;
    double ke = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) ke += u[1 + d] * u[1 + d];
    const double p = (gamma - 1.0) * (u[D + 1] - 0.5 * ke * ir);
    ok = rho > 0.0 && p > 0.0 && isfinite(rho) && isfinite(p);
    const double c = sqrt(gamma * p * ir);
    const double ih[3] = {ih0, ih1, ih2};
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) s += (fabs(u[1 + d] * ir) + c) * ih[d];
    return s;
}

template <int D>
__global__ __launch_bounds__(256) void k_cfl(const double* __restrict__ U, Pad p, Box I, StepInfo* info,
                                             double gamma, double ih0, double ih1, double ih2)
{
    constexpr int NV = D + 2;
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    bool ok = true;
    if (z < box_size(I)) {
        int i, j, k;
        box_ijk(I, z, i, j, k);
        const long long pi = pad_index(p, i, j, k);
        double u[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = U[v * p.vs + pi];
        s = signal_speed<D>(u, gamma, ih0, ih1, ih2, ok);
    }
    cfl_reduce<D>(s, ok, z, info);
}

// ------------------------------------------------------------------------
// a2: WENO reconstruction by successive 1D sweeps x -> y -> z.
// ------------------------------------------------------------------------
// Reconstruction of one 5-zone line in the arithmetic of the path: FP64, or
// the mixed path's FP32 coefficients with FP64 weights.
template <int P, typename T>
__device__ __forceinline__ void weno_line(const double* line, T* c, const WenoArgs& wa)
{
    if constexpr (sizeof(T) == 8) weno1d<P>(line, c, wa);
    else weno1d_mixed<P>(line, c, wa);
}

// Weights for the 1D applications centred at zone (i,j,k): linear when the
// learned gate marked that interior zone smooth.
__device__ __forceinline__ WenoArgs gated(const WenoArgs& wa, const unsigned char* __restrict__ gate, const Box& I,
                                          int i, int j, int k)
{
    WenoArgs w = wa;
    if (gate && i >= 0 && i < I.n[0] && j >= 0 && j < I.n[1] && k >= 0 && k < I.n[2] &&
        gate[((long long)k * I.n[1] + j) * I.n[0] + i])
        w.linear = 1;
    return w;
}

template <int D, int P, typename T>
__global__ __launch_bounds__(256) void k_recon_x(const double* __restrict__ U, Pad p, Box AX,
                                                 T* __restrict__ A, WenoArgs wa0,
                                                 const unsigned char* __restrict__ gate, Box I)
{
    constexpr int NV = D + 2;
    const long long nA = box_size(AX);
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= nA) return;
    int i, j, k;
    box_ijk(AX, z, i, j, k);
    const WenoArgs wa = gated(wa0, gate, I, i, j, k);
    const long long base = pad_index(p, i, j, k);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double line[5];
        T c[P + 1];
#pragma unroll
        for (int o = 0; o < 5; ++o) line[o] = U[v * p.vs + base + (o - 2)];
        weno_line<P, T>(line, c, wa);
        A[(0 * NV + v) * nA + z] = (T)line[2];
#pragma unroll
        for (int a = 1; a <= P; ++a) A[(a * NV + v) * nA + z] = c[a];
    }
}

// The y and z sweeps march along their axis: one thread per (line of zones
// along the axis, chunk of kRecChunk zones of that line, input mode,
// variable).  The thread keeps the five values of its stencil in registers,
// so each input value is read once (plus a four-value halo per chunk), and
// consecutive threads take consecutive x, so every load and store coalesces.
constexpr int kRecChunk = 32;

// Calls f(std::integral_constant<int, I>) for I = B .. E-1 (compile-time loop).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// March one line: input values at src[c0 + (o - 2) * stride], outputs for
// zones c0 .. c0 + (len - 1) * stride of the input box; the output index of
// the first zone is z0, advancing by zstride.  Writes the centre value to
// out0 and the WENO coefficients 1..NC to outc[0..NC-1] (NC may be 0).
template <int P, int NC, typename T, typename G>
__device__ __forceinline__ void march_line(const T* __restrict__ src, long long c0, long long stride, int len,
                                           T* __restrict__ out0, T* const* outc, long long z0, long long zstride,
                                           const WenoArgs& wa0, G&& gate_at)
{
    double w[5];
#pragma unroll
    for (int o = 0; o < 5; ++o) w[o] = (double)src[c0 + (o - 2) * stride];
    // the gate flag of the next zone is loaded with the next stencil value, so
    // the two loads of a step share one round trip
    bool gnext = NC >= 1 && gate_at(0);
    long long zi = z0;
    for (int s = 0; s < len; ++s) {
        out0[zi] = (T)w[2];
        const bool gcur = gnext;
        if constexpr (NC >= 1) {
            WenoArgs wa = wa0;
            if (gcur) wa.linear = 1;
            T c[P + 1];
            weno_line<P, T>(w, c, wa);
#pragma unroll
            for (int q = 1; q <= NC; ++q) outc[q - 1][zi] = c[q];
        }
        if (s + 1 < len) {
#pragma unroll
            for (int o = 0; o < 4; ++o) w[o] = w[o + 1];
            w[4] = (double)src[c0 + (long long)(s + 3) * stride];
            if constexpr (NC >= 1) gnext = gate_at(s + 1);
        }
        zi += zstride;
    }
}

// y sweep: A over AX (x-sweep output, P+1 modes) -> B over BY ((a, b) pairs).
template <int D, int P, typename T>
__global__ __launch_bounds__(256) void k_recon_y(const T* __restrict__ A, Box AX, Box BY,
                                                 T* __restrict__ B, WenoArgs wa0,
                                                 const unsigned char* __restrict__ gate, Box I)
{
    constexpr int NV = D + 2;
    constexpr Pairs<P> PR{};
    const long long nA = box_size(AX), nB = box_size(BY);
    const int nx = BY.n[0], nz = BY.n[2], nch = (BY.n[1] + kRecChunk - 1) / kRecChunk;
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)nx * nz * nch * (P + 1) * NV) return;
    const int ix = (int)(t % nx); t /= nx;
    const int kz = (int)(t % nz); t /= nz;
    const int ch = (int)(t % nch); t /= nch;
    const int v = (int)(t % NV), a = (int)(t / NV);
    const int i = BY.lo[0] + ix, k = BY.lo[2] + kz, j0 = BY.lo[1] + ch * kRecChunk;
    const int len = min(kRecChunk, BY.lo[1] + BY.n[1] - j0);
    const long long c0 = box_index(AX, i, j0, k), z0 = box_index(BY, i, j0, k);
    auto gate_at = [&](int s) {
        const int j = j0 + s;
        return gate && i >= 0 && i < I.n[0] && j >= 0 && j < I.n[1] && k >= 0 && k < I.n[2] &&
               gate[((long long)k * I.n[1] + j) * I.n[0] + i];
    };
    const T* src = A + (long long)(a * NV + v) * nA;
    // one branch per input mode a: the number of WENO outputs is compile-time
    static_for<0, P + 1>([&](auto ac) {
        constexpr int a2 = decltype(ac)::value;
        if (a != a2) return;
        T* outc[P];
#pragma unroll
        for (int b = 1; b <= P - a2; ++b) outc[b - 1] = B + (long long)(PR.at[a2][b] * NV + v) * nB;
        march_line<P, P - a2, T>(src, c0, AX.n[0], len, B + (long long)(PR.at[a2][0] * NV + v) * nB, outc, z0,
                                 BY.n[0], wa0, gate_at);
    });
}

// z sweep (3D): B over BY -> W over R (spatial modes (a, b, c)).
template <int P, typename T>
__global__ __launch_bounds__(256) void k_recon_z(const T* __restrict__ B, Box BY, Box R,
                                                 T* __restrict__ W, WenoArgs wa0,
                                                 const unsigned char* __restrict__ gate, Box I)
{
    constexpr int NV = 5;
    constexpr int NPAIR = (P + 1) * (P + 2) / 2;
    constexpr Modes<3, P> M{};
    constexpr Pairs<P> PR{};
    const long long nB = box_size(BY), nR = box_size(R);
    const int nx = R.n[0], ny = R.n[1], nch = (R.n[2] + kRecChunk - 1) / kRecChunk;
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)nx * ny * nch * NPAIR * NV) return;
    const int ix = (int)(t % nx); t /= nx;
    const int jy = (int)(t % ny); t /= ny;
    const int ch = (int)(t % nch); t /= nch;
    const int v = (int)(t % NV), pi = (int)(t / NV);
    const int i = R.lo[0] + ix, j = R.lo[1] + jy, k0 = R.lo[2] + ch * kRecChunk;
    const int len = min(kRecChunk, R.lo[2] + R.n[2] - k0);
    const long long c0 = box_index(BY, i, j, k0), z0 = box_index(R, i, j, k0);
    const long long sz = (long long)BY.n[0] * BY.n[1], zs = (long long)R.n[0] * R.n[1];
    auto gate_at = [&](int s) {
        const int k = k0 + s;
        return gate && i >= 0 && i < I.n[0] && j >= 0 && j < I.n[1] && k >= 0 && k < I.n[2] &&
               gate[((long long)k * I.n[1] + j) * I.n[0] + i];
    };
    // one branch per input pair (a, b): the number of WENO outputs is compile-time
    static_for<0, P + 1>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        static_for<0, P + 1 - b>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            if (pi != PR.at[a][b]) return;
            T* outc[P];
#pragma unroll
            for (int cc = 1; cc <= P - a - b; ++cc) outc[cc - 1] = W + (long long)(M.at[a][b][cc][0] * NV + v) * nR;
            march_line<P, P - a - b, T>(B + (long long)(pi * NV + v) * nB, c0, sz, len,
                                        W + (long long)(M.at[a][b][0][0] * NV + v) * nR, outc, z0, zs, wa0, gate_at);
        });
    });
}

// ------------------------------------------------------------------------
// a4: ADER predictor.  One wavefront per zone group.
// Node phase: lane = (zone slot, spatial Gauss node; in 3D the node's z index
// is shifted per lane group so that the row stores below hit distinct LDS
// banks); each lane keeps the time-independent part of q at its node in
// registers, evaluates the time modes from LDS (wavefront-uniform values,
// read in batches), forms the physical fluxes at every time node and
// contracts them against the shifted-Legendre time basis.
// Projection phase: the contracted fluxes of the flux time modes e <= P - 2
// go to LDS as one row per (zone, e, axis d, variable), with the nodes of the
// row stored so that axis d is the fastest one.  A lane (2D), a lane pair
// (3D) or, in the first iteration of the FP64 fourth-order instance, a lane
// quad owns a row and projects it in registers with axis d contracted first,
// keeping only the coefficients the update uses (degree >= 1 along d); it
// truncates them to total space-time degree P and applies the derivative
// along d.  The top
// flux time mode e = P - 1 only reaches the zone-constant spatial modes (its
// degree-1 coefficients along each axis), so the node phase folds its axes
// into one weighted node value per variable and the projection phase sums
// that row in fixed chunks.
// Assembly phase: lanes own new-mode targets and add the time-integral
// combination of the differentiated coefficients.
// After the last iteration the face-point states for the Riemann solver are
// evaluated from the final modes.  Blocks are mapped to zone groups so that
// the blocks one XCD runs (every 8th block) take contiguous zones and share
// their L2 cache lines.
// ------------------------------------------------------------------------
template <int D, int P>
struct PredShape {
    static constexpr int NV = D + 2;
    static constexpr int N1 = P + 1;
    static constexpr int NS = ipow_c(N1, D);         // spatial nodes per zone
    static constexpr int ZPW = 64 / NS;              // zones per wavefront
    static constexpr int MS = Modes<D, P>::NS;
    static constexpr int MST = Modes<D, P>::NST;
    static constexpr int MT = MST - MS;              // modes with e >= 1
    static constexpr int ME1 = binom(P - 1 + D, D);  // modes with e == 1
    static constexpr int NE = P;                     // flux time modes feeding a derivative
    static constexpr int NFULL = (NE - 1) * D * NV;  // projected rows per zone (e <= P - 2)
    static constexpr int NROWZ = NFULL + NV;         // + one folded row per variable (e = P - 1)
    static constexpr int RS = NS + 2;                // row stride (elements), padded against bank conflicts
    static constexpr int NG = binom(P - 1 + D, D);   // differentiated coefficients per row
    static constexpr int CH = 8;                     // chunk of a folded row summed by one lane
    static constexpr int NCH = (NS + CH - 1) / CH;
    static constexpr int NPT = 1 << D;               // Gauss points per face (tangential x time)
    static constexpr int NFPZ = D * 2 * NPT;         // face points per zone
    static constexpr int NTGT = ZPW * MT * NV;       // new-mode targets per wavefront
    static constexpr int TPL = (NTGT + 63) / 64;     // targets per lane
};

// Compact index of a differentiated coefficient (lo, o1, o2) with
// lo + o1 + o2 <= P - 1 (o2 = 0 in 2D): lo is the degree along the derivative
// axis, o1 and o2 the degrees along the other axes in increasing axis order.
template <int D, int P>
struct GIdx {
    int at[P][P][P];
    constexpr GIdx() : at{}
    {
        int n = 0;
        for (int o2 = 0; o2 < P; ++o2)
            for (int o1 = 0; o1 < P; ++o1)
                for (int lo = 0; lo < P; ++lo) {
                    const bool ok = lo + o1 + o2 <= P - 1 && (D == 3 || o2 == 0);
                    at[lo][o1][o2] = ok ? n++ : -1;
                }
    }
};

constexpr int kXcds = 8;   // MI355X: workgroups are dispatched round-robin over 8 XCDs

// Block -> group index such that the blocks of one XCD cover a contiguous range.
__device__ __forceinline__ int xcd_group(int b, int ngroups)
{
    const int per = (ngroups + kXcds - 1) / kXcds;
    return (b % kXcds) * per + b / kXcds;
}
// End (exclusive) of the group range of the XCD that block b runs on.
__device__ __forceinline__ int xcd_group_end(int b, int ngroups)
{
    const int per = (ngroups + kXcds - 1) / kXcds;
    return min(ngroups, (b % kXcds + 1) * per);
}
constexpr int kPrefetchAhead = 256;   // about the wavefronts one XCD keeps resident

inline unsigned xcd_blocks(long long ngroups)
{
    const long long per = (ngroups + kXcds - 1) / kXcds;
    return (unsigned)(per * kXcds);
}

// One new-mode target held by a lane: where its value goes in the mode
// buffer, where its differentiated coefficients sit in the rows of the
// e = 0 flux time mode (one per axis), where the folded row of its variable
// starts, its time degree and whether its spatial degree is zero.
template <int D>
struct Target {
    int valid, soff, off[D], top, te, zero;
};

// Constants of the predictor lanes, built at compile time and read from
// constant memory at kernel start.
// NodeRows: for each Gauss node index i along an axis, the monic Legendre
// basis at x_i followed by the projection weights proj[0][i] and proj[1][i]
// (a few distinct rows shared by all lanes, so the loads coalesce).
template <int P>
struct NodeRows {
    double r[P + 1][P + 3];
    constexpr NodeRows() : r{}
    {
        const Rules<P> RL{};
        for (int i = 0; i <= P; ++i) {
            for (int a = 0; a <= P; ++a) r[i][a] = RL.px[a][i];
            r[i][P + 1] = RL.proj[0][i];
            r[i][P + 2] = RL.proj[1][i];
        }
    }
};

template <int P>
__constant__ NodeRows<P> kNodeRows = NodeRows<P>();

// TargetTable: the new-mode targets of each lane, three packed words per
// target: (offset for axis 0) | (offset for axis 1) << 16, (offset for axis 2)
// | (folded row) << 16, (mode-buffer index) | te << 16 | zero << 20 | valid << 21.
template <int D, int P>
struct TargetTable {
    static constexpr int TPL = PredShape<D, P>::TPL;
    int t[64][TPL][3];
    constexpr TargetTable() : t{}
    {
        using S = PredShape<D, P>;
        constexpr int NV = S::NV, MS = S::MS, MST = S::MST, MT = S::MT;
        const Modes<D, P> M{};
        const GIdx<D, P> GI{};
        for (int lane = 0; lane < 64; ++lane)
            for (int k = 0; k < TPL; ++k) {
                const int g = lane + 64 * k;
                const int valid = g < S::NTGT;
                const int gg = valid ? g : 0;
                const int z = gg / (MT * NV), rem = gg % (MT * NV), mt = rem / NV, v = rem % NV;
                const int a = M.a[MS + mt], b = M.b[MS + mt], c = M.c[MS + mt];
                const int base = z * S::NROWZ * S::RS;
                const int off0 = base + v * S::RS + GI.at[a][b][c];
                const int off1 = base + (NV + v) * S::RS + GI.at[b][a][c];
                const int off2 = (D == 3) ? base + (2 * NV + v) * S::RS + GI.at[c][a][b] : 0;
                const int top = base + (S::NFULL + v) * S::RS;
                const int soff = (z * MST + MS + mt) * NV + v;
                t[lane][k][0] = off0 | (off1 << 16);
                t[lane][k][1] = off2 | (top << 16);
                t[lane][k][2] = soff | (M.e[MS + mt] << 16) | ((a + b + c == 0) << 20) | (valid << 21);
            }
    }
    static_assert(PredShape<D, P>::ZPW * PredShape<D, P>::NROWZ * PredShape<D, P>::RS < (1 << 15),
                  "row offsets fit 16 bits");
};

template <int D, int P>
__constant__ TargetTable<D, P> kTargetTable = TargetTable<D, P>();

// L2 projection weight proj[a][i] for a compile-time a and a lane-varying i.
template <int P>
__device__ __forceinline__ double proj_at(int a, int i)
{
    constexpr Rules<P> RL{};
    double v = 0.0;
#pragma unroll
    for (int k = 0; k <= P; ++k)
        if (i == k) v = RL.proj[a][k];
    return v;
}

// One projected row.  Input: node values at row[h + N1 * (o1n + N1 * o2n)],
// h the node index along the derivative axis.  Output, for every
// (lo, o1, o2) with lo + o1 + o2 <= P - 1, written to row[GIdx(lo, o1, o2)]:
//   g = sum_{hi > lo, hi + o1 + o2 <= emax} D[hi][lo] c(hi, o1, o2),
// c the Gauss L2-projection coefficients in the monic Legendre basis.  The
// bound emax = P - e truncates the flux to total space-time degree P.
template <int D, int P, typename T>
__device__ __forceinline__ void project_row(T* row, int emax)
{
    constexpr int N1 = P + 1;
    constexpr int NO2 = (D == 3) ? N1 : 1;
    constexpr Rules<P> RL{};
    constexpr GIdx<D, P> GI{};
    T c[N1][N1][N1];          // [hi][o1][o2], used for hi >= 1, hi + o1 + o2 <= P
#pragma unroll
    for (int p2 = 0; p2 < NO2; ++p2) {
        T x[N1][N1];          // [o1 node][h]
#pragma unroll
        for (int o = 0; o < N1; ++o)
#pragma unroll
            for (int h = 0; h < N1; ++h) x[o][h] = row[(p2 * N1 + o) * N1 + h];
        T t1[N1][N1];         // [o1 node][hi]
#pragma unroll
        for (int o = 0; o < N1; ++o)
#pragma unroll
            for (int hi = 1; hi <= P; ++hi) {
                T s = T(0);
#pragma unroll
                for (int h = 0; h < N1; ++h)
                    if (RL.proj[hi][h] != 0.0) s += T(RL.proj[hi][h]) * x[o][h];
                t1[o][hi] = s;
            }
#pragma unroll
        for (int hi = 1; hi <= P; ++hi)
#pragma unroll
            for (int o1 = 0; hi + o1 <= P; ++o1) {
                T s = T(0);
#pragma unroll
                for (int o = 0; o < N1; ++o)
                    if (RL.proj[o1][o] != 0.0) s += T(RL.proj[o1][o]) * t1[o][hi];
                if constexpr (D == 3) {
#pragma unroll
                    for (int o2 = 0; hi + o1 + o2 <= P; ++o2) {
                        const T w = T(RL.proj[o2][p2]);
                        if (p2 == 0) c[hi][o1][o2] = w * s;
                        else c[hi][o1][o2] += w * s;
                    }
                } else {
                    c[hi][o1][0] = s;
                }
            }
    }
#pragma unroll
    for (int hi = 1; hi <= P; ++hi)
#pragma unroll
        for (int o1 = 0; hi + o1 <= P; ++o1)
#pragma unroll
            for (int o2 = 0; o2 < NO2 && hi + o1 + o2 <= P; ++o2)
                if (hi + o1 + o2 > emax) c[hi][o1][o2] = T(0);
#pragma unroll
    for (int o2 = 0; o2 < NO2 && o2 <= P - 1; ++o2)
#pragma unroll
        for (int o1 = 0; o1 + o2 <= P - 1; ++o1)
#pragma unroll
            for (int lo = 0; lo + o1 + o2 <= P - 1; ++lo) {
                T s = T(0);
#pragma unroll
                for (int hi = lo + 1; hi + o1 + o2 <= P; ++hi)
                    if (RL.D[hi][lo] != 0.0) s += T(RL.D[hi][lo]) * c[hi][o1][o2];
                row[GI.at[lo][o1][o2]] = s;
            }
}

// Value held by the other lane of an even/odd lane pair (DPP quad_perm 1,0,3,2).
__device__ __forceinline__ double pair_swap(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0xB1, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0xB1, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float pair_swap(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, true));
}

// out[a] = sum over the Gauss nodes h of proj[a][h] v[h] for a0 <= a <= a1.
// The nodes are symmetric about 0 and the monic Legendre basis has the parity
// of its degree, so proj[a][N1-1-h] = (-1)^a proj[a][h]: the sums and
// differences of the node pairs are formed once and shared by all modes (a
// four-node line: 4 additions + 2 multiply-adds per mode instead of 4).
template <int P, typename T>
__device__ __forceinline__ void project_line(const T (&v)[P + 1], T (&out)[P + 1], int a0, int a1)
{
    constexpr int N1 = P + 1, H = N1 / 2;
    constexpr Rules<P> RL{};
    T sp[H > 0 ? H : 1], sm[H > 0 ? H : 1];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        sp[h] = v[h] + v[N1 - 1 - h];
        sm[h] = v[h] - v[N1 - 1 - h];
    }
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        if (a < a0 || a > a1) continue;
        T s = (N1 % 2 == 1 && a % 2 == 0) ? T(RL.proj[a][H]) * v[H] : T(0);
#pragma unroll
        for (int h = 0; h < H; ++h) s += T(RL.proj[a][h]) * (a % 2 ? sm[h] : sp[h]);
        out[a] = s;
    }
}

// project_row in 3D by a lane pair: lane `half` of the pair takes the node
// planes half, half + 2, ... along the second other axis, the pair adds its
// two partial sums (the same two numbers on both lanes, so both hold the same
// result) and both lanes write the same differentiated coefficients.
template <int P, typename T>
__device__ __forceinline__ void project_row_pair(T* row, int emax, int half)
{
    constexpr int N1 = P + 1;
    constexpr int NPL = (N1 + 1) / 2;   // node planes per lane
    constexpr Rules<P> RL{};
    constexpr GIdx<3, P> GI{};
    T c[N1][N1][N1];          // [hi][o1][o2], used for hi >= 1, hi + o1 + o2 <= P
#pragma unroll
    for (int t = 0; t < NPL; ++t) {
        const int p2 = 2 * t + half;
        const bool live = (N1 % 2 == 0) || 2 * t + 1 < N1 || half == 0;
        T w[N1];              // projection weights of this lane's plane
#pragma unroll
        for (int o2 = 0; o2 <= P; ++o2) {
            const T w0 = T(RL.proj[o2][2 * t]);
            const T w1 = (2 * t + 1 < N1) ? T(RL.proj[o2][2 * t + 1]) : T(0);
            w[o2] = half ? w1 : w0;
        }
        T x[N1][N1];          // [o1 node][h]
#pragma unroll
        for (int o = 0; o < N1; ++o)
#pragma unroll
            for (int h = 0; h < N1; ++h) x[o][h] = live ? row[(p2 * N1 + o) * N1 + h] : T(0);
        T t1[N1][N1];         // [o1 node][hi]
        T s1[N1][N1];         // [hi][o1]
        if constexpr (sizeof(T) == 8) {
#pragma unroll
            for (int o = 0; o < N1; ++o) project_line<P, T>(x[o], t1[o], 1, P);
#pragma unroll
            for (int hi = 1; hi <= P; ++hi) {
                T col[N1];
#pragma unroll
                for (int o = 0; o < N1; ++o) col[o] = t1[o][hi];
                project_line<P, T>(col, s1[hi], 0, P - hi);
            }
        } else {
            // FP32: the plain node sums (the node-pair form measured no faster
            // in this instance)
#pragma unroll
            for (int o = 0; o < N1; ++o)
#pragma unroll
                for (int hi = 1; hi <= P; ++hi) {
                    T s = T(0);
#pragma unroll
                    for (int h = 0; h < N1; ++h)
                        if (RL.proj[hi][h] != 0.0) s += T(RL.proj[hi][h]) * x[o][h];
                    t1[o][hi] = s;
                }
#pragma unroll
            for (int hi = 1; hi <= P; ++hi)
#pragma unroll
                for (int o1 = 0; hi + o1 <= P; ++o1) {
                    T s = T(0);
#pragma unroll
                    for (int o = 0; o < N1; ++o)
                        if (RL.proj[o1][o] != 0.0) s += T(RL.proj[o1][o]) * t1[o][hi];
                    s1[hi][o1] = s;
                }
        }
#pragma unroll
        for (int hi = 1; hi <= P; ++hi)
#pragma unroll
            for (int o1 = 0; hi + o1 <= P; ++o1)
#pragma unroll
                for (int o2 = 0; hi + o1 + o2 <= P; ++o2) {
                    if (t == 0) c[hi][o1][o2] = w[o2] * s1[hi][o1];
                    else c[hi][o1][o2] += w[o2] * s1[hi][o1];
                }
    }
#pragma unroll
    for (int hi = 1; hi <= P; ++hi)
#pragma unroll
        for (int o1 = 0; hi + o1 <= P; ++o1)
#pragma unroll
            for (int o2 = 0; hi + o1 + o2 <= P; ++o2) {
                const T own = c[hi][o1][o2];
                c[hi][o1][o2] = own + pair_swap(own);
                if (hi + o1 + o2 > emax) c[hi][o1][o2] = T(0);
            }
#pragma unroll
    for (int o2 = 0; o2 <= P - 1; ++o2)
#pragma unroll
        for (int o1 = 0; o1 + o2 <= P - 1; ++o1)
#pragma unroll
            for (int lo = 0; lo + o1 + o2 <= P - 1; ++lo) {
                T s = T(0);
#pragma unroll
                for (int hi = lo + 1; hi + o1 + o2 <= P; ++hi)
                    if (RL.D[hi][lo] != 0.0) s += T(RL.D[hi][lo]) * c[hi][o1][o2];
                row[GI.at[lo][o1][o2]] = s;
            }
}

// Value held by lane l ^ 2 within a lane quad (DPP quad_perm 2,3,0,1).
__device__ __forceinline__ double quad_swap2(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), 0x4E, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), 0x4E, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float quad_swap2(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x4E, 0xF, 0xF, true));
}

// project_row in 3D at fourth order by a lane quad: lane q of the quad takes
// node plane q along the second other axis; the four partial sums are added
// pairwise ((q0 + q1) + (q2 + q3), the same two numbers in each addition on
// every lane, so all four lanes hold the same result); the differentiated
// coefficients go to dst[GIdx(lo, o1, o2)] (all four lanes store the same values).
template <int P, typename T>
__device__ __forceinline__ void project_row_quad(const T* row, T* dst, int emax, int q)
{
    static_assert(P == 3, "one node plane per lane of the quad");
    constexpr int N1 = P + 1;
    constexpr Rules<P> RL{};
    constexpr GIdx<3, P> GI{};
    T w[N1];                  // projection weights of this lane's plane
#pragma unroll
    for (int o2 = 0; o2 <= P; ++o2) {
        T v = T(0);
#pragma unroll
        for (int k = 0; k < N1; ++k)
            if (q == k) v = T(RL.proj[o2][k]);
        w[o2] = v;
    }
    T x[N1][N1];              // [o1 node][h]
#pragma unroll
    for (int o = 0; o < N1; ++o)
#pragma unroll
        for (int h = 0; h < N1; ++h) x[o][h] = row[(q * N1 + o) * N1 + h];
    T t1[N1][N1];             // [o1 node][hi]
#pragma unroll
    for (int o = 0; o < N1; ++o) project_line<P, T>(x[o], t1[o], 1, P);
    T c[N1][N1][N1];          // [hi][o1][o2], used for hi >= 1, hi + o1 + o2 <= P
#pragma unroll
    for (int hi = 1; hi <= P; ++hi) {
        T col[N1], s1[N1];
#pragma unroll
        for (int o = 0; o < N1; ++o) col[o] = t1[o][hi];
        project_line<P, T>(col, s1, 0, P - hi);
#pragma unroll
        for (int o1 = 0; hi + o1 <= P; ++o1)
#pragma unroll
            for (int o2 = 0; hi + o1 + o2 <= P; ++o2) {
                T own = w[o2] * s1[o1];
                own = own + pair_swap(own);
                own = own + quad_swap2(own);
                c[hi][o1][o2] = (hi + o1 + o2 > emax) ? T(0) : own;
            }
    }
#pragma unroll
    for (int o2 = 0; o2 <= P - 1; ++o2)
#pragma unroll
        for (int o1 = 0; o1 + o2 <= P - 1; ++o1)
#pragma unroll
            for (int lo = 0; lo + o1 + o2 <= P - 1; ++lo) {
                T s = T(0);
#pragma unroll
                for (int hi = lo + 1; hi + o1 + o2 <= P; ++hi)
                    if (RL.D[hi][lo] != 0.0) s += T(RL.D[hi][lo]) * c[hi][o1][o2];
                dst[GI.at[lo][o1][o2]] = s;
            }
}

// For the modes m in [LO, HI) and the variables v: use(m, v, q[m NV + v]),
// with the wavefront-uniform LDS values read in batches of B, all reads of a
// batch issued before any of its uses (one LDS round trip per batch instead
// of a wait before nearly every use).
template <int NV, int LO, int HI, int B, typename T, typename F>
__device__ __forceinline__ void batched_modes(const T* q, F&& use)
{
    constexpr int N = (HI - LO) * NV;
#pragma unroll
    for (int b0 = 0; b0 < N; b0 += B) {
        T qv[B];
#pragma unroll
        for (int i = 0; i < B; ++i)
            if (b0 + i < N) qv[i] = q[LO * NV + b0 + i];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < B; ++i)
            if (b0 + i < N) use(LO + (b0 + i) / NV, (b0 + i) % NV, qv[i]);
    }
}

// Per-lane constants of the predictor: the monic Legendre basis at the lane's
// node along each axis, the node's position in the rows of each derivative
// axis, the node weight of the folded top flux time mode, and the new-mode
// targets the lane owns.  Two ways to obtain the same values: read from the
// compile-time tables (fewer VALU instructions: used by the FP64 instance,
// which runs at two wavefronts per SIMD) or computed in registers (used by the
// FP32 instance, measured faster at its four wavefronts per SIMD).
template <int D, int P, typename T>
struct LaneSetup {
    T px[P + 1], py[P + 1], pz[P + 1];
    int pos[D];
    T kap[D];
    Target<D> tg[PredShape<D, P>::TPL];
};

// Node of a lane: (ii, jj, kk) along x, y, z.  In 3D the z index is
// (ii + jj + g) mod (P+1) in lane group g of (P+1)^2 lanes, so that the lanes of
// a group hold distinct (ii, jj) and distinct (ii, kk) pairs: their stores
// into the rows of every derivative axis then fall into distinct LDS banks.
template <int D, int P>
__device__ __forceinline__ void node_coords(int node, int& ii, int& jj, int& kk)
{
    constexpr int N1 = P + 1;
    ii = node % N1;
    jj = (node / N1) % N1;
    kk = (D == 3) ? (ii + jj + node / (N1 * N1)) % N1 : 0;
}

template <int D, int P, typename T>
__device__ __forceinline__ void node_position(LaneSetup<D, P, T>& L, int node, int ii, int jj, int kk)
{
    constexpr int N1 = P + 1;
    L.pos[0] = ii + N1 * (jj + N1 * kk);
    if constexpr (D == 3) {
        L.pos[1] = jj + N1 * (ii + N1 * kk);
        L.pos[2] = kk + N1 * (ii + N1 * jj);
    } else {
        L.pos[1] = jj + N1 * ii;
    }
}

template <int D, int P, typename T>
__device__ __forceinline__ void lane_setup_tables(LaneSetup<D, P, T>& L, int lane, const T* lam)
{
    using S = PredShape<D, P>;
    constexpr Rules<P> RL{};
    const int node = lane % S::NS;
    int ii, jj, kk;
    node_coords<D, P>(node, ii, jj, kk);
    const double* nr[3] = {kNodeRows<P>.r[ii], kNodeRows<P>.r[jj], kNodeRows<P>.r[kk]};
    // the degree-0 basis function is 1 at every node: a literal, so that the
    // basis products of the modes constant along an axis cost no multiply
    L.px[0] = L.py[0] = L.pz[0] = T(1);
#pragma unroll
    for (int a = 1; a <= P; ++a) {
        L.px[a] = T(nr[0][a]);
        L.py[a] = T(nr[1][a]);
        L.pz[a] = (D == 3) ? T(nr[2][a]) : T(0);
    }
    node_position<D, P, T>(L, node, ii, jj, kk);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double k = RL.D[1][0];
#pragma unroll
        for (int ax = 0; ax < D; ++ax) k *= nr[ax][ax == d ? P + 2 : P + 1];
        L.kap[d] = lam[d] * T(k);
    }
#pragma unroll
    for (int r = 0; r < S::TPL; ++r) {
        const int w0 = kTargetTable<D, P>.t[lane][r][0], w1 = kTargetTable<D, P>.t[lane][r][1],
                  w2 = kTargetTable<D, P>.t[lane][r][2];
        L.tg[r].off[0] = w0 & 0xFFFF;
        L.tg[r].off[1] = w0 >> 16;
        if constexpr (D == 3) L.tg[r].off[2] = w1 & 0xFFFF;
        L.tg[r].top = w1 >> 16;
        L.tg[r].soff = w2 & 0xFFFF;
        L.tg[r].te = (w2 >> 16) & 0xF;
        L.tg[r].zero = (w2 >> 20) & 1;
        L.tg[r].valid = (w2 >> 21) & 1;
    }
}

template <int D, int P, typename T>
__device__ __forceinline__ void lane_setup_computed(LaneSetup<D, P, T>& L, int lane, const T* lam)
{
    using S = PredShape<D, P>;
    constexpr int N1 = P + 1, NV = S::NV, MS = S::MS, MST = S::MST, MT = S::MT, RS = S::RS;
    constexpr Rules<P> RL{};
    constexpr Modes<D, P> M{};
    constexpr GIdx<D, P> GI{};
    const int node = lane % S::NS;
    int ii, jj, kk;
    node_coords<D, P>(node, ii, jj, kk);
    const double xn = gl_node(N1, ii), yn = gl_node(N1, jj), zn = gl_node(N1, kk);
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        L.px[a] = T(mleg(a, xn));
        L.py[a] = T(mleg(a, yn));
        L.pz[a] = (D == 3) ? T(mleg(a, zn)) : T(a == 0 ? 1 : 0);
    }
    node_position<D, P, T>(L, node, ii, jj, kk);
    const int nd[3] = {ii, jj, kk};
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double k = RL.D[1][0];
#pragma unroll
        for (int ax = 0; ax < D; ++ax) k *= proj_at<P>(ax == d ? 1 : 0, nd[ax]);
        L.kap[d] = lam[d] * T(k);
    }
#pragma unroll
    for (int r = 0; r < S::TPL; ++r) {
        const int t = lane + 64 * r;
        L.tg[r].valid = t < S::NTGT;
        const int tt = L.tg[r].valid ? t : 0;
        const int z = tt / (MT * NV);
        const int rem = tt % (MT * NV), mt = rem / NV, v = rem % NV;
        int te = 0, zero = 0, g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
        for (int q = 0; q < MT; ++q)
            if (q == mt) {
                const int a = M.a[MS + q], b = M.b[MS + q], c = M.c[MS + q];
                te = M.e[MS + q];
                zero = (a + b + c == 0);
                g0 = GI.at[a][b][c];
                g1 = GI.at[b][a][c];
                g2 = (D == 3) ? GI.at[c][a][b] : 0;
            }
        L.tg[r].soff = (z * MST + MS + mt) * NV + v;
        const int base = z * S::NROWZ * RS;
        L.tg[r].off[0] = base + v * RS + g0;
        L.tg[r].off[1] = base + (NV + v) * RS + g1;
        if constexpr (D == 3) L.tg[r].off[2] = base + (2 * NV + v) * RS + g2;
        L.tg[r].top = base + (S::NFULL + v) * RS;
        L.tg[r].te = te;
        L.tg[r].zero = zero;
    }
}

// Occupancy: FP64 two wavefronts per SIMD (up to 256 VGPRs); FP32 four, the
// most its LDS rows allow, so its registers are bounded to 128.
template <int D, int P, typename T>
__global__ __launch_bounds__(64, sizeof(T) == 8 ? 2 : 4) void k_predict(const T* __restrict__ W, Box R,
                                                   StepInfo* __restrict__ info, double gamma, int positivity,
                                                   T* __restrict__ FP, T* __restrict__ Qout)
{
    using S = PredShape<D, P>;
    constexpr int NV = S::NV, N1 = S::N1, NS = S::NS, ZPW = S::ZPW, RS = S::RS;
    constexpr int MS = S::MS, MST = S::MST, NE = S::NE;
    constexpr int NFULL = S::NFULL, NROWZ = S::NROWZ, CH = S::CH, NCH = S::NCH;
    constexpr Modes<D, P> M{};
    constexpr Rules<P> RL{};

    __shared__ T sq[ZPW * MST * NV];
    __shared__ T sr[ZPW * NROWZ * RS];
    __shared__ int sbad[ZPW];

    const long long nR = box_size(R);
    const int ngroups = (int)((nR + ZPW - 1) / ZPW);
    const int grp = xcd_group(blockIdx.x, ngroups);
    if (grp >= ngroups) return;                       // whole wavefront, before any barrier
    const int lane = threadIdx.x;
    const long long zbase = (long long)grp * ZPW;
    const T gm1 = T(gamma - 1.0);
    const T lam[3] = {T(info->lam[0]), T(info->lam[1]), T(info->lam[2])};

    {
        // all loads first, then the stores, so the round trips overlap
        constexpr int NL = (ZPW * MST * NV + 63) / 64;
        T wv[NL];
#pragma unroll
        for (int r = 0; r < NL; ++r) {
            const int t = lane + 64 * r;
            const int z = t / (MST * NV), rm = t % (MST * NV), m = rm / NV, v = rm % NV;
            const long long zone = zbase + z;
            wv[r] = (t < ZPW * MST * NV && m < MS && zone < nR) ? W[(long long)(m * NV + v) * nR + zone] : T(0);
        }
#pragma unroll
        for (int r = 0; r < NL; ++r)
            if (lane + 64 * r < ZPW * MST * NV) sq[lane + 64 * r] = wv[r];
    }
    if (lane < ZPW) sbad[lane] = 0;

    const int zs = lane / NS;
    const int node = lane % NS;
    const bool active = zs < ZPW;
    LaneSetup<D, P, T> L;
    if constexpr (sizeof(T) == 8) lane_setup_tables<D, P, T>(L, lane, lam);
    else lane_setup_computed<D, P, T>(L, lane, lam);
    // L2 warm-up: each wavefront touches the spatial modes of the zone group
    // kPrefetchAhead groups further on, which a later wavefront of the same
    // XCD will load (the blocks of one XCD take consecutive groups); the
    // loaded word is only consumed after the Picard iterations, so nothing waits for it.
    unsigned pf = 0;
    if constexpr (sizeof(T) == 8) {
        asm volatile("" ::: "memory");
        const long long pz = (long long)min(grp + kPrefetchAhead, xcd_group_end(blockIdx.x, ngroups) - 1) * ZPW;
        pf = reinterpret_cast<const unsigned*>(W + (long long)(lane < MS * NV ? lane : 0) * nR + pz)[0];
    }
    const T(&px)[P + 1] = L.px;
    const T(&py)[P + 1] = L.py;
    const T(&pz)[P + 1] = L.pz;
    const int(&pos)[D] = L.pos;
    const T(&kap)[D] = L.kap;
    const Target<D>(&tg)[S::TPL] = L.tg;
    __syncthreads();

    // time-independent part of q at this lane's node (the reconstruction)
    T Q0[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Q0[v] = T(0);
    if (active) {
        batched_modes<NV, 0, MS, 50>(sq + zs * MST * NV, [&](int m, int v, T q) {
            Q0[v] += q * (px[M.a[m]] * py[M.b[m]] * pz[M.c[m]]);
        });
    }

    // the P iterations unrolled: each one specialised (first, degree 1, full)
    // and scheduled across its boundaries
#pragma unroll
    for (int it = 0; it < P; ++it) {
        const bool first = it == 0;            // first iterate is time-independent
        const int nfe = first ? 1 : NE - 1;    // projected flux time modes this iteration
        // ---- node phase
        if (active) {
            bool ok = true;
            T* rz = sr + zs * NROWZ * RS;       // row (e, d, v) at rz[((e*D + d)*NV + v)*RS], folded row v at rz[(NFULL + v)*RS]
            if (first) {
                T F[D][NV];
                ok = fluxes<D, T>(Q0, gm1, F);
#pragma unroll
                for (int d = 0; d < D; ++d)
#pragma unroll
                    for (int v = 0; v < NV; ++v) rz[(d * NV + v) * RS + pos[d]] = F[d][v];
            } else {
                // The iterate of iteration it has time degree it (the first one is
                // constant in time): in iteration 1 the modes of time degree >= 2
                // are exactly zero, and their reads are skipped (uniform branch).
                const bool deg1 = it == 1;
                T Qe[P][NV];                        // time modes e = 1..P at the node
#pragma unroll
                for (int e = 0; e < P; ++e)
#pragma unroll
                    for (int v = 0; v < NV; ++v) Qe[e][v] = T(0);
                // the modes are ordered by time degree: those of degree 1 first
                const T* qz = sq + zs * MST * NV;
                auto acc_mode = [&](int m, int v, T q) {
                    Qe[M.e[m] - 1][v] += q * (px[M.a[m]] * py[M.b[m]] * pz[M.c[m]]);
                };
                if (deg1) batched_modes<NV, MS, MS + S::ME1, 26>(qz, acc_mode);
                else batched_modes<NV, MS, MST, 26>(qz, acc_mode);
                T Racc[NE - 1][D][NV];
                T Rtop[NV];
#pragma unroll
                for (int e = 0; e < NE - 1; ++e)
#pragma unroll
                    for (int d = 0; d < D; ++d)
#pragma unroll
                        for (int v = 0; v < NV; ++v) Racc[e][d][v] = T(0);
#pragma unroll
                for (int v = 0; v < NV; ++v) Rtop[v] = T(0);
#pragma unroll
                for (int l = 0; l < N1; ++l) {
                    T U[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        // (in iteration 1 the higher time modes are zero, and the
                        // Horner sum reduces exactly to the degree-1 one)
                        T s = Qe[P - 1][v];
#pragma unroll
                        for (int e = P - 2; e >= 0; --e) s = s * T(RL.t[l]) + Qe[e][v];
                        U[v] = Q0[v] + s * T(RL.t[l]);
                    }
                    T F[D][NV];
                    ok = fluxes<D, T>(U, gm1, F) && ok;
#pragma unroll
                    for (int e = 0; e < NE - 1; ++e)
#pragma unroll
                        for (int d = 0; d < D; ++d)
#pragma unroll
                            for (int v = 0; v < NV; ++v) Racc[e][d][v] += T(RL.tproj[e][l]) * F[d][v];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        T s = kap[0] * F[0][v];
#pragma unroll
                        for (int d = 1; d < D; ++d) s += kap[d] * F[d][v];
                        Rtop[v] += T(RL.tproj[NE - 1][l]) * s;
                    }
                }
#pragma unroll
                for (int e = 0; e < NE - 1; ++e)
#pragma unroll
                    for (int d = 0; d < D; ++d)
#pragma unroll
                        for (int v = 0; v < NV; ++v) rz[((e * D + d) * NV + v) * RS + pos[d]] = Racc[e][d][v];
#pragma unroll
                for (int v = 0; v < NV; ++v) rz[(NFULL + v) * RS + node] = Rtop[v];
            }
            if (positivity && !ok) atomicOr(&sbad[zs], 1);
        }
        __syncthreads();
        // ---- projection phase: one lane (2D) or lane pair (3D) per row; chunk
        //      sums of the folded rows
        {
            const int nfz = nfe * D * NV;
            if constexpr (D == 3 && P == 3 && sizeof(T) == 8) {
                static_assert(ZPW == 1 && 2 * NFULL <= 64, "one lane pair per projected row");
                if (first) {
                    // 15 rows: one lane quad per row (FP64 only: in FP32 the extra
                    // registers cost a wavefront per SIMD)
                    const int r = lane >> 2;
                    if (r < D * NV) project_row_quad<P, T>(sr + r * RS, sr + r * RS, P, lane & 3);
                } else {
                    const int r = lane >> 1;
                    if (r < nfz) project_row_pair<P, T>(sr + r * RS, P - r / (D * NV), lane & 1);
                }
            } else if constexpr (D == 3) {
                static_assert(2 * ZPW * NFULL <= 64, "one lane pair per projected row");
                const int s = lane >> 1;
                if (s < ZPW * nfz) {
                    const int z = s / nfz, r = s % nfz;
                    project_row_pair<P, T>(sr + (z * NROWZ + r) * RS, P - r / (D * NV), lane & 1);
                }
            } else {
                for (int s = lane; s < ZPW * nfz; s += 64) {
                    const int z = s / nfz, r = s % nfz;
                    project_row<D, P, T>(sr + (z * NROWZ + r) * RS, P - r / (D * NV));
                }
            }
            if (!first) {
                for (int s = lane; s < ZPW * NV * NCH; s += 64) {
                    const int z = s / (NV * NCH), r = s % (NV * NCH), v = r / NCH, ch = r % NCH;
                    T* p = sr + (z * NROWZ + NFULL + v) * RS + ch * CH;
                    T acc = p[0];
                    if constexpr (NS % CH == 0) {
#pragma unroll
                        for (int i = 1; i < CH; ++i) acc += p[i];
                    } else {
#pragma unroll
                        for (int i = 1; i < CH; ++i)
                            if (ch * CH + i < NS) acc += p[i];
                    }
                    p[0] = acc;
                }
            }
        }
        __syncthreads();
        // ---- assembly: for target (a, b, c, te), variable v,
        //   q = -sum_e I[e][te] sum_d lam_d g_{e,d,v}(rotated (a, b, c))
        //       - I[P-1][te] [a = b = c = 0] (folded row sum of v)
        // (per target all LDS reads first, then the arithmetic; a lane
        // without a target reads row 0 and stores nothing)
#pragma unroll
        for (int r = 0; r < S::TPL; ++r) {
            const Target<D>& tq = tg[r];
            T gv[NE - 1][D], tv[NCH];
            int ob[D];
#pragma unroll
            for (int d = 0; d < D; ++d) ob[d] = tq.valid ? tq.off[d] : 0;
            const int otop = tq.valid ? tq.top : 0;
#pragma unroll
            for (int e = 0; e < NE - 1; ++e)
#pragma unroll
                for (int d = 0; d < D; ++d) gv[e][d] = sr[ob[d] + e * D * NV * RS];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) tv[ch] = sr[otop + ch * CH];
            __builtin_amdgcn_sched_barrier(0);
            T acc = T(0);
#pragma unroll
            for (int e = 0; e < NE - 1; ++e) {
                if (e >= nfe) continue;
                T ci = T(0);
#pragma unroll
                for (int et = 1; et <= P; ++et)
                    if (tq.te == et) ci = T(RL.I[e][et]);
                T sum = lam[0] * gv[e][0];
#pragma unroll
                for (int d = 1; d < D; ++d) sum += lam[d] * gv[e][d];
                acc += ci * sum;
            }
            if (!first) {
                T ct = T(0);
#pragma unroll
                for (int et = 1; et <= P; ++et)
                    if (tq.te == et && tq.zero) ct = T(RL.I[NE - 1][et]);
                T s = tv[0];
#pragma unroll
                for (int ch = 1; ch < NCH; ++ch) s += tv[ch];
                acc += ct * s;
            }
            if (tq.valid) sq[tq.soff] = -acc;
        }
        __syncthreads();
    }

    if constexpr (sizeof(T) == 8) asm volatile("" ::"v"(pf));   // long completed; consumed before the stores
    if (Qout) {
        for (int t = lane; t < ZPW * MST * NV; t += 64) {
            const int z = t / (MST * NV), r = t % (MST * NV);
            const long long zone = zbase + z;
            if (zone < nR) Qout[(long long)r * nR + zone] = sq[t];
        }
    }
    // face-point states: side 0 at xi_d = -1/2, side 1 at +1/2; point index
    // (time, first tangential axis[, second tangential axis]) with time slowest.
    // A zone with an inadmissible node or face state falls back to its mean.
    constexpr T g = T(0.28867513459481288225);
    constexpr int FPL = (ZPW * S::NFPZ + 63) / 64;    // face points per lane
    T Ufp[FPL][NV];
#pragma unroll
    for (int r = 0; r < FPL; ++r) {
        const int t = lane + 64 * r;
        if (t >= ZPW * S::NFPZ) continue;
        const int z = t / S::NFPZ, rr = t % S::NFPZ;
        const int d = rr / (2 * S::NPT), side = (rr / S::NPT) & 1, pt = rr % S::NPT;
        const int t1 = (d == 0) ? 1 : 0;          // first tangential axis
        int lt, a1, a2 = 0;
        if (D == 3) { lt = pt >> 2; a1 = (pt >> 1) & 1; a2 = pt & 1; }
        else { lt = pt >> 1; a1 = pt & 1; }
        const T xn = side ? T(0.5) : T(-0.5);
        const T x1 = a1 ? g : -g, x2 = a2 ? g : -g;
        // axis ax gets the normal coordinate, the first or the second tangential one
        const T cx = (d == 0) ? xn : x1;
        const T cy = (d == 1) ? xn : (t1 == 1 ? x1 : x2);
        const T cz = (D == 3) ? ((d == 2) ? xn : x2) : 0.0;
        const T tau = T(0.5) + (lt ? g : -g);
        T bx[P + 1], by[P + 1], bz[P + 1], bt[P + 1];
#pragma unroll
        for (int a = 0; a <= P; ++a) {
            bx[a] = T(mleg(a, (double)cx));
            by[a] = T(mleg(a, (double)cy));
            bz[a] = T(mleg(a, (double)cz));
        }
        bt[0] = T(1);
#pragma unroll
        for (int e = 1; e <= P; ++e) bt[e] = bt[e - 1] * tau;
#pragma unroll
        for (int v = 0; v < NV; ++v) Ufp[r][v] = T(0);
        batched_modes<NV, 0, MST, 50>(sq + z * MST * NV, [&](int m, int v, T q) {
            Ufp[r][v] += q * (bx[M.a[m]] * by[M.b[m]] * bz[M.c[m]] * bt[M.e[m]]);
        });
        if (positivity && !admissible<D, T>(Ufp[r], gm1)) atomicOr(&sbad[z], 1);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < FPL; ++r) {
        const int t = lane + 64 * r;
        if (t >= ZPW * S::NFPZ) continue;
        const int z = t / S::NFPZ, rr = t % S::NFPZ;
        const long long zone = zbase + z;
        if (zone >= nR) continue;
        const bool fb = sbad[z] != 0;
#pragma unroll
        for (int v = 0; v < NV; ++v)
            FP[((long long)rr * NV + v) * nR + zone] = fb ? sq[z * MST * NV + v] : Ufp[r][v];
    }
    if (positivity && lane == 0) {
        unsigned long long nb = 0;
        for (int z = 0; z < ZPW; ++z) nb += (sbad[z] != 0 && zbase + z < nR) ? 1ull : 0ull;
        if (nb) atomicAdd(&info->fallback, nb);
    }
}

// ------------------------------------------------------------------------
// a5: Riemann solver at the face Gauss points and the space-time average of
// the face flux (always summed in FP64).  One thread per face along axis dir.
// ------------------------------------------------------------------------
// NPT points per face: 2^D for the ADER step (tangential axes and time),
// 2^(D-1) for a Runge-Kutta stage (tangential axes only).
// SV: the Riemann solver (HOG_HLLC ... HOG_HLLI), a compile-time constant so
// that each instance keeps only its own solver's registers and instructions.
// Divisions by Newton-refined reciprocals (a few ulp instead of correctly
// rounded quotients: a quarter fewer instructions for FP64 HLLC) and, in FP32,
// the hardware square root.
template <int D, typename T, int NPT, int SV>
__global__ __launch_bounds__(256) void k_riemann(const T* __restrict__ FP, Box R, Box FB, int dir,
                                                 double gamma, double* __restrict__ F)
{
    constexpr int NV = D + 2;
    const long long nF = box_size(FB), nR = box_size(R);
    const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nF) return;
    int i, j, k;
    box_ijk(FB, f, i, j, k);
    const long long zl = box_index(R, i, j, k);
    const long long zr = box_index(R, i + (dir == 0), j + (dir == 1), k + (dir == 2));
    double Fb[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Fb[v] = 0.0;
    constexpr double w = 1.0 / NPT;
#pragma unroll
    for (int pt = 0; pt < NPT; ++pt) {
        T UL[NV], UR[NV], Fp[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            UL[v] = FP[((long long)((dir * 2 + 1) * NPT + pt) * NV + v) * nR + zl];
            UR[v] = FP[((long long)((dir * 2 + 0) * NPT + pt) * NV + v) * nR + zr];
        }
        riemann<D, T, true>(UL, UR, dir, SV, T(gamma), Fp);
#pragma unroll
        for (int v = 0; v < NV; ++v) Fb[v] += w * (double)Fp[v];     // face average in FP64
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v * nF + f] = Fb[v];
}

// Launch k_riemann with the solver as a template argument.
template <int D, typename T, int NPT = (1 << D)>
inline void launch_riemann(int solver, unsigned blocks, hipStream_t s, const T* FP, Box R, Box FB, int dir,
                           double gamma, double* F)
{
    switch (solver) {
    case 0: k_riemann<D, T, NPT, 0><<<blocks, 256, 0, s>>>(FP, R, FB, dir, gamma, F); break;
    case 1: k_riemann<D, T, NPT, 1><<<blocks, 256, 0, s>>>(FP, R, FB, dir, gamma, F); break;
    case 2: k_riemann<D, T, NPT, 2><<<blocks, 256, 0, s>>>(FP, R, FB, dir, gamma, F); break;
    case 3: k_riemann<D, T, NPT, 3><<<blocks, 256, 0, s>>>(FP, R, FB, dir, gamma, F); break;
    default: k_riemann<D, T, NPT, 4><<<blocks, 256, 0, s>>>(FP, R, FB, dir, gamma, F); break;
    }
}

// ------------------------------------------------------------------------
// a6 + a7: conservative update into the other state buffer (always FP64),
// then the CFL signal speed of the new state.
// ------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_update(const double* __restrict__ Uo, double* __restrict__ Un, Pad p,
                                                Box I, const double* __restrict__ Fx, Box FBx,
                                                const double* __restrict__ Fy, Box FBy,
                                                const double* __restrict__ Fz, Box FBz, StepInfo* info,
                                                double gamma, double ih0, double ih1, double ih2)
{
    constexpr int NV = D + 2;
    if (info->halted) return;                   // uniform: the run stopped at a non-physical state
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    bool ok = true;
    if (z < box_size(I)) {
        int i, j, k;
        box_ijk(I, z, i, j, k);
        const long long pi = pad_index(p, i, j, k);
        const double lx = info->lam[0], ly = info->lam[1], lz = info->lam[2];
        const long long nx = box_size(FBx), ny = box_size(FBy);
        const long long xm = box_index(FBx, i - 1, j, k), xp = box_index(FBx, i, j, k);
        const long long ym = box_index(FBy, i, j - 1, k), yp = box_index(FBy, i, j, k);
        double u[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double q = Uo[v * p.vs + pi];
            q = q - lx * (Fx[v * nx + xp] - Fx[v * nx + xm]);
            q = q - ly * (Fy[v * ny + yp] - Fy[v * ny + ym]);
            if constexpr (D == 3) {
                const long long nz = box_size(FBz);
                const long long zm = box_index(FBz, i, j, k - 1), zp = box_index(FBz, i, j, k);
                q = q - lz * (Fz[v * nz + zp] - Fz[v * nz + zm]);
            }
            u[v] = q;
            Un[v * p.vs + pi] = q;
        }
        s = signal_speed<D>(u, gamma, ih0, ih1, ih2, ok);
    }
    cfl_reduce<D>(s, ok, z, info);
}

// ------------------------------------------------------------------------
// State transfer between a user buffer and the padded interior.
// ------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_pack(const double* __restrict__ src, double* __restrict__ U, Pad p,
                                              Box I, int aos)
{
    constexpr int NV = D + 2;
    const long long N = box_size(I);
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= N) return;
    int i, j, k;
    box_ijk(I, z, i, j, k);
    const long long pi = pad_index(p, i, j, k);
#pragma unroll
    for (int v = 0; v < NV; ++v) U[v * p.vs + pi] = aos ? src[z * NV + v] : src[v * N + z];
}

template <int D>
__global__ __launch_bounds__(256) void k_unpack(const double* __restrict__ U, double* __restrict__ dst, Pad p,
                                                Box I, int aos)
{
    constexpr int NV = D + 2;
    const long long N = box_size(I);
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= N) return;
    int i, j, k;
    box_ijk(I, z, i, j, k);
    const long long pi = pad_index(p, i, j, k);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double x = U[v * p.vs + pi];
        if (aos) dst[z * NV + v] = x;
        else dst[v * N + z] = x;
    }
}

} // namespace hog

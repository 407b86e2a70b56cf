// hog_o2.h -- the second-order scheme of Sec. II.2 (Figs. 3-7) as one fused
// gfx950 kernel per step: MC-limited slopes of the conserved variables
// (Fig. 3), the pointwise predictor of the time mode (Fig. 4, read as the
// Hancock step of MUSCL-Hancock), the face states at the face centre and half
// time step with the Riemann solver (Fig. 5), the flux-difference update
// (Figs. 6-7) and the CFL signal speed of the new state (Fig. 7).
//
// Where the paper runs one kernel per stage with the 5-mode array U(:,:,:,:,5)
// and three flux arrays in device memory, here a workgroup owns a tile of
// zone columns and marches along the last axis, so the modes, face states and
// fluxes live in registers and LDS only: HBM sees the state read once and the
// new state written once.  Boundary conditions are applied at load time
// (periodic wrap or zero-gradient clamp of the zone index), so the padded
// ghost layers are never read or written.
//
// Thread layout: a TX x TY grid of zone columns (3D: 32 x 16, one workgroup of
// 8 wavefronts per compute unit; 2D: a row of 256, two per compute unit) whose
// outer ring is a halo of one zone (its modes are needed for the faces of the
// tile); the tile proper is the (TX-2) x (TY-2) inner part.  Per plane of the
// march axis a thread computes the modes of its zone, hands its +x / +y face
// states to its neighbours through LDS, solves the Riemann problems at its
// -x, -y and -z faces, hands the -x / -y fluxes back, and updates the zone of
// the previous plane once the z flux above it is known.
#pragma once
#include "hog_kernels.h"

namespace hog {

template <int D> struct O2Shape;
template <> struct O2Shape<3> { static constexpr int TX = 32, TY = 16, NT = 512, MINB = 1; };
template <> struct O2Shape<2> { static constexpr int TX = 256, TY = 1, NT = 256, MINB = 2; };

// Block max of the signal speed (up to 16 wavefronts) and one 64-bit atomic max.
__device__ __forceinline__ void o2_block_max(double s, StepInfo* info)
{
    __shared__ double red[16];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s = fmax(s, __shfl_xor(s, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = red[0];
        for (int q = 1; q < (int)(blockDim.x >> 6); ++q) b = fmax(b, red[q]);
        atomicMax(&info->smax_bits, (unsigned long long)__double_as_longlong(b));
    }
}

// Monotonised-central limiter with a compression factor (Fig. 3), from the
// forward difference a and the backward difference b: 0 unless both have the
// same strict sign, else that sign times min(|a+b|/2, cfac |a|, cfac |b|).
__device__ __forceinline__ double mc_slope(double a, double b, double cfac)
{
    const double m = fmin(0.5 * fabs(a + b), fmin(cfac * fabs(a), cfac * fabs(b)));
    return (a > 0.0 && b > 0.0) ? m : ((a < 0.0 && b < 0.0) ? -m : 0.0);
}

// Zone index along one axis after the boundary condition: clamp to the two
// zones beyond the interior that the scheme reads, then wrap (periodic) or
// clamp (outflow); an external axis reads the caller's ghost layers.
// Periodic axes have n >= 3, so one wrap suffices.
__device__ __forceinline__ int o2_src(int x, int n, int bc)
{
    x = min(max(x, -2), n + 1);
    if (bc == 2) return x;
    if (bc == 0) return x < 0 ? x + n : (x >= n ? x - n : x);
    return min(max(x, 0), n - 1);
}

struct O2Args {
    int n[3];        // interior zones per axis (n[2] = 1 in 2D)
    int bc[3];
    int zc;          // planes of the march axis per workgroup
    int positivity;  // 1: zones with an inadmissible face value fall back to their mean
    double gamma;
    double ih[3];    // 1 / dx_d
};

// Modes of one zone: slopes S[d][v] and the time mode T[v] = dt dU/dt from the
// mean u, the neighbours nb(d, v, side) along each axis (side 0 below, 1 above)
// and lam[d] = dt/dx_d.  Returns false if a face value U +- S_d/2 or a face
// state U +- S_d/2 + T/2 is inadmissible.  Without HANCOCK (a Runge-Kutta
// stage) the time mode is zero and only U +- S_d/2 is checked.
template <int D, bool HANCOCK, typename NB>
__device__ __forceinline__ bool o2_modes(const double* u, NB&& nb, const double* lam, double gm1,
                                         double (*S)[D + 2], double* T)
{
    constexpr int NV = D + 2;
    bool ok = true;
#pragma unroll
    for (int v = 0; v < NV; ++v) T[v] = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double Wm[NV], Wp[NV], Fm[NV], Fp[NV], pm, pp, um, up;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            S[d][v] = mc_slope(nb(d, v, 1) - u[v], u[v] - nb(d, v, 0), v == 0 ? 2.0 : 1.5);
            Wm[v] = u[v] - 0.5 * S[d][v];
            Wp[v] = u[v] + 0.5 * S[d][v];
        }
        if constexpr (!HANCOCK) {
            ok = ok && admissible<D, double, true>(Wm, gm1) && admissible<D, double, true>(Wp, gm1);
            continue;
        }
        flux_dir<D, double, true>(Wm, gm1, d, Fm, pm, um);
        flux_dir<D, double, true>(Wp, gm1, d, Fp, pp, up);
        ok = ok && Wm[0] > 0.0 && pm > 0.0 && isfinite(Wm[0]) && isfinite(pm);
        ok = ok && Wp[0] > 0.0 && pp > 0.0 && isfinite(Wp[0]) && isfinite(pp);
#pragma unroll
        for (int v = 0; v < NV; ++v) T[v] -= lam[d] * (Fp[v] - Fm[v]);
    }
    if constexpr (!HANCOCK) return ok;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double Wm[NV], Wp[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Wm[v] = u[v] - 0.5 * S[d][v] + 0.5 * T[v];
            Wp[v] = u[v] + 0.5 * S[d][v] + 0.5 * T[v];
        }
        ok = ok && admissible<D, double, true>(Wm, gm1) && admissible<D, double, true>(Wp, gm1);
    }
    return ok;
}

// Debug taps of the step: modes of the predictor box and the face fluxes
// (written only by the TAPS instantiation).
struct O2Taps {
    double* Q;
    Box R;
    double* F[3];
    Box FB[3];
};

// RK: a Runge-Kutta stage -- no time mode, and instead of the new state the
// kernel writes dt L of the interior zones to Lout ([v][zone], x fastest).
template <int D, int SOLVER, bool TAPS, bool RK>
__global__ __launch_bounds__(O2Shape<D>::NT, O2Shape<D>::MINB) void k_o2_step(const double* __restrict__ Uo, double* __restrict__ Un, Pad p,
                                                 O2Args a, StepInfo* info, O2Taps tp, double* __restrict__ Lout)
{
    using Sh = O2Shape<D>;
    constexpr int TX = Sh::TX, TY = Sh::TY, NT = TX * TY, NV = D + 2;
    constexpr int LX = TX + 2, LY = (D == 3) ? TY + 2 : 1, NL = LX * LY;
    constexpr int NRING = NL - NT;   // 3D: 4 (TX + 1); 2D: 2
    constexpr int E = (D == 3) ? NT : 1;
    __shared__ double sU[NV][NL];    // plane of the state around the tile
    __shared__ double sXp[NV][NT];   // +x face states
    __shared__ double sFx[NV][NT];   // -x face fluxes
    __shared__ double sYp[NV][E];
    __shared__ double sFy[NV][E];

    if constexpr (!RK) {
        if (info->halted) return;               // uniform: the run stopped at a non-physical state
    }
    // block -> (column tile, march chunk); the blocks of one XCD take a contiguous range
    const int n0 = a.n[0], n1 = a.n[1];
    const int nm = a.n[D - 1];                      // zones along the march axis
    const int nbx = (n0 + TX - 3) / (TX - 2);
    const int nby = (D == 3) ? (n1 + TY - 3) / (TY - 2) : 1;
    const int nbm = (nm + a.zc - 1) / a.zc;
    const int nb = nbx * nby * nbm;
    int b = xcd_group(blockIdx.x, nb);
    if (b >= nb) return;
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby;
    const int bm = b / nby;
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const int x0 = bx * (TX - 2), y0 = by * (TY - 2);
    const int ci = x0 - 1 + tx;                       // zone column of this thread
    const int cj = (D == 3) ? y0 - 1 + ty : 0;
    const int m0 = bm * a.zc, m1 = min(m0 + a.zc, nm);
    const bool live = ci <= n0 && (D == 2 || cj <= n1);      // zone within the predictor box
    const bool inner = tx >= 1 && tx <= TX - 2 && ci < n0 && (D == 2 || (ty >= 1 && ty <= TY - 2 && cj < n1));
    // fallback counting: each predictor-box zone is counted by one block only
    const bool own_x = ci >= (bx == 0 ? -1 : x0) && ci <= (bx == nbx - 1 ? n0 : x0 + TX - 3);
    const bool own_y = D == 2 || (cj >= (by == 0 ? -1 : y0) && cj <= (by == nby - 1 ? n1 : y0 + TY - 3));
    const int own_m_lo = bm == 0 ? -1 : m0, own_m_hi = bm == nbm - 1 ? nm : m1 - 1;

    const double gm1 = a.gamma - 1.0;
    const double lam[3] = {info->lam[0], info->lam[1], info->lam[2]};

    // global pad index of zone (x, y) of the tile plane at march coordinate m, after the boundary condition
    auto gidx = [&](int x, int y, int m) -> long long {
        const int sx = o2_src(x, n0, a.bc[0]);
        if constexpr (D == 3) return pad_index(p, sx, o2_src(y, n1, a.bc[1]), o2_src(m, nm, a.bc[2]));
        else return pad_index(p, sx, o2_src(m, nm, a.bc[1]), 0);
    };
    // this thread's ring slot of the LDS plane (threads tid < NRING)
    int rx = 0, ry = 0;
    if constexpr (D == 3) {
        if (tid < LX) { rx = tid; ry = 0; }
        else if (tid < 2 * LX) { rx = tid - LX; ry = LY - 1; }
        else { const int r = tid - 2 * LX; rx = (r & 1) ? LX - 1 : 0; ry = 1 + (r >> 1); }
    } else {
        rx = (tid == 0) ? 0 : LX - 1;
    }
    const int own_l = (D == 3 ? (ty + 1) * LX : 0) + tx + 1;
    const int ring_l = ry * LX + rx;
    const int gx_own = ci, gy_own = cj;
    const int gx_ring = x0 - 2 + rx, gy_ring = y0 - 2 + ry;

    double Um[NV], Uc[NV], Up[NV], Uq[NV], Rq[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) { Uq[v] = 0.0; Rq[v] = 0.0; }
    const double* Uv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Uv[v] = Uo + v * p.vs;
    auto load = [&](double* dst, int x, int y, int m) {
        const long long g = gidx(x, y, m);
#pragma unroll
        for (int v = 0; v < NV; ++v) dst[v] = Uv[v][g];
    };
    // prologue: planes m0-2 .. m0 in registers, plane m0-1 in LDS
    load(Um, gx_own, gy_own, m0 - 2);
    load(Uc, gx_own, gy_own, m0 - 1);
    load(Up, gx_own, gy_own, m0);
    if (tid < NRING) {
        double t[NV];
        load(t, gx_ring, gy_ring, m0 - 1);
#pragma unroll
        for (int v = 0; v < NV; ++v) sU[v][ring_l] = t[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) sU[v][own_l] = Uc[v];

    // zp_prev: +z face state of the previous plane's zone; acc: that zone's
    // increment so far (x / y flux differences and its -z flux term)
    double zp_prev[NV], acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) { zp_prev[v] = 0.0; acc[v] = 0.0; }
    double smax = 0.0;
    unsigned long long nfb = 0;
    double* const Q = TAPS ? tp.Q : nullptr;
    double* const Fx = TAPS ? tp.F[0] : nullptr;
    double* const Fy = TAPS ? tp.F[1] : nullptr;
    double* const Fz = TAPS ? tp.F[2] : nullptr;
    const Box& R = tp.R;
    const Box& FBx = tp.FB[0];
    const Box& FBy = tp.FB[1];
    const Box& FBz = tp.FB[2];
    const long long nR = TAPS ? box_size(R) : 0;

    for (int m = m0 - 1; m <= m1; ++m) {
        __syncthreads();   // A: plane m complete in LDS
        const bool xy_plane = m >= m0 && m < m1;      // planes whose x / y faces are needed
        double S[D][NV], T[NV];
        {
            auto nb = [&](int d, int v, int side) -> double {
                if (d == D - 1) return side ? Up[v] : Um[v];
                const int off = (d == 0) ? 1 : LX;
                return sU[v][side ? own_l + off : own_l - off];
            };
            bool ok = o2_modes<D, !RK>(Uc, nb, lam, gm1, S, T);
            if (!ok && a.positivity) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    T[v] = 0.0;
#pragma unroll
                    for (int d = 0; d < D; ++d) S[d][v] = 0.0;
                }
                if (live && own_x && own_y && m >= own_m_lo && m <= own_m_hi) ++nfb;
            }
        }
        if (TAPS && live && own_x && own_y && m >= own_m_lo && m <= own_m_hi) {
            const int i = ci, j = (D == 3) ? cj : m, k = (D == 3) ? m : 0;
            const long long r = box_index(R, i, j, k);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                Q[(long long)v * nR + r] = Uc[v];
#pragma unroll
                for (int d = 0; d < D; ++d) Q[((long long)(1 + d) * NV + v) * nR + r] = S[d][v];
                Q[((long long)(1 + D) * NV + v) * nR + r] = T[v];
            }
        }
        // face states at the half step (Fig. 5): +/- faces along each axis; the
        // +x / +y states go to the neighbours through LDS
        double xm[NV], ym[NV], zm[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double h = 0.5 * T[v];
            xm[v] = Uc[v] - 0.5 * S[0][v] + h;
            sXp[v][tid] = Uc[v] + 0.5 * S[0][v] + h;
            if constexpr (D == 3) {
                ym[v] = Uc[v] - 0.5 * S[1][v] + h;
                sYp[v][tid] = Uc[v] + 0.5 * S[1][v] + h;
            }
            zm[v] = Uc[v] - 0.5 * S[D - 1][v] + h;
        }
        // face m - 1/2 along the march axis lies between planes m-1 and m: both
        // states are this thread's, so it is solved before the exchange
        const bool zface = m >= m0;
        double Fzm[NV];
        if (zface) riemann<D, double, true>(zp_prev, zm, D - 1, SOLVER, a.gamma, Fzm);
#pragma unroll
        for (int v = 0; v < NV; ++v) zp_prev[v] = Uc[v] + 0.5 * S[D - 1][v] + 0.5 * T[v];
        if (zface && m - 1 >= m0 && inner) {
            // update of the zone of plane m-1: increment of Fig. 6 added to the mean (Fig. 7)
            const int i = ci, j = (D == 3) ? cj : m - 1, k = (D == 3) ? m - 1 : 0;
            if constexpr (RK) {
                const long long N = (long long)n0 * n1 * (D == 3 ? nm : 1);
                const long long zi = ((long long)k * n1 + j) * n0 + i;
#pragma unroll
                for (int v = 0; v < NV; ++v) Lout[v * N + zi] = acc[v] - lam[D - 1] * Fzm[v];
            } else {
                double u[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) u[v] = Um[v] + (acc[v] - lam[D - 1] * Fzm[v]);
                const long long pi = pad_index(p, i, j, k);
#pragma unroll
                for (int v = 0; v < NV; ++v) Un[v * p.vs + pi] = u[v];
                bool ok = true;
                const double sp = signal_speed<D>(u, a.gamma, a.ih[0], a.ih[1], a.ih[2], ok);
                if (ok) smax = fmax(smax, sp);
                else atomicMin(&info->bad, (unsigned long long)(((long long)k * n1 + j) * n0 + i));
            }
        }
        if (TAPS && zface && inner) {
            Box FB = (D == 3) ? FBz : FBy;
            double* Fm = (D == 3) ? Fz : Fy;
            const int i = ci, j = (D == 3) ? cj : m - 1, k = (D == 3) ? m - 1 : 0;
            const long long nF = box_size(FB);
            const long long f = box_index(FB, i, j, k);    // face m - 1/2
#pragma unroll
            for (int v = 0; v < NV; ++v) Fm[v * nF + f] = Fzm[v];
        }
        // the -z flux term of this plane's zone; the x / y terms follow below
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = zface ? lam[D - 1] * Fzm[v] : 0.0;
        __syncthreads();   // B: face states visible; plane m no longer read
        // own zone of plane m+2 for the next iteration (in flight during the
        // Riemann solves); plane m+1 into LDS (the ring read here)
        if (m + 2 <= m1 + 1) load(Uq, gx_own, gy_own, m + 2);
#pragma unroll
        for (int v = 0; v < NV; ++v) sU[v][own_l] = Up[v];
        if (tid < NRING) {
            load(Rq, gx_ring, gy_ring, m + 1);
#pragma unroll
            for (int v = 0; v < NV; ++v) sU[v][ring_l] = Rq[v];
        }
        double Fxm[NV], Fym[NV];
        if (xy_plane && tx >= 1) {
            double L[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) L[v] = sXp[v][tid - 1];
            riemann<D, double, true>(L, xm, 0, SOLVER, a.gamma, Fxm);
#pragma unroll
            for (int v = 0; v < NV; ++v) sFx[v][tid] = Fxm[v];
        }
        if constexpr (D == 3) {
            if (xy_plane && ty >= 1) {
                double L[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) L[v] = sYp[v][tid - TX];
                riemann<D, double, true>(L, ym, 1, SOLVER, a.gamma, Fym);
#pragma unroll
                for (int v = 0; v < NV; ++v) sFy[v][tid] = Fym[v];
            }
        }
        __syncthreads();   // C: -x / -y fluxes visible
        if (TAPS && xy_plane && inner) {
            const int i = ci, j = (D == 3) ? cj : m, k = (D == 3) ? m : 0;
            const long long nF = box_size(FBx);
            const long long f = box_index(FBx, i, j, k);   // face i + 1/2
#pragma unroll
            for (int v = 0; v < NV; ++v) Fx[v * nF + f] = sFx[v][tid + 1];
            if (tx == 1) {
                const long long fm = box_index(FBx, i - 1, j, k);
#pragma unroll
                for (int v = 0; v < NV; ++v) Fx[v * nF + fm] = Fxm[v];
            }
            if constexpr (D == 3) {
                const long long nFy = box_size(FBy);
                const long long g = box_index(FBy, i, j, k);
#pragma unroll
                for (int v = 0; v < NV; ++v) Fy[v * nFy + g] = sFy[v][tid + TX];
                if (ty == 1) {
                    const long long gm = box_index(FBy, i, j - 1, k);
#pragma unroll
                    for (int v = 0; v < NV; ++v) Fy[v * nFy + gm] = Fym[v];
                }
            } else {
                (void)Fy;
            }
        }
        // increment of this plane's zone so far, completed one plane later
        if (xy_plane && inner) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double d = -lam[0] * (sFx[v][tid + 1] - Fxm[v]);
                if constexpr (D == 3) d -= lam[1] * (sFy[v][tid + TX] - Fym[v]);
                acc[v] = d + acc[v];
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Um[v] = Uc[v];
            Uc[v] = Up[v];
            Up[v] = Uq[v];
        }
    }
    if (a.positivity && nfb) atomicAdd(&info->fallback, nfb);
    if constexpr (!RK) o2_block_max(smax, info);
}

} // namespace hog

// hog_rk.h -- Runge-Kutta time stepping on gfx950 (the paper's comparison of
// ADER with two-, three- and five-stage Runge-Kutta schemes, Sec. I.1 and
// Table IV).  Each stage applies the method-of-lines operator
//   dt L(U) = -sum_d dt/dx_d (F_d(+1/2) - F_d(-1/2))
// built from the same WENO reconstruction (or, at second order, the MC slopes
// of the fused kernel) and Riemann solver as the ADER step, with the face
// points in space only (2-point Gauss per tangential axis), and then the
// Shu-Osher combination u(i) = sum_k alpha_ik u(k) + beta_ik dt L(u(k)).
#pragma once
#include "hog_kernels.h"

namespace hog {

// Face-point states of the spatial polynomials (one thread per zone of the
// predictor box R): W [m][v] over R -> FP [d][side][pt][v] over R with
// 2^(D-1) points per face (pt = 2 a1 + a2 over the two tangential axes,
// first tangential axis outer).  With the positivity option a zone whose
// polynomial is inadmissible at one of its face points uses its mean there
// (first order); such zones are counted in info->fallback.
template <int D, int P>
__global__ __launch_bounds__(256) void k_face_points(const double* __restrict__ W, Box R, StepInfo* info,
                                                     double gamma, int positivity, double* __restrict__ FP)
{
    constexpr int NV = D + 2, NPT = 1 << (D - 1), NQ = 2 * D * NPT;
    constexpr Modes<D, P> M{};
    constexpr int NS = Modes<D, P>::NS;
    constexpr double g = 0.28867513459481288225;     // 2-point Gauss node on [-1/2, 1/2]
    const long long nR = box_size(R);
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool fb = false;
    if (z < nR) {
        // values at the face points, variable by variable (stored as they are
        // made); density and squared momentum of every point are kept for the
        // admissibility check, which completes with the energy
        double rho[NQ], ke[NQ];
        bool ok = true;
        const double gm1 = gamma - 1.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double w[NS];
#pragma unroll
            for (int m = 0; m < NS; ++m) w[m] = W[((long long)m * NV + v) * nR + z];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int t1 = (d == 0) ? 1 : 0, t2 = (D == 3) ? ((d == 2) ? 1 : 2) : -1;
#pragma unroll
                for (int side = 0; side < 2; ++side)
#pragma unroll
                    for (int pt = 0; pt < NPT; ++pt) {
                        double x[3] = {0.0, 0.0, 0.0};
                        x[d] = side ? 0.5 : -0.5;
                        x[t1] = ((D == 3 ? pt >> 1 : pt) & 1) ? g : -g;
                        if (t2 >= 0) x[t2] = (pt & 1) ? g : -g;
                        double s = 0.0;
#pragma unroll
                        for (int m = 0; m < NS; ++m)
                            s += w[m] * (mleg(M.a[m], x[0]) * mleg(M.b[m], x[1]) * mleg(M.c[m], x[2]));
                        const int q = (d * 2 + side) * NPT + pt;
                        FP[((long long)q * NV + v) * nR + z] = s;
                        if (v == 0) { rho[q] = s; ke[q] = 0.0; }
                        else if (v <= D) ke[q] += s * s;
                        else {
                            // the pressure as in admissible(): gm1 (E - 0.5 |m|^2 / rho)
                            const double pr = gm1 * (s - 0.5 * ke[q] / rho[q]);
                            ok = ok && rho[q] > 0.0 && pr > 0.0 && isfinite(rho[q]) && isfinite(pr);
                        }
                    }
            }
        }
        if (positivity && !ok) {
            fb = true;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double mean = W[(long long)v * nR + z];
#pragma unroll
                for (int q = 0; q < NQ; ++q) FP[((long long)q * NV + v) * nR + z] = mean;
            }
        }
    }
    if (positivity) {
        const unsigned long long nb = __popcll(__ballot(fb));
        if ((threadIdx.x & 63) == 0 && nb) atomicAdd(&info->fallback, nb);
    }
}

// Shu-Osher tables: rows (i, k, alpha_ik, beta_ik) of u(i) = sum_k alpha_ik
// u(k) + beta_ik dt L(u(k)) with the published coefficients: SSP-RK(2,2) and
// SSP-RK(3,3) of Shu and Osher, SSP-RK(5,4) of Spiteri and Ruuth.
struct RkRow {
    int i, k;
    double alpha, beta;
};
inline int rk_rows(int stepper, const RkRow** rows)
{
    static const RkRow r2[] = {{1, 0, 1.0, 1.0}, {2, 0, 0.5, 0.0}, {2, 1, 0.5, 0.5}};
    static const RkRow r3[] = {{1, 0, 1.0, 1.0}, {2, 0, 0.75, 0.0}, {2, 1, 0.25, 0.25},
                               {3, 0, 1.0 / 3.0, 0.0}, {3, 2, 2.0 / 3.0, 2.0 / 3.0}};
    static const RkRow r54[] = {{1, 0, 1.0, 0.391752226571890},
                                {2, 0, 0.444370493651235, 0.0}, {2, 1, 0.555629506348765, 0.368410593050371},
                                {3, 0, 0.620101851488403, 0.0}, {3, 2, 0.379898148511597, 0.251891774271694},
                                {4, 0, 0.178079954393132, 0.0}, {4, 3, 0.821920045606868, 0.544974750228521},
                                {5, 2, 0.517231671970585, 0.0}, {5, 3, 0.096059710526147, 0.063692468666290},
                                {5, 4, 0.386708617503269, 0.226007483236906}};
    if (stepper == 2) { *rows = r2; return 3; }
    if (stepper == 3) { *rows = r3; return 5; }
    if (stepper == 4) { *rows = r54; return 10; }
    *rows = nullptr;
    return 0;
}
inline int rk_nstages(int stepper) { return stepper == 2 ? 2 : (stepper == 3 ? 3 : (stepper == 4 ? 5 : 0)); }
// dt L(u(k)) is stored for later stages when some row with i > k + 1 uses it
inline bool rk_keep_L(int stepper, int k)
{
    const RkRow* r;
    const int n = rk_rows(stepper, &r);
    for (int t = 0; t < n; ++t)
        if (r[t].k == k && r[t].i > k + 1 && r[t].beta != 0.0) return true;
    return false;
}

// Terms of one Shu-Osher stage in the order of its table: coef[t] times the
// stage state src[t] (padded layout), a stored dt L (interior layout), or,
// for src[t] == nullptr, the dt L of the current stage.
struct RkStage {
    int n;
    const double* src[6];
    int padded[6];
    double coef[6];
};

// One stage: dt L of the current state from the face fluxes F[d] (or read
// from Lin when the fused second-order kernel made it), stored to Lout if
// later stages need it, then the stage combination into dst (padded); on the
// last stage also the CFL signal speed and non-physical check of the result.
template <int D>
__global__ __launch_bounds__(256) void k_rk_combine(Pad p, Box I, const double* __restrict__ Fx, Box FBx,
                                                    const double* __restrict__ Fy, Box FBy,
                                                    const double* __restrict__ Fz, Box FBz,
                                                    const double* __restrict__ Lin, double* __restrict__ Lout,
                                                    RkStage st, double* __restrict__ dst, StepInfo* info,
                                                    int last, double gamma, double ih0, double ih1, double ih2)
{
    constexpr int NV = D + 2;
    if (last && info->halted) return;           // uniform: the run stopped at a non-physical state
    const long long N = box_size(I);
    const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    bool ok = true;
    if (z < N) {
        int i, j, k;
        box_ijk(I, z, i, j, k);
        const long long pi = pad_index(p, i, j, k);
        double L[NV];
        if (Lin) {
#pragma unroll
            for (int v = 0; v < NV; ++v) L[v] = Lin[v * N + z];
        } else {
            const double lx = info->lam[0], ly = info->lam[1], lz = info->lam[2];
            const long long nx = box_size(FBx), ny = box_size(FBy);
            const long long xm = box_index(FBx, i - 1, j, k), xp = box_index(FBx, i, j, k);
            const long long ym = box_index(FBy, i, j - 1, k), yp = box_index(FBy, i, j, k);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double q = 0.0;
                q -= lx * (Fx[v * nx + xp] - Fx[v * nx + xm]);
                q -= ly * (Fy[v * ny + yp] - Fy[v * ny + ym]);
                if constexpr (D == 3) {
                    const long long nz = box_size(FBz);
                    const long long zm = box_index(FBz, i, j, k - 1), zp = box_index(FBz, i, j, k);
                    q -= lz * (Fz[v * nz + zp] - Fz[v * nz + zm]);
                }
                L[v] = q;
            }
        }
        if (Lout) {
#pragma unroll
            for (int v = 0; v < NV; ++v) Lout[v * N + z] = L[v];
        }
        double u[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = 0.0;
        for (int t = 0; t < st.n; ++t) {
            const double* src = st.src[t];
            const double c = st.coef[t];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double x = !src ? L[v] : (st.padded[t] ? src[v * p.vs + pi] : src[v * N + z]);
                u[v] += c * x;
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) dst[v * p.vs + pi] = u[v];
        if (last) s = signal_speed<D>(u, gamma, ih0, ih1, ih2, ok);
    }
    if (last) cfl_reduce<D>(s, ok, z, info);
}

} // namespace hog

// hog_char.h -- WENO reconstruction on characteristic variables (FP64): the
// alternative to the component-wise reconstruction on conserved variables
// that Sec. I.1 uses.  Each 1D application of the successive x -> y -> z
// sweeps projects the five stencil points of all variables on the
// characteristic fields of the flux Jacobian along its axis, evaluated at the
// mean of the zone the application is centred at; applies the 1D WENO
// operator to each field; and maps the coefficients back.
//
// Fields, in the order of the right eigenvectors r_k (columns of R): the
// u_n - c acoustic wave r = (1, u - c n, H - u_n c), the entropy wave
// r = (1, u, |u|^2/2), one shear wave per tangential axis t (in increasing
// axis order) r = (0, e_t, u_t), and the u_n + c acoustic wave
// r = (1, u + c n, H + u_n c).  Their left eigenvectors (rows of R^-1), with
// b1 = (gamma - 1)/c^2 and b2 = b1 |u|^2 / 2, applied to a state
// (rho, m, E):
//   l_-  . U = ((b2 + u_n/c) rho - b1 u.m - m_n/c + b1 E) / 2
//   l_0  . U = (1 - b2) rho + b1 u.m - b1 E
//   l_t  . U = m_t - u_t rho
//   l_+  . U = ((b2 - u_n/c) rho - b1 u.m + m_n/c + b1 E) / 2
#pragma once
#include <hip/hip_runtime.h>
#include "hog_kernels.h"

namespace hog {

// The scalars both projections need, from the conserved reference state.
template <int D>
struct CharFrame {
    double u[3], c, ic, H, b1, b2, q2h;
};

template <int D, int DIR>
__device__ __forceinline__ CharFrame<D> char_frame(const double* ref, double gamma)
{
    constexpr int NV = D + 2;
    CharFrame<D> f;
    const double ir = 1.0 / ref[0];
    double q2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        f.u[d] = d < D ? ref[1 + d] * ir : 0.0;
        q2 += f.u[d] * f.u[d];
    }
    const double p = (gamma - 1.0) * (ref[NV - 1] - 0.5 * ref[0] * q2);
    f.c = sqrt(gamma * p * ir);
    f.ic = 1.0 / f.c;
    f.H = (ref[NV - 1] + p) * ir;
    f.b1 = (gamma - 1.0) / (f.c * f.c);
    f.b2 = 0.5 * f.b1 * q2;
    f.q2h = 0.5 * q2;
    return f;
}

// Characteristic values w[k] of one conserved state U.
template <int D, int DIR>
__device__ __forceinline__ void char_project(const CharFrame<D>& f, const double* U, double* w)
{
    constexpr int NV = D + 2;
    double um = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) um += f.u[d] * U[1 + d];
    const double un = f.u[DIR], mn = U[1 + DIR], rho = U[0], E = U[NV - 1];
    const double base = f.b2 * rho - f.b1 * um + f.b1 * E;
    const double acc = (un * rho - mn) * f.ic;
    w[0] = 0.5 * (base + acc);
    w[1] = (1.0 - f.b2) * rho + f.b1 * um - f.b1 * E;
    int k = 2;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (d == DIR) continue;
        w[k++] = U[1 + d] - f.u[d] * rho;
    }
    w[NV - 1] = 0.5 * (base - acc);
}

// Conserved coefficient from characteristic coefficients cw[k] (R cw).
template <int D, int DIR>
__device__ __forceinline__ void char_back(const CharFrame<D>& f, const double* cw, double* out)
{
    constexpr int NV = D + 2;
    const double cm = cw[0], c0 = cw[1], cp = cw[NV - 1];
    const double un = f.u[DIR];
    out[0] = cm + c0 + cp;
    double E = (f.H - un * f.c) * cm + f.q2h * c0 + (f.H + un * f.c) * cp;
    int k = 2;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double m = f.u[d] * (cm + c0 + cp);
        if (d == DIR) {
            m += f.c * (cp - cm);
        } else {
            m += cw[k];
            E += f.u[d] * cw[k];
            ++k;
        }
        out[1 + d] = m;
    }
    out[NV - 1] = E;
}

// One 1D application on characteristic variables: line[v][0..4] of all
// variables, ref the conserved mean of the centre zone; out[v][1..P].
template <int D, int P, int DIR>
__device__ __forceinline__ void weno_char_line(const double (&line)[D + 2][5], const double* ref, double gamma,
                                               const WenoArgs& wa, double (&out)[D + 2][P + 1])
{
    constexpr int NV = D + 2;
    const CharFrame<D> f = char_frame<D, DIR>(ref, gamma);
    double w[NV][5];
#pragma unroll
    for (int o = 0; o < 5; ++o) {
        double u[NV], wk[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = line[v][o];
        char_project<D, DIR>(f, u, wk);
#pragma unroll
        for (int k = 0; k < NV; ++k) w[k][o] = wk[k];
    }
    double cw[NV][P + 1];
#pragma unroll
    for (int k = 0; k < NV; ++k) weno1d<P>(w[k], cw[k], wa);
#pragma unroll
    for (int a = 1; a <= P; ++a) {
        double ca[NV], o[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) ca[k] = cw[k][a];
        char_back<D, DIR>(f, ca, o);
#pragma unroll
        for (int v = 0; v < NV; ++v) out[v][a] = o[v];
    }
}

// x sweep: one thread per zone of AX, all variables.
template <int D, int P>
__global__ __launch_bounds__(256) void k_recon_x_char(const double* __restrict__ U, Pad p, Box AX,
                                                      double* __restrict__ A, WenoArgs wa0, double gamma,
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
    double line[NV][5], ref[NV], out[NV][P + 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
#pragma unroll
        for (int o = 0; o < 5; ++o) line[v][o] = U[v * p.vs + base + (o - 2)];
        ref[v] = line[v][2];
    }
    weno_char_line<D, P, 0>(line, ref, gamma, wa, out);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        A[(0 * NV + v) * nA + z] = line[v][2];
#pragma unroll
        for (int a = 1; a <= P; ++a) A[(a * NV + v) * nA + z] = out[v][a];
    }
}

// y and z sweeps: one thread per (line along the axis, chunk of kRecChunk
// zones, input mode) marching with all variables' stencils in registers; the
// reference of each application is the zone mean of its centre zone (mode 0
// of the input array at that zone).
template <int D, int P, int DIR, int NC>
__device__ __forceinline__ void march_line_char(const double* __restrict__ src, const double* __restrict__ mean,
                                                long long nsrc, long long c0, long long stride, int len,
                                                double* const* out0, double* const* outc, long long nout,
                                                long long z0, long long zstride, const WenoArgs& wa0, double gamma,
                                                const unsigned char* __restrict__ gate, const Box& I, int i, int j,
                                                int k)
{
    constexpr int NV = D + 2;
    double w[NV][5];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int o = 0; o < 5; ++o) w[v][o] = src[v * nsrc + c0 + (o - 2) * stride];
    long long zi = z0;
    for (int s = 0; s < len; ++s) {
#pragma unroll
        for (int v = 0; v < NV; ++v) out0[v][zi] = w[v][2];
        if constexpr (NC >= 1) {
            const int jj = (DIR == 1) ? j + s : j, kk = (DIR == 2) ? k + s : k;
            const WenoArgs wa = gated(wa0, gate, I, i, jj, kk);
            double ref[NV], out[NV][P + 1];
            const long long cc = c0 + (long long)s * stride;
#pragma unroll
            for (int v = 0; v < NV; ++v) ref[v] = mean[v * nsrc + cc];
            weno_char_line<D, P, DIR>(w, ref, gamma, wa, out);
#pragma unroll
            for (int q = 1; q <= NC; ++q)
#pragma unroll
                for (int v = 0; v < NV; ++v) outc[q - 1][v * nout + zi] = out[v][q];
        }
        if (s + 1 < len) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
#pragma unroll
                for (int o = 0; o < 4; ++o) w[v][o] = w[v][o + 1];
                w[v][4] = src[v * nsrc + c0 + (long long)(s + 3) * stride];
            }
        }
        zi += zstride;
    }
}

template <int D, int P>
__global__ __launch_bounds__(256) void k_recon_y_char(const double* __restrict__ A, Box AX, Box BY,
                                                      double* __restrict__ B, WenoArgs wa0, double gamma,
                                                      const unsigned char* __restrict__ gate, Box I)
{
    constexpr int NV = D + 2;
    constexpr Pairs<P> PR{};
    const long long nA = box_size(AX), nB = box_size(BY);
    const int nx = BY.n[0], nz = BY.n[2], nch = (BY.n[1] + kRecChunk - 1) / kRecChunk;
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)nx * nz * nch * (P + 1)) return;
    const int ix = (int)(t % nx); t /= nx;
    const int kz = (int)(t % nz); t /= nz;
    const int ch = (int)(t % nch);
    const int a = (int)(t / nch);
    const int i = BY.lo[0] + ix, k = BY.lo[2] + kz, j0 = BY.lo[1] + ch * kRecChunk;
    const int len = min(kRecChunk, BY.lo[1] + BY.n[1] - j0);
    const long long c0 = box_index(AX, i, j0, k), z0 = box_index(BY, i, j0, k);
    static_for<0, P + 1>([&](auto ac) {
        constexpr int a2 = decltype(ac)::value;
        if (a != a2) return;
        double* o0[1] = {B + (long long)PR.at[a2][0] * NV * nB};
        double* oc[P];
#pragma unroll
        for (int b = 1; b <= P - a2; ++b) oc[b - 1] = B + (long long)PR.at[a2][b] * NV * nB;
        double* outs0[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) outs0[v] = o0[0] + (long long)v * nB;
        march_line_char<D, P, 1, P - a2>(A + (long long)a2 * NV * nA, A, nA, c0, AX.n[0], len, outs0, oc, nB, z0,
                                         BY.n[0], wa0, gamma, gate, I, i, j0, k);
    });
}

template <int P>
__global__ __launch_bounds__(256) void k_recon_z_char(const double* __restrict__ B, Box BY, Box R,
                                                      double* __restrict__ W, WenoArgs wa0, double gamma,
                                                      const unsigned char* __restrict__ gate, Box I)
{
    constexpr int NV = 5;
    constexpr int NPAIR = (P + 1) * (P + 2) / 2;
    constexpr Modes<3, P> M{};
    constexpr Pairs<P> PR{};
    const long long nB = box_size(BY), nR = box_size(R);
    const int nx = R.n[0], ny = R.n[1], nch = (R.n[2] + kRecChunk - 1) / kRecChunk;
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)nx * ny * nch * NPAIR) return;
    const int ix = (int)(t % nx); t /= nx;
    const int jy = (int)(t % ny); t /= ny;
    const int ch = (int)(t % nch);
    const int pi = (int)(t / nch);
    const int i = R.lo[0] + ix, j = R.lo[1] + jy, k0 = R.lo[2] + ch * kRecChunk;
    const int len = min(kRecChunk, R.lo[2] + R.n[2] - k0);
    const long long c0 = box_index(BY, i, j, k0), z0 = box_index(R, i, j, k0);
    const long long sz = (long long)BY.n[0] * BY.n[1], zs = (long long)R.n[0] * R.n[1];
    static_for<0, P + 1>([&](auto bc) {
        constexpr int b = decltype(bc)::value;
        static_for<0, P + 1 - b>([&](auto ac) {
            constexpr int a = decltype(ac)::value;
            if (pi != PR.at[a][b]) return;
            double* oc[P];
#pragma unroll
            for (int cc = 1; cc <= P - a - b; ++cc) oc[cc - 1] = W + (long long)M.at[a][b][cc][0] * NV * nR;
            double* outs0[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) outs0[v] = W + ((long long)M.at[a][b][0][0] * NV + v) * nR;
            march_line_char<3, P, 2, P - a - b>(B + (long long)PR.at[a][b] * NV * nB, B, nB, c0, sz, len, outs0,
                                                oc, nR, z0, zs, wa0, gamma, gate, I, i, j, k0);
        });
    });
}

} // namespace hog

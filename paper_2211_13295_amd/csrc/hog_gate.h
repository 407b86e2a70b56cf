// hog_gate.h -- learned smooth-zone gate on gfx950: stencil features, BF16
// MFMA inference, training-data harvest, and the training kernels (forward,
// backward, weight gradients, Adam).
//
// Network: x (BF16) -> h1 = relu(W1 x + b1) (64) -> h2 = relu(W2 h1 + b2) (64)
// -> logit = w3 . h2 + b3; W1, W2, w3 and the layer inputs in BF16, biases,
// accumulation and activations in FP32 (activations rounded to BF16 as the
// next layer's input).  A zone is gated ("smooth") when logit >= the logit of
// the threshold probability; the 1D WENO applications centred at a gated
// interior zone then use the linear weights.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "hog_kernels.h"

namespace hog {

constexpr int kHidden = 64;

template <int D>
struct GateShape {
    static constexpr int NV = D + 2;
    static constexpr int NC = 4 * D + 1;          // cross: centre + 4 per axis
    static constexpr int NF = NV * NC;            // 36 (2D) / 65 (3D)
    static constexpr int NFP = (NF + 15) / 16 * 16;   // padded to the MFMA K step
    static constexpr int NPARAM = kHidden * NF + kHidden + kHidden * kHidden + kHidden + kHidden + 1;
};

// Device copy of the gate (BF16 weights, FP32 biases).
template <int D>
struct GateParams {
    using G = GateShape<D>;
    uint16_t W1[kHidden][G::NFP];   // zero-padded columns
    float b1[kHidden];
    uint16_t W2[kHidden][kHidden];
    float b2[kHidden];
    uint16_t w3[kHidden];
    float b3;
    float logit_thr;
};

__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ float bfround(float x) { return bf2f(f2bf(x)); }

// Features of variable v of zone (i,j,k) from the padded state: the 13-zone
// cross (centre, x-2, x-1, x+1, x+2, y-2, ..., z+2; 9 zones in 2D), centred on
// the zone value and scaled by (max - min + 1e-12 max(1, |centre|)), in FP64,
// then FP32.
template <int D>
__device__ __forceinline__ void gate_features_var(const double* __restrict__ U, const Pad& p, int i, int j, int k,
                                                  int v, float* f)
{
    using G = GateShape<D>;
    const long long c0 = pad_index(p, i, j, k);
    const long long st[3] = {1, p.np[0], (long long)p.np[0] * p.np[1]};
    const double* u = U + v * p.vs + c0;
    double val[G::NC];
    val[0] = u[0];
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        val[1 + 4 * ax + 0] = u[-2 * st[ax]];
        val[1 + 4 * ax + 1] = u[-1 * st[ax]];
        val[1 + 4 * ax + 2] = u[1 * st[ax]];
        val[1 + 4 * ax + 3] = u[2 * st[ax]];
    }
    double mx = val[0], mn = val[0];
#pragma unroll
    for (int s = 1; s < G::NC; ++s) { mx = fmax(mx, val[s]); mn = fmin(mn, val[s]); }
    const double scale = mx - mn + 1e-12 * fmax(1.0, fabs(val[0]));
#pragma unroll
    for (int s = 0; s < G::NC; ++s) f[s] = (float)((val[s] - val[0]) / scale);
}

// All features of zone (i,j,k), ordered [variable][cross].
template <int D>
__device__ __forceinline__ void gate_features(const double* __restrict__ U, const Pad& p, int i, int j, int k,
                                              float* f)
{
    using G = GateShape<D>;
#pragma unroll
    for (int v = 0; v < G::NV; ++v) gate_features_var<D>(U, p, i, j, k, v, f + v * G::NC);
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// One wavefront evaluates the gate on 16 interior zones with BF16 MFMA
// (16x16x16, FP32 accumulation).  Operand layout of the 16x16x16 BF16 MFMA
// on CDNA: A lane l holds A[l%16][4(l/16)+0..3], B lane l holds
// B[4(l/16)+0..3][l%16], the result lane l holds D[4(l/16)+0..3][l%16].
template <int D>
__global__ __launch_bounds__(64) void k_gate_infer(const double* __restrict__ U, Pad p, Box I,
                                                   const GateParams<D>* __restrict__ gp,
                                                   unsigned char* __restrict__ flags, float* __restrict__ logits)
{
    using G = GateShape<D>;
    __shared__ uint16_t sx[16][G::NFP];
    __shared__ float sh[16][kHidden + 1];
    const long long N = box_size(I);
    const int lane = threadIdx.x;
    const long long z0 = (long long)blockIdx.x * 16;
    // features: one (zone, variable) per lane and round
    for (int t = lane; t < 16 * G::NV; t += 64) {
        const int zl = t & 15, v = t >> 4;
        const long long z = z0 + zl;
        float f[G::NC];
        if (z < N) {
            int i, j, k;
            box_ijk(I, z, i, j, k);
            gate_features_var<D>(U, p, i, j, k, v, f);
        } else {
#pragma unroll
            for (int q = 0; q < G::NC; ++q) f[q] = 0.0f;
        }
#pragma unroll
        for (int q = 0; q < G::NC; ++q) sx[zl][v * G::NC + q] = f2bf(f[q]);
    }
    for (int t = lane; t < 16 * (G::NFP - G::NF); t += 64)
        sx[t / (G::NFP - G::NF)][G::NF + t % (G::NFP - G::NF)] = (uint16_t)0;
    __syncthreads();
    const int r = lane & 15, g4 = lane >> 4;
    // layer 1: [16 x NFP] x [NFP x 64]
    f32x4 acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < G::NFP / 16; ++kc) {
        bf16x4 a;
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = (short)sx[r][16 * kc + 4 * g4 + q];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            bf16x4 b;
#pragma unroll
            for (int q = 0; q < 4; ++q) b[q] = (short)gp->W1[16 * nt + r][16 * kc + 4 * g4 + q];
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[nt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int col = 16 * nt + r;
            sh[4 * g4 + q][col] = bfround(fmaxf(acc[nt][q] + gp->b1[col], 0.0f));
        }
    __syncthreads();
    // layer 2: [16 x 64] x [64 x 64]
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
        bf16x4 a;
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = (short)f2bf(sh[r][16 * kc + 4 * g4 + q]);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            bf16x4 b;
#pragma unroll
            for (int q = 0; q < 4; ++q) b[q] = (short)gp->W2[16 * nt + r][16 * kc + 4 * g4 + q];
            acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[nt], 0, 0, 0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int col = 16 * nt + r;
            sh[4 * g4 + q][col] = bfround(fmaxf(acc[nt][q] + gp->b2[col], 0.0f));
        }
    __syncthreads();
    // layer 3 on the VALU
    if (lane < 16) {
        const long long z = z0 + lane;
        float s = gp->b3;
#pragma unroll
        for (int q = 0; q < kHidden; ++q) s += sh[lane][q] * bf2f(gp->w3[q]);
        if (z < N) {
            if (flags) flags[z] = s >= gp->logit_thr ? 1 : 0;
            if (logits) logits[z] = s;
        }
    }
}

// Largest |omega_k / gamma_k - 1| of the nonlinear weights of one 1D WENO
// application (the smoothness measure the gate is trained on).
template <int P>
__device__ __forceinline__ double weno_deviation(const double* v, const WenoArgs& wa)
{
    const double l1 = 0.5 * v[0] - 2.0 * v[1] + 1.5 * v[2];
    const double l2 = 0.5 * v[0] - v[1] + 0.5 * v[2];
    const double m1 = 0.5 * (v[3] - v[1]);
    const double m2 = 0.5 * v[1] - v[2] + 0.5 * v[3];
    const double r1 = -1.5 * v[2] + 2.0 * v[3] - 0.5 * v[4];
    const double r2 = 0.5 * v[2] - v[3] + 0.5 * v[4];
    constexpr double k13_3 = 13.0 / 3.0;
    const double bL = wa.eps + (l1 * l1 + k13_3 * l2 * l2);
    const double bC = wa.eps + (m1 * m1 + k13_3 * m2 * m2);
    const double bR = wa.eps + (r1 * r1 + k13_3 * r2 * r2);
    if constexpr (P == 2) {
        const double aL = wa.g[0] / (bL * bL), aC = wa.g[1] / (bC * bC), aR = wa.g[2] / (bR * bR);
        const double s = aL + aC + aR;
        return fmax(fabs(aL / s / wa.g[0] - 1.0), fmax(fabs(aC / s / wa.g[1] - 1.0), fabs(aR / s / wa.g[2] - 1.0)));
    } else {
        const double h1 = (11.0 * (v[0] - v[4]) + 82.0 * (v[3] - v[1])) * (1.0 / 120.0);
        const double h2 = (-3.0 * (v[0] + v[4]) + 40.0 * (v[1] + v[3]) - 74.0 * v[2]) * (1.0 / 56.0);
        const double h3 = ((v[4] - v[0]) + 2.0 * (v[1] - v[3])) * (1.0 / 12.0);
        const double s1 = h1 + 0.1 * h3;
        const double bH = wa.eps + (s1 * s1 + k13_3 * h2 * h2 + (781.0 / 20.0) * h3 * h3);
        const double aH = wa.g[0] / (bH * bH), aL = wa.g[1] / (bL * bL), aC = wa.g[2] / (bC * bC),
                     aR = wa.g[3] / (bR * bR);
        const double s = aH + aL + aC + aR;
        return fmax(fmax(fabs(aH / s / wa.g[0] - 1.0), fabs(aL / s / wa.g[1] - 1.0)),
                    fmax(fabs(aC / s / wa.g[2] - 1.0), fabs(aR / s / wa.g[3] - 1.0)));
    }
}

// Training samples of listed interior zones: features (FP32) and the largest
// weight deviation over the variables and the 1D applications centred at the
// zone (x sweep of the zone averages, y sweeps of the x-sweep modes, z sweeps
// of the y-sweep modes; needs the FP64 sweep outputs A and B of this state).
template <int D, int P>
__global__ __launch_bounds__(256) void k_harvest(const double* __restrict__ U, Pad p, Box I,
                                                 const double* __restrict__ A, Box AX,
                                                 const double* __restrict__ B, Box BY,
                                                 const long long* __restrict__ zones, long long n, WenoArgs wa,
                                                 float* __restrict__ feat, float* __restrict__ maxdev)
{
    using G = GateShape<D>;
    constexpr int NV = D + 2;
    constexpr Pairs<P> PR{};
    const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const long long z = zones[s];
    if (z < 0 || z >= box_size(I)) {      // not an interior zone: NaN sample, nothing read
        const float nan = __builtin_nanf("");
#pragma unroll
        for (int q = 0; q < G::NF; ++q) feat[(long long)q * n + s] = nan;
        maxdev[s] = nan;
        return;
    }
    int i, j, k;
    box_ijk(I, z, i, j, k);
    float f[G::NF];
    gate_features<D>(U, p, i, j, k, f);
#pragma unroll
    for (int q = 0; q < G::NF; ++q) feat[(long long)q * n + s] = f[q];
    double dmax = 0.0;
    const long long nA = box_size(AX), nB = box_size(BY);
    const long long pc = pad_index(p, i, j, k), ca = box_index(AX, i, j, k), cb = box_index(BY, i, j, k);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double line[5];
#pragma unroll
        for (int o = 0; o < 5; ++o) line[o] = U[v * p.vs + pc + (o - 2)];
        dmax = fmax(dmax, weno_deviation<P>(line, wa));
#pragma unroll
        for (int a = 0; a < P; ++a) {
#pragma unroll
            for (int o = 0; o < 5; ++o) line[o] = A[(a * NV + v) * nA + ca + (o - 2) * AX.n[0]];
            dmax = fmax(dmax, weno_deviation<P>(line, wa));
        }
        if constexpr (D == 3) {
            const long long sz = (long long)BY.n[0] * BY.n[1];
#pragma unroll
            for (int b = 0; b < P; ++b)
#pragma unroll
                for (int a = 0; a + b < P; ++a) {
#pragma unroll
                    for (int o = 0; o < 5; ++o) line[o] = B[(PR.at[a][b] * NV + v) * nB + cb + (o - 2) * sz];
                    dmax = fmax(dmax, weno_deviation<P>(line, wa));
                }
        }
    }
    maxdev[s] = (float)dmax;
}

// ------------------------------------------------------------------------
// Training (FP32 VALU, BF16-rounded operands as in inference; deterministic).
// Parameter vector (FP32): W1[64][NF], b1[64], W2[64][64], b2[64], w3[64], b3.
// ------------------------------------------------------------------------
template <int NF>
struct MlpOffsets {
    static constexpr int W1 = 0;
    static constexpr int B1 = W1 + kHidden * NF;
    static constexpr int W2 = B1 + kHidden;
    static constexpr int B2 = W2 + kHidden * kHidden;
    static constexpr int W3 = B2 + kHidden;
    static constexpr int B3 = W3 + kHidden;
    static constexpr int N = B3 + 1;
};

// Per sample: forward, loss term and the backward pass down to dh1; stores
// the values the weight gradients need, feature-major ([feature][sample]).
template <int NF>
__global__ __launch_bounds__(128) void k_mlp_fwd_bwd(const float* __restrict__ X, const float* __restrict__ y,
                                                     const float* __restrict__ cw, int n,
                                                     const float* __restrict__ prm, float* __restrict__ xb,
                                                     float* __restrict__ h1o, float* __restrict__ h2o,
                                                     float* __restrict__ d1o, float* __restrict__ d2o,
                                                     float* __restrict__ dzo, float* __restrict__ losso,
                                                     float* __restrict__ logito)
{
    using O = MlpOffsets<NF>;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float x[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) {
        x[q] = bfround(X[(long long)s * NF + q]);
        if (xb) xb[(long long)q * n + s] = x[q];
    }
    float z1[kHidden], h1[kHidden];
    for (int o = 0; o < kHidden; ++o) {
        float acc = prm[O::B1 + o];
#pragma unroll
        for (int q = 0; q < NF; ++q) acc += bfround(prm[O::W1 + o * NF + q]) * x[q];
        z1[o] = acc;
        h1[o] = bfround(fmaxf(acc, 0.0f));
    }
    float z2[kHidden], h2[kHidden];
    for (int o = 0; o < kHidden; ++o) {
        float acc = prm[O::B2 + o];
#pragma unroll 8
        for (int q = 0; q < kHidden; ++q) acc += bfround(prm[O::W2 + o * kHidden + q]) * h1[q];
        z2[o] = acc;
        h2[o] = bfround(fmaxf(acc, 0.0f));
    }
    float logit = prm[O::B3];
    for (int q = 0; q < kHidden; ++q) logit += bfround(prm[O::W3 + q]) * h2[q];
    if (logito) logito[s] = logit;
    if (!y) return;
    const float yy = y[s], c = cw ? cw[s] : 1.0f;
    const float pr = 1.0f / (1.0f + expf(-logit));
    losso[s] = c * (fmaxf(logit, 0.0f) - logit * yy + log1pf(expf(-fabsf(logit))));
    const float dz = c * (pr - yy) / (float)n;
    dzo[s] = dz;
    float d2[kHidden];
    for (int o = 0; o < kHidden; ++o) {
        d2[o] = z2[o] > 0.0f ? dz * bfround(prm[O::W3 + o]) : 0.0f;
        d2o[(long long)o * n + s] = d2[o];
        h1o[(long long)o * n + s] = h1[o];
        h2o[(long long)o * n + s] = h2[o];
    }
    for (int q = 0; q < kHidden; ++q) {
        float acc = 0.0f;
#pragma unroll 8
        for (int o = 0; o < kHidden; ++o) acc += d2[o] * bfround(prm[O::W2 + o * kHidden + q]);
        d1o[(long long)q * n + s] = z1[q] > 0.0f ? acc : 0.0f;
    }
}

// Weight gradients: one thread per parameter, sum over the batch in sample
// order (deterministic).
template <int NF>
__global__ __launch_bounds__(256) void k_mlp_wgrad(const float* __restrict__ xb, const float* __restrict__ h1,
                                                   const float* __restrict__ h2, const float* __restrict__ d1,
                                                   const float* __restrict__ d2, const float* __restrict__ dz,
                                                   int n, float* __restrict__ grad)
{
    using O = MlpOffsets<NF>;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= O::N) return;
    const float *a = nullptr, *b = nullptr;
    if (t < O::B1) { a = d1 + (long long)(t / NF) * n; b = xb + (long long)(t % NF) * n; }
    else if (t < O::W2) { a = d1 + (long long)(t - O::B1) * n; }
    else if (t < O::B2) { const int u = t - O::W2; a = d2 + (long long)(u / kHidden) * n; b = h1 + (long long)(u % kHidden) * n; }
    else if (t < O::W3) { a = d2 + (long long)(t - O::B2) * n; }
    else if (t < O::B3) { a = dz; b = h2 + (long long)(t - O::W3) * n; }
    else { a = dz; }
    float acc = 0.0f;
    if (b) {
        for (int s = 0; s < n; ++s) acc += a[s] * b[s];
    } else {
        for (int s = 0; s < n; ++s) acc += a[s];
    }
    grad[t] = acc;
}

// Adam on the FP32 masters.
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ prm, float* __restrict__ m,
                                                  float* __restrict__ v, const float* __restrict__ grad, int np,
                                                  float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= np) return;
    const float g = grad[t];
    const float mm = b1 * m[t] + (1.0f - b1) * g;
    const float vv = b2 * v[t] + (1.0f - b2) * g * g;
    m[t] = mm;
    v[t] = vv;
    prm[t] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// Sum of n values in a fixed order (one block).
__global__ __launch_bounds__(256) void k_sum_fixed(const float* __restrict__ x, int n, float* __restrict__ out)
{
    __shared__ float part[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) s += x[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0] / (float)n;
}

} // namespace hog

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
    // device layout of the features in inference: each variable's block padded
    // to 16 columns (32 bytes, written as two 16-byte stores)
    static constexpr int NCB = 16;
    static_assert(NC <= NCB, "a cross fits one 16-column block");
    static constexpr int NFL = NV * NCB;          // 64 (2D) / 80 (3D)
    static constexpr int NFP = (NFL + 31) / 32 * 32;   // padded to the MFMA K step (32)
    static constexpr int NPARAM = kHidden * NF + kHidden + kHidden * kHidden + kHidden + kHidden + 1;
};

// Device copy of the gate (BF16 weights, FP32 biases).  W1's columns are in
// the device feature layout (variable v, cross point q at column v NCB + q;
// the pad columns are zero).
template <int D>
struct __align__(16) GateParams {
    using G = GateShape<D>;
    uint16_t W1[kHidden][G::NFP];
    float b1[kHidden];
    uint16_t W2[kHidden][kHidden];
    float b2[kHidden];
    uint16_t w3[kHidden];
    float b3;
    float logit_thr;
};

// FP32 -> BF16 with round to nearest even (gfx950's conversion instruction)
__device__ __forceinline__ uint16_t f2bf(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ float bfround(float x) { return bf2f(f2bf(x)); }

// Features of variable v of zone (i,j,k) from the padded state: the 13-zone
// cross (centre, x-2, x-1, x+1, x+2, y-2, ..., z+2; 9 zones in 2D), centred on
// the zone value and scaled by (max - min + 1e-12 max(1, |centre|)), in FP64,
// then FP32.  RCP: multiply by the reciprocal of the scale instead of dividing
// (inference; the harvest keeps the division of the definition).
template <int D, bool RCP = false>
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
    if constexpr (RCP) {
        const double r = 1.0 / scale;
#pragma unroll
        for (int s = 0; s < G::NC; ++s) f[s] = (float)((val[s] - val[0]) * r);
    } else {
#pragma unroll
        for (int s = 0; s < G::NC; ++s) f[s] = (float)((val[s] - val[0]) / scale);
    }
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
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Gate inference.  Each wavefront keeps the network as MFMA operand fragments
// in registers (loaded once) and loops over tiles of 64 interior zones: lane l
// computes the features of zone l of the tile, one variable per round, into an
// LDS row of the tile (the first variable of the next tile is loaded before
// the network runs on this one).  Per 16-zone slice the three layers run
// transposed, as BF16 MFMAs with FP32 accumulation: H1^T = W1 X^T (A = W1,
// B = the slice's feature rows), H2^T = W2 relu(H1)^T, logit = w3 relu(H2)^T
// (A = w3 in row 0).  A layer's output fragment holds, for zone l%16, the
// hidden units 16 nt + 4 (l/16) + q (q = 0..3) of output tile nt; these are
// exactly the eight inputs per K chunk the next layer's B fragment needs for
// the same zone once the next layer's weight columns are stored in the order
// position 32 kc + 8 g + i <- unit 16 (2 kc + i/4) + 4 g + i%4 (gate_unit),
// so the hidden activations never leave the registers.  The biases of the two
// hidden layers (kept in LDS) are the accumulators' initial values.  Operand layout of
// gfx950's 16x16x32 BF16 MFMA: A lane l holds A[l%16][8(l/16)+0..7], B lane l
// holds B[8(l/16)+0..7][l%16], the result lane l holds D[4(l/16)+0..3][l%16].
constexpr int kGateWaves = 4;   // wavefronts per workgroup
constexpr int kGateTile = 64;   // zones per wavefront and tile

// Hidden unit whose activation sits at input position p of layers 2 and 3.
__host__ __device__ constexpr int gate_unit(int p)
{
    return 16 * (2 * (p / 32) + (p % 8) / 4) + 4 * ((p % 32) / 8) + p % 4;
}

template <int D>
struct GateLds {
    static constexpr int RS = GateShape<D>::NFP + 8;   // row stride (shorts): 16-byte aligned rows, padded
};

// relu of an output fragment pair, rounded to BF16, as one B fragment: the
// values are rounded in pairs, then the negative ones (sign bit set, so
// negative as 16-bit integers) are replaced by zero with a packed integer max
typedef short i16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t relu_bf16x2(float a, float b)
{
    const bf16x2 pr = __builtin_convertvector(f32x2{a, b}, bf16x2);
    const i16x2 m = __builtin_elementwise_max(__builtin_bit_cast(i16x2, pr), i16x2{0, 0});
    return __builtin_bit_cast(uint32_t, m);
}
__device__ __forceinline__ bf16x8 gate_hidden(const f32x4& lo, const f32x4& hi)
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 w = {relu_bf16x2(lo[0], lo[1]), relu_bf16x2(lo[2], lo[3]), relu_bf16x2(hi[0], hi[1]),
                     relu_bf16x2(hi[2], hi[3])};
    return __builtin_bit_cast(bf16x8, w);
}

// FP64 -> FP32 (round to nearest even), kept as an FP32 value so that the
// following FP32 -> BF16 conversion rounds it again, as the definition does
__device__ __forceinline__ float to_f32(double x)
{
    float f = (float)x;
    asm volatile("" : "+v"(f));
    return f;
}

template <int D>
__global__ __launch_bounds__(64 * kGateWaves, 3) void k_gate_infer(const double* __restrict__ U, Pad p, Box I,
                                                                const GateParams<D>* __restrict__ gp,
                                                                unsigned char* __restrict__ flags,
                                                                float* __restrict__ logits)
{
    using G = GateShape<D>;
    constexpr int KC = G::NFP / 32;
    constexpr int RS = GateLds<D>::RS;
    __shared__ __align__(16) uint16_t sx[kGateWaves][kGateTile][RS];
    __shared__ __align__(16) float sb[2][kHidden];   // biases of the hidden layers
    __shared__ __align__(16) uint16_t sw3[kHidden + 8];   // last layer's weights, then 8 zeros
    const long long N = box_size(I);
    const long long ntiles = (N + kGateTile - 1) / kGateTile;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = lane & 15, g4 = lane >> 4;
    uint16_t(*row)[RS] = sx[wv];
    if (threadIdx.x < 2 * kHidden) sb[threadIdx.x / kHidden][threadIdx.x % kHidden] = threadIdx.x < kHidden
        ? gp->b1[threadIdx.x] : gp->b2[threadIdx.x - kHidden];
    if (threadIdx.x < kHidden + 8) sw3[threadIdx.x] = threadIdx.x < kHidden ? gp->w3[threadIdx.x] : 0;
    __syncthreads();

    // A fragments of the first two weight matrices
    bf16x8 w1[KC][4], w2[2][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int col = 16 * nt + r;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) w1[kc][nt] = *reinterpret_cast<const bf16x8*>(&gp->W1[col][32 * kc + 8 * g4]);
#pragma unroll
        for (int kc = 0; kc < 2; ++kc) w2[kc][nt] = *reinterpret_cast<const bf16x8*>(&gp->W2[col][32 * kc + 8 * g4]);
    }
    const float b3 = gp->b3, thr = gp->logit_thr;
    // the pad columns past the features stay zero
#pragma unroll
    for (int q = G::NFL; q < G::NFP; q += 2) reinterpret_cast<uint32_t*>(row[lane])[q / 2] = 0u;

    const long long st[3] = {1, p.np[0], (long long)p.np[0] * p.np[1]};
    auto centre = [&](long long t) {
        const long long z = t * kGateTile + lane;
        int i = 0, j = 0, k = 0;
        if (z < N) box_ijk(I, z, i, j, k);
        else box_ijk(I, 0, i, j, k);   // a valid zone; its result is not stored
        return pad_index(p, i, j, k);
    };
    auto load_cross = [&](long long c0, int v, double* out) {
        const double* u = U + v * p.vs + c0;
        out[0] = u[0];
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            out[1 + 4 * ax + 0] = u[-2 * st[ax]];
            out[1 + 4 * ax + 1] = u[-1 * st[ax]];
            out[1 + 4 * ax + 2] = u[1 * st[ax]];
            out[1 + 4 * ax + 3] = u[2 * st[ax]];
        }
    };
    double val[2][G::NC];
    long long t = (long long)blockIdx.x * kGateWaves + wv;
    const long long tstride = (long long)gridDim.x * kGateWaves;
    long long c0 = centre(t);
    if (t < ntiles) load_cross(c0, 0, val[0]);
    for (; t < ntiles; t += tstride) {
        // features of zone `lane`, variable by variable; the cross of the next
        // variable is loaded while the current one is scaled (two buffers).
        // Scale from the differences to the centre (max - min of the cross is
        // the largest minus the smallest difference, the centre's being 0).
        // Each variable's 13 features and 3 zero pads are one 32-byte block of
        // the row, written as two 16-byte stores.
        uint16_t* rw = row[lane];
#pragma unroll
        for (int v = 0; v < G::NV; ++v) {
            if (v + 1 < G::NV) load_cross(c0, v + 1, val[(v + 1) & 1]);
            const double* x = val[v & 1];
            double d[G::NC];
            d[0] = 0.0;
            double mx = 0.0, mn = 0.0;
#pragma unroll
            for (int q = 1; q < G::NC; ++q) {
                d[q] = x[q] - x[0];
                mx = fmax(mx, d[q]);
                mn = fmin(mn, d[q]);
            }
            const double rs = recip(mx - mn + 1e-12 * fmax(1.0, fabs(x[0])));
            // FP64 -> FP32 -> BF16 (round to nearest even), two features per word
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
            uint32_t wd[G::NCB / 2];
#pragma unroll
            for (int q = 0; q < G::NCB; q += 2) {
                const float f0 = q < G::NC ? to_f32(d[q] * rs) : 0.0f;
                const float f1 = q + 1 < G::NC ? to_f32(d[q + 1] * rs) : 0.0f;
                wd[q / 2] = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{f0, f1}, bf16x2));
            }
#pragma unroll
            for (int k = 0; k < G::NCB / 8; ++k)
                *reinterpret_cast<u32x4*>(&rw[v * G::NCB + 8 * k]) =
                    u32x4{wd[4 * k], wd[4 * k + 1], wd[4 * k + 2], wd[4 * k + 3]};
        }
        // the next tile's first variable is in flight while the network runs
        const long long tn = t + tstride;
        const long long c0n = centre(tn);
        if (tn < ntiles) load_cross(c0n, 0, val[0]);
        __builtin_amdgcn_s_waitcnt(0xc07f);       // lgkmcnt(0): this wavefront's rows are written
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int ms = 0; ms < kGateTile / 16; ++ms) {
            const uint16_t* xr = row[16 * ms + r];
            f32x4 a1[4], a2[4];
            // biases of the output units this lane holds: units 16 nt + 4 g + 0..3
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) a1[nt] = *reinterpret_cast<const f32x4*>(&sb[0][16 * nt + 4 * g4]);
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                const bf16x8 x = *reinterpret_cast<const bf16x8*>(&xr[32 * kc + 8 * g4]);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    a1[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1[kc][nt], x, a1[nt], 0, 0, 0);
            }
            const bf16x8 h1[2] = {gate_hidden(a1[0], a1[1]), gate_hidden(a1[2], a1[3])};
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) a2[nt] = *reinterpret_cast<const f32x4*>(&sb[1][16 * nt + 4 * g4]);
#pragma unroll
            for (int kc = 0; kc < 2; ++kc)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    a2[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2[kc][nt], h1[kc], a2[nt], 0, 0, 0);
            const bf16x8 h2[2] = {gate_hidden(a2[0], a2[1]), gate_hidden(a2[2], a2[3])};
            // last layer: A = w3 in row 0, zero elsewhere
            f32x4 a3 = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < 2; ++kc) {
                const bf16x8 w3 = *reinterpret_cast<const bf16x8*>(&sw3[r == 0 ? 32 * kc + 8 * g4 : kHidden]);
                a3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w3, h2[kc], a3, 0, 0, 0);
            }
            const long long zz = t * kGateTile + 16 * ms + r;
            if (g4 == 0 && zz < N) {
                const float s = a3[0] + b3;
                if (flags) flags[zz] = s >= thr ? 1 : 0;
                if (logits) logits[zz] = s;
            }
        }
        c0 = c0n;
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
    }
}

// Workgroups of the inference kernel: enough tiles per wavefront to amortise
// the weight loads, at most the three workgroups per CU that are resident at
// once (166 VGPRs and 53 KB of LDS each).
inline unsigned gate_blocks(long long nzones, int cus)
{
    const long long tiles = (nzones + kGateTile - 1) / kGateTile;
    const long long want = (tiles + kGateWaves - 1) / kGateWaves;
    const long long cap = (long long)cus * 3;
    return (unsigned)(want < cap ? (want > 0 ? want : 1) : cap);
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

// Training on the matrix cores.  Layout of the per-batch arrays (nb = the
// batch rounded up to whole 256-sample chunks; samples past the batch carry
// zero gradients): BF16 arrays transposed, [row][sample], so that an MFMA
// operand fragment (four consecutive samples of one row) is one 8-byte load:
//   XT [NFP][nb] the BF16 inputs, H1T, H2T [64][nb] the BF16 hidden layers,
//   D1T, D2T [2][64][nb] the backward signals of the two hidden layers as
//   BF16 pairs hi + lo (hi = bf16(d), lo = bf16(d - hi): about 16 bits of
//   the FP32 value), dz [nb] the output signal, loss and logit [nb].
struct MlpBatch {
    uint16_t *XT, *H1T, *H2T, *D1T, *D2T;
    float *dz, *loss, *logit;
    int nb;
};

template <int NF>
struct MlpShape {
    static constexpr int NFP = (NF + 15) / 16 * 16;
    static constexpr int KC = NFP / 16;
    static constexpr int RS = (NFP > 2 * kHidden ? NFP : 2 * kHidden) + 4;   // row stride (shorts)
    static constexpr int NT1 = 4 * KC;          // 16x16 tiles of dW1
    static constexpr int NTILE = NT1 + 16;      // and of dW2
};

__device__ __forceinline__ void bf16_split(float x, uint16_t& hi, uint16_t& lo)
{
    hi = f2bf(x);
    lo = f2bf(x - bf2f(hi));
}

// Forward and backward pass of 64 samples per wavefront: per 16-sample slice
// the two hidden layers (16x16x16 BF16 MFMA, FP32 accumulation, weights as
// operand fragments in registers), the output and its loss term, the output
// signal dz = w (sigmoid(logit) - y) / n, d2 = relu'(z2) dz w3, and
// d1 = relu'(z1) (d2 W2) as two MFMA passes over d2 = hi + lo.  y = NULL:
// forward only (logits).
template <int NF>
__global__ __launch_bounds__(64) void k_mlp_fwd_bwd(const float* __restrict__ X, const float* __restrict__ y,
                                                    const float* __restrict__ cw, int n,
                                                    const float* __restrict__ prm, MlpBatch bt,
                                                    float* __restrict__ logit_out)
{
    using O = MlpOffsets<NF>;
    using S = MlpShape<NF>;
    constexpr int KC = S::KC, RS = S::RS;
    __shared__ __align__(16) uint16_t row[64][RS];
    const int lane = threadIdx.x, r = lane & 15, g4 = lane >> 4;
    const int s0 = blockIdx.x * 64;
    const bool train = y != nullptr;
    const float inv_n = 1.0f / (float)n;

    bf16x4 w1[KC][4], w2[4][4], w2t[4][4];
    float b1[4], b2[4], w3[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int col = 16 * nt + r;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int f = 16 * kc + 4 * g4 + q;
                w1[kc][nt][q] = (short)(f < NF ? f2bf(prm[O::W1 + col * NF + f]) : 0);
            }
#pragma unroll
        for (int kc = 0; kc < 4; ++kc)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 16 * kc + 4 * g4 + q;
                w2[kc][nt][q] = (short)f2bf(prm[O::W2 + col * kHidden + k]);
                w2t[kc][nt][q] = (short)f2bf(prm[O::W2 + k * kHidden + col]);
            }
        b1[nt] = prm[O::B1 + col];
        b2[nt] = prm[O::B2 + col];
        w3[nt] = bfround(prm[O::W3 + col]);
    }
    const float b3 = prm[O::B3];

    // inputs of this lane's sample, rounded to BF16 (zero past the batch)
    {
        const int s = s0 + lane;
#pragma unroll 4
        for (int f = 0; f < S::NFP; ++f) {
            const uint16_t x = (s < n && f < NF) ? f2bf(X[(long long)s * NF + f]) : (uint16_t)0;
            row[lane][f] = x;
            if (train) bt.XT[(long long)f * bt.nb + s] = x;
        }
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    for (int ms = 0; ms < 4; ++ms) {
        uint16_t(*rs)[RS] = row + 16 * ms;
        const int sr = s0 + 16 * ms + 4 * g4;          // first sample of this lane's result rows
        // layer 1
        f32x4 z1[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) z1[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            bf16x4 a;
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = (short)rs[r][16 * kc + 4 * g4 + q];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) z1[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, w1[kc][nt], z1[nt], 0, 0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                z1[nt][q] += b1[nt];
                const uint16_t h = f2bf(fmaxf(z1[nt][q], 0.0f));
                rs[4 * g4 + q][16 * nt + r] = h;
                if (train) bt.H1T[(long long)(16 * nt + r) * bt.nb + sr + q] = h;
            }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        // layer 2
        f32x4 z2[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) z2[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            bf16x4 a;
#pragma unroll
            for (int q = 0; q < 4; ++q) a[q] = (short)rs[r][16 * kc + 4 * g4 + q];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) z2[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, w2[kc][nt], z2[nt], 0, 0, 0);
        }
        // output: partial dot products over this lane's columns, summed over the 16 lanes of the row group
        float part[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            float sum = 0.0f;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                z2[nt][q] += b2[nt];
                const uint16_t h = f2bf(fmaxf(z2[nt][q], 0.0f));
                if (train) bt.H2T[(long long)(16 * nt + r) * bt.nb + sr + q] = h;
                sum += bf2f(h) * w3[nt];
            }
            part[q] = sum;
        }
#pragma unroll
        for (int m = 1; m < 16; m <<= 1)
#pragma unroll
            for (int q = 0; q < 4; ++q) part[q] += __shfl_xor(part[q], m, 16);
        float dz[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int s = sr + q;
            const float lg = b3 + part[q];
            dz[q] = 0.0f;
            if (s < n) {
                if (r == q) {
                    if (logit_out) logit_out[s] = lg;
                    if (train) bt.logit[s] = lg;
                }
                if (train) {
                    const float yy = y[s], c = cw ? cw[s] : 1.0f;
                    const float pr = 1.0f / (1.0f + expf(-lg));
                    dz[q] = c * (pr - yy) * inv_n;
                    if (r == q) bt.loss[s] = c * (fmaxf(lg, 0.0f) - lg * yy + log1pf(expf(-fabsf(lg))));
                }
            } else if (train && r == q) {
                bt.loss[s] = 0.0f;
            }
            if (train && r == q) bt.dz[s] = dz[q];
        }
        if (!train) continue;
        // d2 = relu'(z2) dz w3, written as hi / lo rows (columns 0..63 / 64..127) and transposed to memory
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float d2 = z2[nt][q] > 0.0f ? dz[q] * w3[nt] : 0.0f;
                uint16_t hi, lo;
                bf16_split(d2, hi, lo);
                const int col = 16 * nt + r;
                rs[4 * g4 + q][col] = hi;
                rs[4 * g4 + q][kHidden + col] = lo;
                bt.D2T[(long long)col * bt.nb + sr + q] = hi;
                bt.D2T[((long long)kHidden + col) * bt.nb + sr + q] = lo;
            }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        // d1 = relu'(z1) (d2 W2)
        f32x4 d1[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) d1[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int part2 = 0; part2 < 2; ++part2)
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) {
                bf16x4 a;
#pragma unroll
                for (int q = 0; q < 4; ++q) a[q] = (short)rs[r][part2 * kHidden + 16 * kc + 4 * g4 + q];
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    d1[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, w2t[kc][nt], d1[nt], 0, 0, 0);
            }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float d = z1[nt][q] > 0.0f ? d1[nt][q] : 0.0f;
                uint16_t hi, lo;
                bf16_split(d, hi, lo);
                const int col = 16 * nt + r;
                bt.D1T[(long long)col * bt.nb + sr + q] = hi;
                bt.D1T[((long long)kHidden + col) * bt.nb + sr + q] = lo;
            }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
    }
}

// Weight gradients as MFMA tiles: one wavefront per (16x16 output tile,
// chunk of 256 samples) sums dW1 = d1^T x or dW2 = d2^T h1 over its chunk
// (two passes, d = hi + lo) and stores the partial tile; k_mlp_reduce adds
// the chunks in order.
template <int NF>
__global__ __launch_bounds__(64) void k_mlp_wgrad(MlpBatch bt, float* __restrict__ partial)
{
    using S = MlpShape<NF>;
    const int lane = threadIdx.x, r = lane & 15, g4 = lane >> 4;
    const int tl = blockIdx.x, ch = blockIdx.y;
    int mt, ntl;
    const uint16_t *A, *Bm;
    if (tl < S::NT1) { mt = tl / S::KC; ntl = tl % S::KC; A = bt.D1T; Bm = bt.XT; }
    else { mt = (tl - S::NT1) / 4; ntl = (tl - S::NT1) % 4; A = bt.D2T; Bm = bt.H1T; }
    const long long nb = bt.nb;
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
    const long long c0 = (long long)ch * 256;
#pragma unroll 4
    for (int ks = 0; ks < 16; ++ks) {
        const long long s = c0 + 16 * ks + 4 * g4;
        const bf16x4 b = *reinterpret_cast<const bf16x4*>(Bm + (long long)(16 * ntl + r) * nb + s);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const bf16x4 a = *reinterpret_cast<const bf16x4*>(A + ((long long)h * kHidden + 16 * mt + r) * nb + s);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
    }
    float* out = partial + ((long long)ch * S::NTILE + tl) * 256;
#pragma unroll
    for (int q = 0; q < 4; ++q) out[(4 * g4 + q) * 16 + r] = acc[q];
}

// Gradient vector: the weight tiles summed over the chunks in order, the
// biases and the output weights by one wavefront per parameter row (lanes
// take every 64th sample, then a fixed-order tree over the lanes).
template <int NF>
__global__ __launch_bounds__(64) void k_mlp_reduce(MlpBatch bt, const float* __restrict__ partial, int nchunk,
                                                   float* __restrict__ grad)
{
    using O = MlpOffsets<NF>;
    using S = MlpShape<NF>;
    const int lane = threadIdx.x;
    const int b = blockIdx.x;
    const int nwt = (S::NTILE * 256 + 63) / 64;      // blocks for the weight tiles
    if (b < nwt) {
        const int e = b * 64 + lane;                  // element of the tile set
        if (e >= S::NTILE * 256) return;
        const int tl = e / 256, w = e % 256, i = w / 16, j = w % 16;
        float sum = 0.0f;
        for (int c = 0; c < nchunk; ++c) sum += partial[((long long)c * S::NTILE + tl) * 256 + w];
        if (tl < S::NT1) {
            const int o = 16 * (tl / S::KC) + i, f = 16 * (tl % S::KC) + j;
            if (f < NF) grad[O::W1 + o * NF + f] = sum;
        } else {
            const int t2 = tl - S::NT1;
            const int o = 16 * (t2 / 4) + i, q = 16 * (t2 % 4) + j;
            grad[O::W2 + o * kHidden + q] = sum;
        }
        return;
    }
    const int rrow = b - nwt;                          // 0..63 b1, 64..127 b2, 128..191 w3, 192 b3
    const long long nb = bt.nb;
    float sum = 0.0f;
    for (long long s = lane; s < nb; s += 64) {
        if (rrow < 64) sum += bf2f(bt.D1T[rrow * nb + s]) + bf2f(bt.D1T[(kHidden + rrow) * nb + s]);
        else if (rrow < 128) sum += bf2f(bt.D2T[(rrow - 64) * nb + s]) + bf2f(bt.D2T[(kHidden + rrow - 64) * nb + s]);
        else if (rrow < 192) sum += bt.dz[s] * bf2f(bt.H2T[(rrow - 128) * nb + s]);
        else sum += bt.dz[s];
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) sum += __shfl_xor(sum, m, 64);
    if (lane == 0) {
        if (rrow < 64) grad[O::B1 + rrow] = sum;
        else if (rrow < 128) grad[O::B2 + rrow - 64] = sum;
        else if (rrow < 192) grad[O::W3 + rrow - 128] = sum;
        else grad[O::B3] = sum;
    }
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

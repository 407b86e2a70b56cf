// hog_physics.h -- pointwise device routines of the ADER-WENO Euler update:
// equation of state, physical fluxes, Riemann solvers and the 1D WENO
// operator.  These are the "routine seq" pieces of the paper's structure
// (Sec. II.2: Predictor_Ptwise, Riemann_Solver_Ptwise, Eval_Tstep_Ptwise),
// written as inlined device functions on registers.
#pragma once
#include <hip/hip_runtime.h>

namespace hog {

struct WenoArgs {
    double eps;      // epsilon of the nonlinear weights
    double g[4];     // O3: (L, C, R, -); O4: (H, L, C, R)
    int linear;      // 1: weights fixed to the linear ones
};

// The device routines below are templates on the arithmetic type T: double
// on the FP64 path, float where the mixed path computes in FP32.


// Physical fluxes of the Euler equations along all D axes at one point;
// returns whether the state is admissible (rho > 0, p > 0, finite).
// FP64 reciprocal from the hardware estimate refined by two Newton steps
// r <- r + r (1 - x r) (within a few ulp of 1/x; 0, negative or non-finite x
// give a non-finite or negative result, which the admissibility check below
// rejects).  Used for the FP64 fluxes of the predictor, the FP64 Riemann
// solvers and the nonlinear WENO weights (whose denominators are at least
// eps^2 > 0).  FP32 keeps the correctly rounded division, which measured
// faster in the FP32 predictor.
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float recip(float x) { return 1.0f / x; }

template <int D, typename T = double>
__device__ __forceinline__ bool fluxes(const T* U, T gm1, T (*F)[D + 2])
{
    const T rho = U[0];
    const T ir = recip(rho);
    T u[D];
    T ke = T(0);
#pragma unroll
    for (int d = 0; d < D; ++d) { u[d] = U[1 + d] * ir; ke += U[1 + d] * u[d]; }
    const T p = gm1 * (U[D + 1] - T(0.5) * ke);
    const T Ep = U[D + 1] + p;
    // momentum fluxes m_k m_d / rho + p delta_kd: the off-diagonal product is
    // shared by the two axes that need it
#pragma unroll
    for (int d = 0; d < D; ++d) {
        F[d][0] = U[1 + d];
        F[d][1 + d] = U[1 + d] * u[d] + p;
#pragma unroll
        for (int k = 0; k < d; ++k) {
            F[d][1 + k] = U[1 + k] * u[d];
            F[k][1 + d] = F[d][1 + k];
        }
        F[d][D + 1] = Ep * u[d];
    }
    return rho > T(0) && p > T(0) && isfinite(rho) && isfinite(p);
}

// FP32 reciprocal from the hardware estimate (1 ulp) refined by one Newton
// step: three instructions instead of the correctly rounded division's ten.
__device__ __forceinline__ float recip_nr(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double recip_nr(double x) { return recip(x); }

// a / b: the division, or with RCP a times the Newton-refined reciprocal of b
// (a few ulp instead of correctly rounded, about half the instructions of an
// FP64 division and a third of an FP32 one).
template <bool RCP, typename T>
__device__ __forceinline__ T dv(T a, T b)
{
    if constexpr (RCP) return a * recip_nr(b);
    else return a / b;
}

// Square root: with RCP in FP32 the hardware one (1 ulp instead of the
// correctly rounded sequence); FP64 always correctly rounded.
template <bool RCP, typename T>
__device__ __forceinline__ T root(T x)
{
    if constexpr (RCP && sizeof(T) == 4) return __builtin_amdgcn_sqrtf(x);
    else return sqrt(x);
}

// Pressure of an ideal gas from the conserved variables of D dimensions.
template <int D, typename T = double, bool RCP = false>
__device__ __forceinline__ T pressure(const T* U, T gm1)
{
    T ke = T(0);
#pragma unroll
    for (int d = 0; d < D; ++d) ke += U[1 + d] * U[1 + d];
    return gm1 * (U[D + 1] - dv<RCP>(T(0.5) * ke, U[0]));
}

// rho > 0, p > 0 and both finite.
template <int D, typename T = double, bool RCP = false>
__device__ __forceinline__ bool admissible(const T* U, T gm1)
{
    const T p = pressure<D, T, RCP>(U, gm1);
    return U[0] > T(0) && p > T(0) && isfinite(U[0]) && isfinite(p);
}

// Flux of one axis.
template <int D, typename T = double, bool RCP = false>
__device__ __forceinline__ void flux_dir(const T* U, T gm1, int dir, T* F, T& p, T& un)
{
    const T ir = dv<RCP>(T(1), U[0]);
    T ke = T(0);
#pragma unroll
    for (int d = 0; d < D; ++d) ke += U[1 + d] * U[1 + d];
    p = gm1 * (U[D + 1] - T(0.5) * ke * ir);
    un = U[1 + dir] * ir;
    F[0] = U[1 + dir];
#pragma unroll
    for (int k = 0; k < D; ++k) F[1 + k] = U[1 + k] * un + (k == dir ? p : T(0));
    F[D + 1] = (U[D + 1] + p) * un;
}

// Riemann solvers at a face with normal axis dir.  solver: 0 HLLC, 1 HLL,
// 2 Rusanov, 3 HLLEM, 4 HLLI (the solvers Sec. I.1 favours for their small
// operation count and cache use; Fig. 5 builds HLL/HLLEM fluxes).
// HLLC follows Toro, Spruce and Speares with Einfeldt wave-speed bounds built
// from Roe averages; branch ties resolved as S_L >= 0 -> left, S* >= 0 -> left
// star, S_R > 0 -> right star, else right.
// HLLEM (Einfeldt) and HLLI (Dumbser and Balsara) take the HLL flux and remove
// the part of its dissipation that falls on the linearly degenerate waves of
// Roe's linearisation: the entropy wave of strength drho - dp / c~^2 along
// (1, u~, |u~|^2 / 2) and one shear wave per tangential axis t of strength
// rho~ du_t (rho~ = sqrt(rho_L rho_R)) along (0, e_t, u~_t), scaled by
// delta = c~ / (c~ + |u~_n|) (HLLEM) or 1 - min(u~_n, 0)/S_L - max(u~_n, 0)/S_R
// (HLLI, which makes an isolated moving contact exact).
// RCP: divisions as products with Newton-refined reciprocals (see dv).
template <int D, typename T = double, bool RCP = false>
__device__ __forceinline__ void riemann(const T* UL, const T* UR, int dir, int solver, T gamma, T* F)
{
    constexpr int NV = D + 2;
    const T gm1 = gamma - T(1);
    T FL[NV], FR[NV], pL, pR, uL, uR;
    flux_dir<D, T, RCP>(UL, gm1, dir, FL, pL, uL);
    flux_dir<D, T, RCP>(UR, gm1, dir, FR, pR, uR);
    const T rL = UL[0], rR = UR[0];
    const T cL = root<RCP>(dv<RCP>(gamma * pL, rL)), cR = root<RCP>(dv<RCP>(gamma * pR, rR));
    if (solver == 2) {
        const T s = fmax(fabs(uL) + cL, fabs(uR) + cR);
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] = T(0.5) * (FL[v] + FR[v]) - T(0.5) * s * (UR[v] - UL[v]);
        return;
    }
    const T sL = root<RCP>(rL), sR = root<RCP>(rR);
    const T isum = dv<RCP>(T(1), sL + sR);
    const T HL = dv<RCP>(UL[NV - 1] + pL, rL), HR = dv<RCP>(UR[NV - 1] + pR, rR);
    T q2 = T(0), utn = T(0), ut[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        ut[d] = (dv<RCP>(UL[1 + d], sL) + dv<RCP>(UR[1 + d], sR)) * isum;
        q2 += ut[d] * ut[d];
        if (d == dir) utn = ut[d];
    }
    const T Ht = (sL * HL + sR * HR) * isum;
    const T ct = root<RCP>(gm1 * (Ht - T(0.5) * q2));
    const T SL = fmin(uL - cL, utn - ct);
    const T SR = fmax(uR + cR, utn + ct);
    if (solver == 1 || solver >= 3) {
        if (SL >= T(0)) {
#pragma unroll
            for (int v = 0; v < NV; ++v) F[v] = FL[v];
        } else if (SR <= T(0)) {
#pragma unroll
            for (int v = 0; v < NV; ++v) F[v] = FR[v];
        } else {
            const T id = dv<RCP>(T(1), SR - SL);
#pragma unroll
            for (int v = 0; v < NV; ++v) F[v] = (SR * FL[v] - SL * FR[v] + SL * SR * (UR[v] - UL[v])) * id;
            if (solver >= 3) {
                // degenerate-wave content of the jump, from primitive jumps
                const T ae = (rR - rL) - dv<RCP>(pR - pL, ct * ct);
                const T rt = sL * sR;
                const T irL = dv<RCP>(T(1), rL), irR = dv<RCP>(T(1), rR);
                T J[NV];
                J[0] = ae;
                J[NV - 1] = T(0.5) * ae * q2;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    J[1 + d] = ae * ut[d];
                    if (d != dir) {
                        const T at = rt * (UR[1 + d] * irR - UL[1 + d] * irL);
                        J[1 + d] += at;
                        J[NV - 1] += at * ut[d];
                    }
                }
                const T delta = (solver == 3) ? dv<RCP>(ct, ct + fabs(utn))
                                              : T(1) - dv<RCP>(fmin(utn, T(0)), SL) - dv<RCP>(fmax(utn, T(0)), SR);
                const T k = SL * SR * id * delta;
#pragma unroll
                for (int v = 0; v < NV; ++v) F[v] -= k * J[v];
            }
        }
        return;
    }
    const T mL = rL * (SL - uL), mR = rR * (SR - uR);
    const T Ss = dv<RCP>(pR - pL + mL * uL - mR * uR, mL - mR);
    if (SL >= T(0)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] = FL[v];
        return;
    }
    // in the order S_L >= 0, S* >= 0, S_R > 0, else the right flux (a NaN speed
    // fails every test and falls through to the right flux)
    const bool left = Ss >= T(0);
    if (!left && !(SR > T(0))) {
#pragma unroll
        for (int v = 0; v < NV; ++v) F[v] = FR[v];
        return;
    }
    // star state on the side the contact leaves behind
    const T* Uk = left ? UL : UR;
    const T* Fk = left ? FL : FR;
    const T Sk = left ? SL : SR;
    const T rk = left ? rL : rR;
    const T uk = left ? uL : uR;
    const T pk = left ? pL : pR;
    const T mk = left ? mL : mR;
    const T f = dv<RCP>(mk, Sk - Ss);
    const T irk = dv<RCP>(T(1), rk);
    T Us[NV];
    Us[0] = f;
#pragma unroll
    for (int d = 0; d < D; ++d) Us[1 + d] = f * (d == dir ? Ss : Uk[1 + d] * irk);
    Us[NV - 1] = f * (Uk[NV - 1] * irk + (Ss - uk) * (Ss + dv<RCP>(pk, mk)));
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v] = Fk[v] + Sk * (Us[v] - Uk[v]);
}

// 1D WENO operator on five zone averages v[0..4] (offsets -2..2): returns the
// undivided Legendre coefficients c[1..P] of the zone polynomial.  P = 2:
// convex combination of the three quadratics; P = 3: WENO-AO combination of
// the cubic truncation of the centred quartic fit with the three quadratics.
template <int P>
__device__ __forceinline__ void weno1d(const double* v, double* c, const WenoArgs& wa)
{
    // quadratic candidates on {-2,-1,0}, {-1,0,1}, {0,1,2}
    const double l1 = 0.5 * v[0] - 2.0 * v[1] + 1.5 * v[2];
    const double l2 = 0.5 * v[0] - v[1] + 0.5 * v[2];
    const double m1 = 0.5 * (v[3] - v[1]);
    const double m2 = 0.5 * v[1] - v[2] + 0.5 * v[3];
    const double r1 = -1.5 * v[2] + 2.0 * v[3] - 0.5 * v[4];
    const double r2 = 0.5 * v[2] - v[3] + 0.5 * v[4];
    constexpr double k13_3 = 13.0 / 3.0;
    if constexpr (P == 2) {
        double wL = wa.g[0], wC = wa.g[1], wR = wa.g[2];
        if (!wa.linear) {
            const double bL = wa.eps + (l1 * l1 + k13_3 * l2 * l2);
            const double bC = wa.eps + (m1 * m1 + k13_3 * m2 * m2);
            const double bR = wa.eps + (r1 * r1 + k13_3 * r2 * r2);
            const double aL = wa.g[0] * recip(bL * bL), aC = wa.g[1] * recip(bC * bC),
                         aR = wa.g[2] * recip(bR * bR);
            const double is = recip(aL + aC + aR);
            wL = aL * is; wC = aC * is; wR = aR * is;
        }
        c[1] = wL * l1 + wC * m1 + wR * r1;
        c[2] = wL * l2 + wC * m2 + wR * r2;
    } else {
        const double h1 = (11.0 * (v[0] - v[4]) + 82.0 * (v[3] - v[1])) * (1.0 / 120.0);
        const double h2 = (-3.0 * (v[0] + v[4]) + 40.0 * (v[1] + v[3]) - 74.0 * v[2]) * (1.0 / 56.0);
        const double h3 = ((v[4] - v[0]) + 2.0 * (v[1] - v[3])) * (1.0 / 12.0);
        const double gH = wa.g[0], gL = wa.g[1], gC = wa.g[2], gR = wa.g[3];
        double wH = gH, wL = gL, wC = gC, wR = gR;
        if (!wa.linear) {
            const double s1 = h1 + 0.1 * h3;
            const double bH = wa.eps + (s1 * s1 + k13_3 * h2 * h2 + (781.0 / 20.0) * h3 * h3);
            const double bL = wa.eps + (l1 * l1 + k13_3 * l2 * l2);
            const double bC = wa.eps + (m1 * m1 + k13_3 * m2 * m2);
            const double bR = wa.eps + (r1 * r1 + k13_3 * r2 * r2);
            const double aH = gH * recip(bH * bH), aL = gL * recip(bL * bL), aC = gC * recip(bC * bC),
                         aR = gR * recip(bR * bR);
            const double is = recip(aH + aL + aC + aR);
            wH = aH * is; wL = aL * is; wC = aC * is; wR = aR * is;
        }
        const double r = wH * recip(gH);
        c[1] = r * (h1 - gL * l1 - gC * m1 - gR * r1) + wL * l1 + wC * m1 + wR * r1;
        c[2] = r * (h2 - gL * l2 - gC * m2 - gR * r2) + wL * l2 + wC * m2 + wR * r2;
        c[3] = r * h3;
    }
}

// Mixed-precision 1D WENO: the candidate coefficients are formed from FP64
// stencil differences and rounded to FP32; the smoothness indicators, the
// epsilon division and the nonlinear weights are FP64 (from the FP32
// candidates); the weights are rounded to FP32 for the FP32 combination.
template <int P>
__device__ __forceinline__ void weno1d_mixed(const double* v, float* c, const WenoArgs& wa)
{
    const float l1 = (float)(0.5 * v[0] - 2.0 * v[1] + 1.5 * v[2]);
    const float l2 = (float)(0.5 * v[0] - v[1] + 0.5 * v[2]);
    const float m1 = (float)(0.5 * (v[3] - v[1]));
    const float m2 = (float)(0.5 * v[1] - v[2] + 0.5 * v[3]);
    const float r1 = (float)(-1.5 * v[2] + 2.0 * v[3] - 0.5 * v[4]);
    const float r2 = (float)(0.5 * v[2] - v[3] + 0.5 * v[4]);
    constexpr double k13_3 = 13.0 / 3.0;
    auto is2 = [](float a, float b) { const double x = a, y = b; return x * x + k13_3 * y * y; };
    if constexpr (P == 2) {
        float wL = (float)wa.g[0], wC = (float)wa.g[1], wR = (float)wa.g[2];
        if (!wa.linear) {
            const double bL = wa.eps + is2(l1, l2), bC = wa.eps + is2(m1, m2), bR = wa.eps + is2(r1, r2);
            const double aL = wa.g[0] * recip(bL * bL), aC = wa.g[1] * recip(bC * bC),
                         aR = wa.g[2] * recip(bR * bR);
            const double is = recip(aL + aC + aR);
            wL = (float)(aL * is); wC = (float)(aC * is); wR = (float)(aR * is);
        }
        c[1] = wL * l1 + wC * m1 + wR * r1;
        c[2] = wL * l2 + wC * m2 + wR * r2;
    } else {
        const float h1 = (float)((11.0 * (v[0] - v[4]) + 82.0 * (v[3] - v[1])) * (1.0 / 120.0));
        const float h2 = (float)((-3.0 * (v[0] + v[4]) + 40.0 * (v[1] + v[3]) - 74.0 * v[2]) * (1.0 / 56.0));
        const float h3 = (float)(((v[4] - v[0]) + 2.0 * (v[1] - v[3])) * (1.0 / 12.0));
        const double gH = wa.g[0];
        float wH = (float)wa.g[0], wL = (float)wa.g[1], wC = (float)wa.g[2], wR = (float)wa.g[3];
        double ratio = 1.0;
        if (!wa.linear) {
            const double s1 = (double)h1 + 0.1 * (double)h3;
            const double bH = wa.eps + (s1 * s1 + k13_3 * (double)h2 * h2 + (781.0 / 20.0) * (double)h3 * h3);
            const double bL = wa.eps + is2(l1, l2), bC = wa.eps + is2(m1, m2), bR = wa.eps + is2(r1, r2);
            const double aH = gH * recip(bH * bH), aL = wa.g[1] * recip(bL * bL), aC = wa.g[2] * recip(bC * bC),
                         aR = wa.g[3] * recip(bR * bR);
            const double is = recip(aH + aL + aC + aR);
            ratio = aH * is * recip(gH);
            wL = (float)(aL * is); wC = (float)(aC * is); wR = (float)(aR * is);
            wH = (float)(aH * is);
        }
        (void)wH;
        const float r = (float)ratio;
        const float gL = (float)wa.g[1], gC = (float)wa.g[2], gR = (float)wa.g[3];
        c[1] = r * (h1 - gL * l1 - gC * m1 - gR * r1) + wL * l1 + wC * m1 + wR * r1;
        c[2] = r * (h2 - gL * l2 - gC * m2 - gR * r2) + wL * l2 + wC * m2 + wR * r2;
        c[3] = r * h3;
    }
}

} // namespace hog

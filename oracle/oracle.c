/*
 * oracle.c -- plain, slow FP64 CPU reference of one ADER-WENO time step for
 * the 2D/3D compressible Euler equations of an ideal gas.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load or call this library.  It shares
 * no code, header, table or constant generator with the GPU library.
 *
 * What it computes (paper, Sec. I.1 and Sec. II.2, Fig. 1): per time step
 *   (1) ghost zones (Fig. 1, Boundary_Conditions),
 *   (2) WENO reconstruction of the conserved variables in every zone
 *       (Sec. I.1: reconstruction done directly on the conserved variables),
 *   (3) an ADER predictor that extends the zone polynomial in time
 *       (Sec. I.1, Fig. 4 Predictor / Predictor_Ptwise),
 *   (4) a Riemann-solver flux at the faces from the predicted space-time
 *       polynomials (Fig. 5 Make_Flux_X, HLLC / HLL / Rusanov),
 *   (5) the conservative flux-difference update (Fig. 6 Make_dU_dt and
 *       Fig. 7 Update_U_Timestep),
 *   (6) the CFL time step of the new state with a min over zones (Fig. 7).
 * The paper prints the scheme only at second order with the predictor and
 * Riemann solver left empty; the second-order path follows Figs. 3-7 with the
 * pointwise predictor read as a Hancock step; the third/fourth order formulas here are the
 * readings stated in the design notes (successive x->y->z WENO sweeps with
 * L/C/R quadratic candidates at O3 and a WENO-AO combination at O4, a Picard
 * predictor with tensor Gauss-Legendre L2 projection, 2-point Gauss face
 * quadrature in the face directions and in time).
 *
 * Besides the one-step ADER update, the oracle takes the Runge-Kutta steppers
 * the paper compares against (Sec. I.1, Table IV): the same reconstruction and
 * Riemann solver per stage with face points in space only, combined in
 * Shu-Osher form (rk_step below).
 *
 * Everything is written in the most direct form: polynomials are evaluated
 * mode by mode, projections are sums over all quadrature nodes, and the
 * derivative / time-integral maps are applied term by term.  No blocking,
 * sum factorisation or fusion.
 *
 * Parity pins (tests/test_oracle_*.py) tie every function to closed forms,
 * exactness properties and exact solutions, not to this file.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#define OG 3            /* ghost width: reconstruction radius 2 + one face neighbour */
#define MAXP 3
#define MAXV 5
#define MAXST 35        /* space-time modes at d=3, p=3 */
#define MAXNODE 256     /* (p+1)^(d+1) at d=3, p=3 */

/* Configuration, mirrored by a ctypes.Structure in oracle/oracle.py. */
typedef struct {
    int ndim;          /* 2 or 3 */
    int nx, ny, nz;    /* interior zones; nz = 1 in 2D */
    int order;         /* 2 (the scheme of Figs. 3-7), 3 or 4: polynomial degree p = order - 1 */
    int riemann;       /* 0 HLLC, 1 HLL, 2 Rusanov, 3 HLLEM, 4 HLLI */
    int bc[3];         /* per axis: 0 periodic, 1 outflow (zero gradient) */
    int linear_weno;   /* 1: nonlinear weights replaced by the linear ones */
    int positivity;    /* 1: first-order fallback in zones with an inadmissible predicted state */
    double gamma;
    double dx, dy, dz;
    double cfl;
    double weno_eps;   /* epsilon in omega~ = gamma_k / (eps + IS_k)^2 */
    double g3[3];      /* O3 linear weights for the L, C, R quadratics */
    double g4[4];      /* O4 linear weights for the H (cubic), L, C, R members */
    int stepper;       /* 0 ADER (the predictor / Hancock step); 2, 3, 4: SSP-RK with 2, 3, 5 stages */
    int char_recon;    /* 1: WENO on characteristic variables (orders 3 and 4) */
} ocfg;

/* ------------------------------------------------------------------------ */
/* 1D bases on the reference zone                                            */
/* ------------------------------------------------------------------------ */

/* Zero-mean orthogonal Legendre polynomials on [-1/2, 1/2]. */
static double leg(int a, double x)
{
    switch (a) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return x * x - 1.0 / 12.0;
    default: return x * x * x - 0.15 * x;
    }
}
/* int_{-1/2}^{1/2} leg(a)^2 */
static double leg_norm(int a)
{
    static const double n[4] = {1.0, 1.0 / 12.0, 1.0 / 180.0, 1.0 / 2800.0};
    return n[a];
}
/* d/dx leg(a) = sum_{a'} dleg(a, a') leg(a'):  P1' = P0, P2' = 2 P1,
 * P3' = 3 x^2 - 3/20 = 3 P2 + (3/12 - 3/20) P0 = 3 P2 + P0 / 10. */
static double dleg(int a, int ap)
{
    if (a == 1 && ap == 0) return 1.0;
    if (a == 2 && ap == 1) return 2.0;
    if (a == 3 && ap == 2) return 3.0;
    if (a == 3 && ap == 0) return 0.1;
    return 0.0;
}
/* Shifted Legendre polynomials on [0, 1] (time projection basis). */
static double sleg(int e, double t)
{
    switch (e) {
    case 0: return 1.0;
    case 1: return 2.0 * t - 1.0;
    case 2: return 6.0 * t * t - 6.0 * t + 1.0;
    default: return 20.0 * t * t * t - 30.0 * t * t + 12.0 * t - 1.0;
    }
}
static double sleg_norm(int e) { return 1.0 / (2.0 * e + 1.0); }
/* int_0^tau sleg(e) = sum_{e'} tint(e, e') tau^e'. */
static double tint(int e, int ep)
{
    static const double T[4][5] = {
        {0, 1, 0, 0, 0},          /* tau */
        {0, -1, 1, 0, 0},         /* tau^2 - tau */
        {0, 1, -3, 2, 0},         /* 2 tau^3 - 3 tau^2 + tau */
        {0, -1, 6, -10, 5},       /* 5 tau^4 - 10 tau^3 + 6 tau^2 - tau */
    };
    return T[e][ep];
}
static double ipow(double t, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= t;
    return r;
}

/* Gauss-Legendre rule with n = 2, 3, 4 points on [-1/2, 1/2] (weights sum to 1),
 * from the closed forms of the roots of the Legendre polynomials on [-1, 1]. */
static void gauss(int n, double *x, double *w)
{
    if (n == 2) {
        double a = 1.0 / sqrt(3.0);
        x[0] = -a; x[1] = a; w[0] = w[1] = 1.0;
    } else if (n == 3) {
        double a = sqrt(3.0 / 5.0);
        x[0] = -a; x[1] = 0.0; x[2] = a;
        w[0] = w[2] = 5.0 / 9.0; w[1] = 8.0 / 9.0;
    } else {
        double r = 2.0 / 7.0 * sqrt(6.0 / 5.0);
        double a = sqrt(3.0 / 7.0 - r), b = sqrt(3.0 / 7.0 + r);
        double wa = (18.0 + sqrt(30.0)) / 36.0, wb = (18.0 - sqrt(30.0)) / 36.0;
        x[0] = -b; x[1] = -a; x[2] = a; x[3] = b;
        w[0] = wb; w[1] = wa; w[2] = wa; w[3] = wb;
    }
    for (int i = 0; i < n; ++i) { x[i] *= 0.5; w[i] *= 0.5; }
}

/* ------------------------------------------------------------------------ */
/* Mode lists                                                                */
/* ------------------------------------------------------------------------ */
/* Space-time modes (a, b, c, e) with a+b+c+e <= p, enumerated e outermost,
 * then c, then b, then a; in 2D c = 0.  The e = 0 block is the spatial list. */
typedef struct { int a, b, c, e; } mode4;

static int st_modes(int ndim, int p, mode4 *m)
{
    int n = 0;
    int cmax = (ndim == 3) ? p : 0;
    for (int e = 0; e <= p; ++e)
        for (int c = 0; c <= cmax; ++c)
            for (int b = 0; b <= p; ++b)
                for (int a = 0; a <= p; ++a)
                    if (a + b + c + e <= p) { m[n].a = a; m[n].b = b; m[n].c = c; m[n].e = e; ++n; }
    return n;
}
static int find_mode(const mode4 *m, int n, int a, int b, int c, int e)
{
    for (int i = 0; i < n; ++i)
        if (m[i].a == a && m[i].b == b && m[i].c == c && m[i].e == e) return i;
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Equation of state and physical fluxes                                     */
/* ------------------------------------------------------------------------ */
static double pressure(const ocfg *c, const double *U)
{
    int nv = c->ndim + 2;
    double rho = U[0], ke = 0.0;
    for (int d = 0; d < c->ndim; ++d) ke += U[1 + d] * U[1 + d];
    ke = 0.5 * ke / rho;
    return (c->gamma - 1.0) * (U[nv - 1] - ke);
}

/* A state the Euler fluxes are defined for: rho > 0, p > 0, both finite. */
static int admissible(const ocfg *c, const double *U)
{
    double p = pressure(c, U);
    return U[0] > 0.0 && p > 0.0 && isfinite(U[0]) && isfinite(p);
}

/* Physical flux of the Euler equations along axis dir. */
static void phys_flux(const ocfg *c, int dir, const double *U, double *F)
{
    int nd = c->ndim, nv = nd + 2;
    double rho = U[0];
    double un = U[1 + dir] / rho;
    double p = pressure(c, U);
    F[0] = U[1 + dir];
    for (int d = 0; d < nd; ++d) F[1 + d] = U[1 + d] * un + (d == dir ? p : 0.0);
    F[nv - 1] = (U[nv - 1] + p) * un;
}

/* ------------------------------------------------------------------------ */
/* Riemann solvers (paper Sec. I.1 lists Rusanov, HLL, HLLC, HLLI as the     */
/* favoured low-cache solvers; Fig. 5 calls one per face point).             */
/* ------------------------------------------------------------------------ */
void oracle_riemann(const ocfg *c, int dir, const double *UL, const double *UR, double *F)
{
    int nd = c->ndim, nv = nd + 2;
    double g = c->gamma;
    double FL[MAXV], FR[MAXV];
    phys_flux(c, dir, UL, FL);
    phys_flux(c, dir, UR, FR);
    double rL = UL[0], rR = UR[0];
    double pL = pressure(c, UL), pR = pressure(c, UR);
    double uL = UL[1 + dir] / rL, uR = UR[1 + dir] / rR;
    double cL = sqrt(g * pL / rL), cR = sqrt(g * pR / rR);

    if (c->riemann == 2) { /* Rusanov */
        double s = fmax(fabs(uL) + cL, fabs(uR) + cR);
        for (int v = 0; v < nv; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * s * (UR[v] - UL[v]);
        return;
    }
    /* Einfeldt wave-speed bounds from Roe averages. */
    double sL = sqrt(rL), sR = sqrt(rR);
    double HL = (UL[nv - 1] + pL) / rL, HR = (UR[nv - 1] + pR) / rR;
    double vel2 = 0.0, ut_n = 0.0;
    for (int d = 0; d < nd; ++d) {
        double ut = (sL * UL[1 + d] / rL + sR * UR[1 + d] / rR) / (sL + sR);
        vel2 += ut * ut;
        if (d == dir) ut_n = ut;
    }
    double Ht = (sL * HL + sR * HR) / (sL + sR);
    double ct = sqrt((g - 1.0) * (Ht - 0.5 * vel2));
    double SL = fmin(uL - cL, ut_n - ct);
    double SR = fmax(uR + cR, ut_n + ct);

    if (c->riemann == 1 || c->riemann == 3 || c->riemann == 4) { /* HLL, HLLEM, HLLI */
        if (SL >= 0.0) { for (int v = 0; v < nv; ++v) F[v] = FL[v]; return; }
        if (SR <= 0.0) { for (int v = 0; v < nv; ++v) F[v] = FR[v]; return; }
        for (int v = 0; v < nv; ++v)
            F[v] = (SR * FL[v] - SL * FR[v] + SL * SR * (UR[v] - UL[v])) / (SR - SL);
        if (c->riemann == 1) return;
        /* HLLEM (Einfeldt) and HLLI (Dumbser and Balsara): the HLL flux minus
         * part of its dissipation in the linearly degenerate fields (the
         * entropy wave and the nd-1 shear waves).  The jump is split on the
         * right eigenvectors of Roe's matrix: with Roe velocity ut, enthalpy
         * Ht and sound speed ct,
         *   entropy wave  r = (1, ut, |ut|^2/2),
         *                 alpha = (g-1)/ct^2 (drho (Ht - |ut|^2) + ut . dm - dE),
         *   shear wave t  r = (0, e_t, ut_t),  alpha = dm_t - ut_t drho,
         * the rows of the inverse eigenvector matrix that belong to these
         * fields.  The anti-diffusion factor delta in [0, 1] is
         *   HLLEM: ct / (ct + |ut_n|)                (1 for a resting contact),
         *   HLLI:  1 - min(ut_n, 0)/SL - max(ut_n, 0)/SR
         * (an isolated contact moving at ut_n is then resolved exactly). */
        double ut[3] = {0.0, 0.0, 0.0}, dU[MAXV] = {0.0};
        for (int d = 0; d < nd; ++d) ut[d] = (sL * UL[1 + d] / rL + sR * UR[1 + d] / rR) / (sL + sR);
        for (int v = 0; v < nv; ++v) dU[v] = UR[v] - UL[v];
        double udm = 0.0;
        for (int d = 0; d < nd; ++d) udm += ut[d] * dU[1 + d];
        double a_e = (g - 1.0) / (ct * ct) * (dU[0] * (Ht - vel2) + udm - dU[nv - 1]);
        double proj[MAXV];
        proj[0] = a_e;
        for (int d = 0; d < nd; ++d) proj[1 + d] = a_e * ut[d];
        proj[nv - 1] = a_e * 0.5 * vel2;
        for (int d = 0; d < nd; ++d) {
            if (d == dir) continue;
            double a_t = dU[1 + d] - ut[d] * dU[0];
            proj[1 + d] += a_t;
            proj[nv - 1] += a_t * ut[d];
        }
        double delta = (c->riemann == 3) ? ct / (ct + fabs(ut_n))
                                         : 1.0 - fmin(ut_n, 0.0) / SL - fmax(ut_n, 0.0) / SR;
        double k = SL * SR / (SR - SL) * delta;
        for (int v = 0; v < nv; ++v) F[v] -= k * proj[v];
        return;
    }
    /* HLLC (Toro, Spruce and Speares): contact speed and star states. */
    double Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR))
              / (rL * (SL - uL) - rR * (SR - uR));
    if (SL >= 0.0) { for (int v = 0; v < nv; ++v) F[v] = FL[v]; return; }
    if (Ss >= 0.0) {
        double f = rL * (SL - uL) / (SL - Ss);
        double Us[MAXV];
        Us[0] = f;
        for (int d = 0; d < nd; ++d) Us[1 + d] = f * (d == dir ? Ss : UL[1 + d] / rL);
        Us[nv - 1] = f * (UL[nv - 1] / rL + (Ss - uL) * (Ss + pL / (rL * (SL - uL))));
        for (int v = 0; v < nv; ++v) F[v] = FL[v] + SL * (Us[v] - UL[v]);
        return;
    }
    if (SR > 0.0) {
        double f = rR * (SR - uR) / (SR - Ss);
        double Us[MAXV];
        Us[0] = f;
        for (int d = 0; d < nd; ++d) Us[1 + d] = f * (d == dir ? Ss : UR[1 + d] / rR);
        Us[nv - 1] = f * (UR[nv - 1] / rR + (Ss - uR) * (Ss + pR / (rR * (SR - uR))));
        for (int v = 0; v < nv; ++v) F[v] = FR[v] + SR * (Us[v] - UR[v]);
        return;
    }
    for (int v = 0; v < nv; ++v) F[v] = FR[v];
}

void oracle_phys_flux(const ocfg *c, int dir, const double *U, double *F) { phys_flux(c, dir, U, F); }

/* ------------------------------------------------------------------------ */
/* 1D WENO operator R_p on a line of five zone averages v[-2..2]             */
/* ------------------------------------------------------------------------ */
/* Output c[1..p] are the undivided Legendre coefficients of the zone
 * polynomial c0 + c1 P1 + ... + cp Pp; the mean c0 = v0 is untouched. */
/* linear: use the linear weights; dev (may be NULL): receives
 * max_k |omega_k / gamma_k - 1| of the nonlinear weights (the smoothness
 * measure the learned gate is trained to predict). */
static void weno1d_core(const ocfg *cf, int p, const double *v5, int linear, double *out, double *dev)
{
    const double *v = v5 + 2;   /* v[-2..2] */
    /* Quadratic candidates reproducing the averages of {-2,-1,0}, {-1,0,1}, {0,1,2}. */
    double L1 = 0.5 * (v[-2] - 4.0 * v[-1] + 3.0 * v[0]);
    double L2 = 0.5 * (v[-2] - 2.0 * v[-1] + v[0]);
    double C1 = 0.5 * (v[1] - v[-1]);
    double C2 = 0.5 * (v[-1] - 2.0 * v[0] + v[1]);
    double R1 = 0.5 * (-3.0 * v[0] + 4.0 * v[1] - v[2]);
    double R2 = 0.5 * (v[0] - 2.0 * v[1] + v[2]);
    /* Smoothness indicators: sum over derivative orders l >= 1 of int (d^l p)^2. */
    double ISL = L1 * L1 + 13.0 / 3.0 * L2 * L2;
    double ISC = C1 * C1 + 13.0 / 3.0 * C2 * C2;
    double ISR = R1 * R1 + 13.0 / 3.0 * R2 * R2;
    double eps = cf->weno_eps;
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (p == 2) {
        double wL, wC, wR;
        double aL = cf->g3[0] / ((eps + ISL) * (eps + ISL));
        double aC = cf->g3[1] / ((eps + ISC) * (eps + ISC));
        double aR = cf->g3[2] / ((eps + ISR) * (eps + ISR));
        double s = aL + aC + aR;
        if (dev) {
            double d0 = fabs(aL / s / cf->g3[0] - 1.0), d1 = fabs(aC / s / cf->g3[1] - 1.0);
            double d2 = fabs(aR / s / cf->g3[2] - 1.0);
            *dev = fmax(d0, fmax(d1, d2));
        }
        if (linear) {
            wL = cf->g3[0]; wC = cf->g3[1]; wR = cf->g3[2];
        } else {
            wL = aL / s; wC = aC / s; wR = aR / s;
        }
        out[1] = wL * L1 + wC * C1 + wR * R1;
        out[2] = wL * L2 + wC * C2 + wR * R2;
        return;
    }
    /* p == 3: WENO-AO.  High member: the cubic truncation of the centred
     * five-zone quartic fit. */
    double H1 = (11.0 * v[-2] - 82.0 * v[-1] + 82.0 * v[1] - 11.0 * v[2]) / 120.0;
    double H2 = (-3.0 * v[-2] + 40.0 * v[-1] - 74.0 * v[0] + 40.0 * v[1] - 3.0 * v[2]) / 56.0;
    double H3 = (-v[-2] + 2.0 * v[-1] - 2.0 * v[1] + v[2]) / 12.0;
    double t = H1 + H3 / 10.0;
    double ISH = t * t + 13.0 / 3.0 * H2 * H2 + 781.0 / 20.0 * H3 * H3;
    double gH = cf->g4[0], gL = cf->g4[1], gC = cf->g4[2], gR = cf->g4[3];
    double wH, wL, wC, wR;
    double aH = gH / ((eps + ISH) * (eps + ISH));
    double aL = gL / ((eps + ISL) * (eps + ISL));
    double aC = gC / ((eps + ISC) * (eps + ISC));
    double aR = gR / ((eps + ISR) * (eps + ISR));
    double s = aH + aL + aC + aR;
    if (dev) {
        double d0 = fabs(aH / s / gH - 1.0), d1 = fabs(aL / s / gL - 1.0);
        double d2 = fabs(aC / s / gC - 1.0), d3 = fabs(aR / s / gR - 1.0);
        *dev = fmax(fmax(d0, d1), fmax(d2, d3));
    }
    if (linear) {
        wH = gH; wL = gL; wC = gC; wR = gR;
    } else {
        wH = aH / s; wL = aL / s; wC = aC / s; wR = aR / s;
    }
    double r = wH / gH;
    out[1] = r * (H1 - gL * L1 - gC * C1 - gR * R1) + wL * L1 + wC * C1 + wR * R1;
    out[2] = r * (H2 - gL * L2 - gC * C2 - gR * R2) + wL * L2 + wC * C2 + wR * R2;
    out[3] = r * H3;
}

void oracle_weno1d(const ocfg *cf, int p, const double *v5, double *out)
{
    weno1d_core(cf, p, v5, cf->linear_weno, out, NULL);
}

/* ------------------------------------------------------------------------ */
/* Multi-D reconstruction of one zone by successive x -> y -> z sweeps        */
/* ------------------------------------------------------------------------ */
/* blk: nv * 5^d zone averages around the zone, index [v][dz][dy][dx] with
 * offsets -2..2 stored at 0..4 (2D: [v][dy][dx]).  W: spatial modes in the
 * st_modes order (e = 0 block), [mode][v]. */
/* fl (may be NULL): gate flags of the zones the x-sweep lines are centred at,
 * [dz][dy] (2D: [dy]); an application centred at a flagged zone uses the
 * linear weights.  maxdev (may be NULL): max_k |omega_k/gamma_k - 1| over all
 * variables and all applications centred at the zone itself. */
static void recon_block_char(const ocfg *cf, const double *blk, double *W, const unsigned char *fl,
                             double *maxdev);

void oracle_recon_block_ex(const ocfg *cf, const double *blk, double *W, const unsigned char *fl,
                           double *maxdev)
{
    if (cf->char_recon) { recon_block_char(cf, blk, W, fl, maxdev); return; }
    int nd = cf->ndim, nv = nd + 2, p = cf->order - 1;
    mode4 m[MAXST];
    int nst = st_modes(nd, p, m);
    (void)nst;
    int nzb = (nd == 3) ? 5 : 1;
    int ms = 0;
    mode4 sm[MAXST];
    for (int i = 0; i < nst; ++i) if (m[i].e == 0) sm[ms++] = m[i];
    int zc = (nd == 3) ? 2 : 0;                 /* z index of the zone itself */
    double dmax = 0.0;
#define FLAG(z, y) (cf->linear_weno || (fl && fl[(z) * 5 + (y)]))
    for (int v = 0; v < nv; ++v) {
        const double *b = blk + (size_t)v * nzb * 25;
        /* x sweep on every (dz, dy) line: A[a][dz][dy] */
        double A[MAXP + 1][5][5];
        for (int z = 0; z < nzb; ++z)
            for (int y = 0; y < 5; ++y) {
                double line[5], c[4];
                for (int x = 0; x < 5; ++x) line[x] = b[(z * 5 + y) * 5 + x];
                double dv = 0.0;
                weno1d_core(cf, p, line, FLAG(z, y), c, &dv);
                if (z == zc && y == 2) dmax = fmax(dmax, dv);
                A[0][z][y] = line[2];
                for (int a = 1; a <= p; ++a) A[a][z][y] = c[a];
            }
        /* y sweep: B[a][b][dz] = first p-a outputs of R_p(A[a] along y) */
        double B[MAXP + 1][MAXP + 1][5];
        for (int z = 0; z < nzb; ++z)
            for (int a = 0; a <= p; ++a) {
                double line[5], c[4];
                for (int y = 0; y < 5; ++y) line[y] = A[a][z][y];
                B[a][0][z] = line[2];
                if (p - a >= 1) {
                    double dv = 0.0;
                    weno1d_core(cf, p, line, FLAG(z, 2), c, &dv);
                    if (z == zc) dmax = fmax(dmax, dv);
                    for (int bb = 1; bb <= p - a; ++bb) B[a][bb][z] = c[bb];
                }
            }
        /* z sweep (3D): C[a][b][c] = first p-a-b outputs of R_p(B[a][b] along z) */
        for (int k = 0; k < ms; ++k) {
            int a = sm[k].a, bb = sm[k].b, cc = sm[k].c;
            double val;
            if (nd == 2) {
                val = B[a][bb][0];
            } else if (cc == 0) {
                val = B[a][bb][2];
            } else {
                double line[5], c[4];
                for (int z = 0; z < 5; ++z) line[z] = B[a][bb][z];
                double dv = 0.0;
                weno1d_core(cf, p, line, FLAG(2, 2), c, &dv);
                dmax = fmax(dmax, dv);
                val = c[cc];
            }
            W[k * nv + v] = val;
        }
    }
#undef FLAG
    if (maxdev) *maxdev = dmax;
}

/* ------------------------------------------------------------------------ */
/* Characteristic-variable reconstruction (the alternative to the            */
/* component-wise reconstruction on conserved variables, Sec. I.1)           */
/* ------------------------------------------------------------------------ */
/* Right eigenvectors of the Jacobian of the flux along axis dir at the
 * conserved state U, as the columns of R: the u_n - c acoustic wave, the
 * entropy wave, one shear wave per tangential axis (in increasing axis order)
 * and the u_n + c acoustic wave. */
static void char_right(const ocfg *c, int dir, const double *U, double R[MAXV][MAXV])
{
    int nd = c->ndim, nv = nd + 2;
    double rho = U[0], u[3] = {0.0, 0.0, 0.0}, q2 = 0.0;
    for (int d = 0; d < nd; ++d) { u[d] = U[1 + d] / rho; q2 += u[d] * u[d]; }
    double p = pressure(c, U);
    double a = sqrt(c->gamma * p / rho);
    double H = (U[nv - 1] + p) / rho;
    memset(R, 0, sizeof(double) * MAXV * MAXV);
    R[0][0] = 1.0;
    R[0][1] = 1.0;
    R[0][nv - 1] = 1.0;
    for (int d = 0; d < nd; ++d) {
        R[1 + d][0] = u[d] - (d == dir ? a : 0.0);
        R[1 + d][1] = u[d];
        R[1 + d][nv - 1] = u[d] + (d == dir ? a : 0.0);
    }
    R[nv - 1][0] = H - u[dir] * a;
    R[nv - 1][1] = 0.5 * q2;
    R[nv - 1][nv - 1] = H + u[dir] * a;
    int col = 2;
    for (int d = 0; d < nd; ++d) {
        if (d == dir) continue;
        R[1 + d][col] = 1.0;
        R[nv - 1][col] = u[d];
        ++col;
    }
}

/* Inverse of the n x n matrix A by Gauss-Jordan elimination with partial
 * pivoting. */
static void invert(int n, double A[MAXV][MAXV], double X[MAXV][MAXV])
{
    double M[MAXV][2 * MAXV];
    for (int r = 0; r < n; ++r)
        for (int q = 0; q < n; ++q) { M[r][q] = A[r][q]; M[r][n + q] = (r == q) ? 1.0 : 0.0; }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
        if (piv != col)
            for (int q = 0; q < 2 * n; ++q) { double t = M[col][q]; M[col][q] = M[piv][q]; M[piv][q] = t; }
        double inv = 1.0 / M[col][col];
        for (int q = 0; q < 2 * n; ++q) M[col][q] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double f = M[r][col];
            for (int q = 0; q < 2 * n; ++q) M[r][q] -= f * M[col][q];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int q = 0; q < n; ++q) X[r][q] = M[r][n + q];
}

void oracle_char_eigen(const ocfg *c, int dir, const double *U, double *R, double *L)
{
    double Rm[MAXV][MAXV], Lm[MAXV][MAXV];
    int nv = c->ndim + 2;
    char_right(c, dir, U, Rm);
    invert(nv, Rm, Lm);
    for (int r = 0; r < nv; ++r)
        for (int q = 0; q < nv; ++q) { R[r * nv + q] = Rm[r][q]; L[r * nv + q] = Lm[r][q]; }
}

/* One 1D application on characteristic variables: lines[v][0..4] of all
 * variables along axis dir, ref the conserved state that defines the fields
 * (the mean of the zone the application is centred at).  Projects each
 * point on the fields (w = L u), applies the WENO operator to each field and
 * maps the coefficients back (c = R c_w).  out[v][1..p]; *dev receives the
 * largest weight deviation over the fields. */
static void weno_char(const ocfg *cf, int p, int dir, const double *ref, double lines[MAXV][5], int linear,
                      double out[MAXV][4], double *dev)
{
    int nv = cf->ndim + 2;
    double R[MAXV][MAXV], L[MAXV][MAXV];
    char_right(cf, dir, ref, R);
    invert(nv, R, L);
    double cw[MAXV][4];
    double dmax = 0.0;
    for (int k = 0; k < nv; ++k) {
        double w[5];
        for (int o = 0; o < 5; ++o) {
            w[o] = 0.0;
            for (int v = 0; v < nv; ++v) w[o] += L[k][v] * lines[v][o];
        }
        double dv = 0.0;
        weno1d_core(cf, p, w, linear, cw[k], &dv);
        dmax = fmax(dmax, dv);
    }
    for (int v = 0; v < nv; ++v)
        for (int a = 0; a <= p; ++a) {
            out[v][a] = 0.0;
            if (a == 0) continue;
            for (int k = 0; k < nv; ++k) out[v][a] += R[v][k] * cw[k][a];
        }
    if (dev) *dev = dmax;
}

/* The successive x -> y -> z sweeps of oracle_recon_block_ex with every 1D
 * application done on characteristic variables (weno_char): the x
 * application on the line through (dz, dy) takes the fields of that line's
 * centre zone, the y application of plane dz those of zone (0, 0, dz), the
 * z application those of the zone itself. */
static void recon_block_char(const ocfg *cf, const double *blk, double *W, const unsigned char *fl, double *maxdev)
{
    int nd = cf->ndim, nv = nd + 2, p = cf->order - 1;
    mode4 m[MAXST];
    int nst = st_modes(nd, p, m);
    int nzb = (nd == 3) ? 5 : 1;
    int zc = (nd == 3) ? 2 : 0;
    double dmax = 0.0;
#define BLK(v, z, y, x) blk[(((v) * nzb + (z)) * 5 + (y)) * 5 + (x)]
#define FLAG(z, y) (cf->linear_weno || (fl && fl[(z) * 5 + (y)]))
    double A[MAXP + 1][5][5][MAXV];
    for (int z = 0; z < nzb; ++z)
        for (int y = 0; y < 5; ++y) {
            double lines[MAXV][5], ref[MAXV], c[MAXV][4], dv = 0.0;
            for (int v = 0; v < nv; ++v) {
                for (int x = 0; x < 5; ++x) lines[v][x] = BLK(v, z, y, x);
                ref[v] = BLK(v, z, y, 2);
            }
            weno_char(cf, p, 0, ref, lines, FLAG(z, y), c, &dv);
            if (z == zc && y == 2) dmax = fmax(dmax, dv);
            for (int v = 0; v < nv; ++v) {
                A[0][z][y][v] = lines[v][2];
                for (int a = 1; a <= p; ++a) A[a][z][y][v] = c[v][a];
            }
        }
    double B[MAXP + 1][MAXP + 1][5][MAXV];
    for (int z = 0; z < nzb; ++z) {
        double ref[MAXV];
        for (int v = 0; v < nv; ++v) ref[v] = BLK(v, z, 2, 2);
        for (int a = 0; a <= p; ++a) {
            double lines[MAXV][5], c[MAXV][4], dv = 0.0;
            for (int v = 0; v < nv; ++v) {
                for (int y = 0; y < 5; ++y) lines[v][y] = A[a][z][y][v];
                B[a][0][z][v] = lines[v][2];
            }
            if (p - a < 1) continue;
            weno_char(cf, p, 1, ref, lines, FLAG(z, 2), c, &dv);
            if (z == zc) dmax = fmax(dmax, dv);
            for (int v = 0; v < nv; ++v)
                for (int bb = 1; bb <= p - a; ++bb) B[a][bb][z][v] = c[v][bb];
        }
    }
    double C[MAXP + 1][MAXP + 1][MAXP + 1][MAXV];
    for (int a = 0; a <= p; ++a)
        for (int bb = 0; a + bb <= p; ++bb) {
            for (int v = 0; v < nv; ++v) C[a][bb][0][v] = B[a][bb][zc][v];
            if (nd == 2 || p - a - bb < 1) continue;
            double lines[MAXV][5], ref[MAXV], c[MAXV][4], dv = 0.0;
            for (int v = 0; v < nv; ++v) {
                for (int z = 0; z < 5; ++z) lines[v][z] = B[a][bb][z][v];
                ref[v] = BLK(v, 2, 2, 2);
            }
            weno_char(cf, p, 2, ref, lines, FLAG(2, 2), c, &dv);
            dmax = fmax(dmax, dv);
            for (int v = 0; v < nv; ++v)
                for (int cc = 1; cc <= p - a - bb; ++cc) C[a][bb][cc][v] = c[v][cc];
        }
    int k = 0;
    for (int i = 0; i < nst; ++i) {
        if (m[i].e != 0) continue;
        for (int v = 0; v < nv; ++v) W[k * nv + v] = C[m[i].a][m[i].b][m[i].c][v];
        ++k;
    }
#undef BLK
#undef FLAG
    if (maxdev) *maxdev = dmax;
}

void oracle_recon_block(const ocfg *cf, const double *blk, double *W)
{
    oracle_recon_block_ex(cf, blk, W, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Space-time polynomial evaluation                                          */
/* ------------------------------------------------------------------------ */
/* q: [mode][v] in st_modes order.  (xi, eta, zeta) in [-1/2,1/2], tau in [0,1]. */
static void eval_modes(int nv, int nst, const mode4 *m, const double *q, double xi, double eta,
                       double zeta, double tau, double *U)
{
    for (int v = 0; v < nv; ++v) U[v] = 0.0;
    for (int i = 0; i < nst; ++i) {
        double phi = leg(m[i].a, xi) * leg(m[i].b, eta) * leg(m[i].c, zeta) * ipow(tau, m[i].e);
        for (int v = 0; v < nv; ++v) U[v] += q[i * nv + v] * phi;
    }
}
void oracle_eval_q(const ocfg *cf, const double *q, double xi, double eta, double zeta,
                   double tau, double *U)
{
    mode4 m[MAXST];
    int nst = st_modes(cf->ndim, cf->order - 1, m);
    eval_modes(cf->ndim + 2, nst, m, q, xi, eta, zeta, tau, U);
}

/* ------------------------------------------------------------------------ */
/* ADER predictor (Picard iteration with L2 projection of the fluxes)        */
/* ------------------------------------------------------------------------ */
/* W: spatial modes [ms][v]; q out: space-time modes [nst][v].
 * lam[d] = dt / dx_d.  q(.,tau=0) = W and, for k = 1..p,
 *   q_k = W - int_0^tau sum_d lam_d d/dxi_d  Proj[ F_d(q_{k-1}) ] dtau'
 * with Proj the L2 projection onto the space-time total-degree-p span of
 * leg x leg x leg x sleg computed with the tensor Gauss rule of p+1 points per
 * axis on [-1/2,1/2]^d x [0,1]. */
int oracle_predict(const ocfg *cf, const double *lam, const double *W, double *q)
{
    int troubled = 0;
    int nd = cf->ndim, nv = nd + 2, p = cf->order - 1, n1 = p + 1;
    mode4 m[MAXST];
    int nst = st_modes(nd, p, m);
    double gx[4], gw[4];
    gauss(n1, gx, gw);
    int nz_nodes = (nd == 3) ? n1 : 1;

    for (int i = 0; i < nst * nv; ++i) q[i] = 0.0;
    int ms = 0;
    for (int i = 0; i < nst; ++i) if (m[i].e == 0) { for (int v = 0; v < nv; ++v) q[i * nv + v] = W[ms * nv + v]; ++ms; }

    double f[3][MAXST][MAXV];
    for (int it = 1; it <= p; ++it) {
        memset(f, 0, sizeof f);
        for (int kz = 0; kz < nz_nodes; ++kz)
            for (int jy = 0; jy < n1; ++jy)
                for (int ix = 0; ix < n1; ++ix)
                    for (int lt = 0; lt < n1; ++lt) {
                        double xi = gx[ix], eta = gx[jy], zeta = (nd == 3) ? gx[kz] : 0.0;
                        double tau = 0.5 + gx[lt];
                        double wt = gw[ix] * gw[jy] * gw[lt] * ((nd == 3) ? gw[kz] : 1.0);
                        double U[MAXV], F[3][MAXV];
                        eval_modes(nv, nst, m, q, xi, eta, zeta, tau, U);
                        if (!admissible(cf, U)) troubled = 1;
                        for (int d = 0; d < nd; ++d) phys_flux(cf, d, U, F[d]);
                        for (int i = 0; i < nst; ++i) {
                            double phi = leg(m[i].a, xi) * leg(m[i].b, eta) * leg(m[i].c, zeta)
                                       * sleg(m[i].e, tau);
                            for (int d = 0; d < nd; ++d)
                                for (int v = 0; v < nv; ++v) f[d][i][v] += wt * phi * F[d][v];
                        }
                    }
        for (int i = 0; i < nst; ++i) {
            double nrm = leg_norm(m[i].a) * leg_norm(m[i].b) * leg_norm(m[i].c) * sleg_norm(m[i].e);
            for (int d = 0; d < nd; ++d)
                for (int v = 0; v < nv; ++v) f[d][i][v] /= nrm;
        }
        /* New iterate: W plus the time integral of minus the flux divergence. */
        double qn[MAXST * MAXV];
        for (int i = 0; i < nst * nv; ++i) qn[i] = (m[i / nv].e == 0) ? q[i] : 0.0;
        for (int d = 0; d < nd; ++d)
            for (int i = 0; i < nst; ++i) {
                int idx[3] = {m[i].a, m[i].b, m[i].c};
                int e = m[i].e;
                for (int ap = 0; ap < idx[d]; ++ap) {
                    double D = dleg(idx[d], ap);
                    if (D == 0.0) continue;
                    for (int ep = 1; ep <= e + 1; ++ep) {
                        double T = tint(e, ep);
                        if (T == 0.0) continue;
                        int t3[3] = {idx[0], idx[1], idx[2]};
                        t3[d] = ap;
                        int j = find_mode(m, nst, t3[0], t3[1], t3[2], ep);
                        for (int v = 0; v < nv; ++v) qn[j * nv + v] -= lam[d] * D * T * f[d][i][v];
                    }
                }
            }
        memcpy(q, qn, sizeof(double) * nst * nv);
    }
    return troubled;
}

/* ------------------------------------------------------------------------ */
/* Grid helpers                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int nd, nv, n[3], np[3];
    size_t vs;          /* stride between variables in the padded array */
} grid_t;

static void grid_init(const ocfg *c, grid_t *g)
{
    g->nd = c->ndim; g->nv = c->ndim + 2;
    g->n[0] = c->nx; g->n[1] = c->ny; g->n[2] = (c->ndim == 3) ? c->nz : 1;
    for (int d = 0; d < 3; ++d) g->np[d] = g->n[d] + ((d < g->nd) ? 2 * OG : 0);
    g->vs = (size_t)g->np[0] * g->np[1] * g->np[2];
}
/* index of zone (i, j, k) (interior numbering, may be negative) in the padded array */
static size_t pidx(const grid_t *g, int i, int j, int k)
{
    int o[3] = {OG, OG, (g->nd == 3) ? OG : 0};
    return ((size_t)(k + o[2]) * g->np[1] + (j + o[1])) * g->np[0] + (i + o[0]);
}
static int wrap(int i, int n, int bc)
{
    if (bc == 0) return ((i % n) + n) % n;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* Copy the interior (SoA [v][nz][ny][nx]) into a padded array and fill the
 * ghost zones: periodic wrap or zero-gradient clamp per axis (this also fills
 * edges and corners). */
static double *make_padded(const ocfg *c, const grid_t *g, const double *U)
{
    double *P = (double *)malloc(sizeof(double) * g->vs * g->nv);
    if (!P) return NULL;
    int o3 = (g->nd == 3) ? OG : 0;
    for (int v = 0; v < g->nv; ++v)
        for (int k = -o3; k < g->n[2] + o3; ++k)
            for (int j = -OG; j < g->n[1] + OG; ++j)
                for (int i = -OG; i < g->n[0] + OG; ++i) {
                    int si = wrap(i, g->n[0], c->bc[0]);
                    int sj = wrap(j, g->n[1], c->bc[1]);
                    int sk = (g->nd == 3) ? wrap(k, g->n[2], c->bc[2]) : 0;
                    P[v * g->vs + pidx(g, i, j, k)] =
                        U[(((size_t)v * g->n[2] + sk) * g->n[1] + sj) * g->n[0] + si];
                }
    return P;
}

/* Gather the 5^d block around zone (i,j,k) from the padded array. */
static void gather_block(const grid_t *g, const double *P, int i, int j, int k, double *blk)
{
    int nzb = (g->nd == 3) ? 5 : 1;
    for (int v = 0; v < g->nv; ++v)
        for (int z = 0; z < nzb; ++z)
            for (int y = 0; y < 5; ++y)
                for (int x = 0; x < 5; ++x) {
                    int kk = (g->nd == 3) ? k + z - 2 : 0;
                    blk[((v * nzb + z) * 5 + y) * 5 + x] = P[v * g->vs + pidx(g, i + x - 2, j + y - 2, kk)];
                }
}

/* Reconstruction + predictor of one zone from the padded array. */
/* Coordinates of face point (dir, side, pt) of a zone: side 0 is the face at
 * xi_dir = -1/2, side 1 the face at +1/2; pt enumerates the 2-point Gauss
 * rule in time (slowest), the first and the second tangential axis. */
static void face_point(int nd, int dir, int side, int pt, double *x, double *tau)
{
    double g = 0.5 / sqrt(3.0);
    int t1 = (dir == 0) ? 1 : 0;
    int t2 = (nd == 3) ? ((dir == 2) ? 1 : 2) : -1;
    int lt, a1, a2 = 0;
    if (nd == 3) { lt = pt / 4; a1 = (pt / 2) % 2; a2 = pt % 2; }
    else { lt = pt / 2; a1 = pt % 2; }
    x[0] = x[1] = x[2] = 0.0;
    x[dir] = side ? 0.5 : -0.5;
    x[t1] = a1 ? g : -g;
    if (t2 >= 0) x[t2] = a2 ? g : -g;
    *tau = 0.5 + (lt ? g : -g);
}

/* Reconstruction + predictor of one zone from the padded array.  With the
 * positivity option, a zone whose predictor met an inadmissible state at any
 * quadrature node, or whose final polynomial is inadmissible at any face
 * point, falls back to its zone mean (first order in space and time).
 * Returns 1 for such a zone. */
/* gate (may be NULL): per interior zone [nz][ny][nx], 1 = the 1D applications
 * centred at that zone use the linear weights; zones outside the interior
 * always use the nonlinear ones. */
static void gather_flags(const grid_t *g, const unsigned char *gate, int i, int j, int k, unsigned char *fl)
{
    int nzb = (g->nd == 3) ? 5 : 1;
    memset(fl, 0, 25);
    if (!gate) return;
    for (int z = 0; z < nzb; ++z)
        for (int y = 0; y < 5; ++y) {
            int jj = j + y - 2, kk = (g->nd == 3) ? k + z - 2 : 0;
            if (i < 0 || i >= g->n[0] || jj < 0 || jj >= g->n[1] || kk < 0 || kk >= g->n[2]) continue;
            fl[z * 5 + y] = gate[((size_t)kk * g->n[1] + jj) * g->n[0] + i];
        }
}

static int zone_q(const ocfg *c, const grid_t *g, const double *P, const double *lam, const unsigned char *gate,
                  int i, int j, int k, double *q)
{
    double blk[MAXV * 125], W[MAXST * MAXV];
    unsigned char fl[25];
    int nd = g->nd, nv = g->nv;
    gather_block(g, P, i, j, k, blk);
    gather_flags(g, gate, i, j, k, fl);
    oracle_recon_block_ex(c, blk, W, fl, NULL);
    int bad = oracle_predict(c, lam, W, q);
    if (!c->positivity) return 0;
    mode4 m[MAXST];
    int nst = st_modes(nd, c->order - 1, m);
    int npt = (nd == 3) ? 8 : 4;
    for (int dir = 0; dir < nd && !bad; ++dir)
        for (int side = 0; side < 2 && !bad; ++side)
            for (int pt = 0; pt < npt && !bad; ++pt) {
                double x[3], tau, U[MAXV];
                face_point(nd, dir, side, pt, x, &tau);
                eval_modes(nv, nst, m, q, x[0], x[1], x[2], tau, U);
                if (!admissible(c, U)) bad = 1;
            }
    if (!bad) return 0;
    int nzb = (nd == 3) ? 5 : 1;
    int centre = (nd == 3) ? (2 * 5 + 2) * 5 + 2 : 2 * 5 + 2;
    for (int t = 0; t < nst * nv; ++t) q[t] = 0.0;
    for (int v = 0; v < nv; ++v) q[v] = blk[v * nzb * 25 + centre];
    return 1;
}

/* Face flux between zone qa (left, lower index) and qb (right) along dir:
 * 2-point Gauss in each tangential direction and in time, weights 1/2 each,
 * summed with tau outermost, then the first tangential axis, then the second. */
static void face_flux(const ocfg *c, int dir, const double *qa, const double *qb, double *Fbar)
{
    int nd = c->ndim, nv = nd + 2;
    double s = 0.5 / sqrt(3.0);
    double pts[2] = {-s, s};
    int t1 = (dir == 0) ? 1 : 0;
    int t2 = (nd == 3) ? ((dir == 2) ? 1 : 2) : -1;
    double wgt = (nd == 3) ? 0.125 : 0.25;
    mode4 m[MAXST];
    int nst = st_modes(nd, c->order - 1, m);
    for (int v = 0; v < nv; ++v) Fbar[v] = 0.0;
    int n2 = (nd == 3) ? 2 : 1;
    for (int lt = 0; lt < 2; ++lt)
        for (int a1 = 0; a1 < 2; ++a1)
            for (int a2 = 0; a2 < n2; ++a2) {
                double xl[3] = {0, 0, 0}, xr[3] = {0, 0, 0};
                xl[dir] = 0.5; xr[dir] = -0.5;
                xl[t1] = xr[t1] = pts[a1];
                if (t2 >= 0) xl[t2] = xr[t2] = pts[a2];
                double tau = 0.5 + pts[lt];
                double UL[MAXV], UR[MAXV], F[MAXV];
                eval_modes(nv, nst, m, qa, xl[0], xl[1], xl[2], tau, UL);
                eval_modes(nv, nst, m, qb, xr[0], xr[1], xr[2], tau, UR);
                oracle_riemann(c, dir, UL, UR, F);
                for (int v = 0; v < nv; ++v) Fbar[v] += wgt * F[v];
            }
}

/* ------------------------------------------------------------------------ */
/* Second-order scheme (Sec. II.2, Figs. 3-7)                                */
/* ------------------------------------------------------------------------ */
/* Monotonised-central limiter with a compression factor (Fig. 3): the
 * limited undivided slope from the forward difference a and the backward
 * difference b.  Fortran's SIGN(0.5, x) is +0.5 at x = 0; the result is 0
 * whenever a and b differ in sign or either is 0. */
double oracle_mc(double a, double b, double cfac)
{
    double m = fmin(0.5 * fabs(a + b), fmin(cfac * fabs(a), cfac * fabs(b)));
    double sa = (a >= 0.0) ? 0.5 : -0.5;
    double sb = (b >= 0.0) ? 0.5 : -0.5;
    return m * (sa + sb);
}

/* Compression factor of Fig. 3: 2 for the density, 1.5 for the others. */
static double o2_cfac(int v) { return v == 0 ? 2.0 : 1.5; }

/* Modes of zone (i, j, k) at second order, stored in the space-time mode
 * order of st_modes(nd, 1): q[0..nv) the zone mean (mode 1 of Fig. 3),
 * q[(1+d)*nv ..] the limited undivided slope along axis d (modes 2-4, Fig. 3),
 * q[(1+nd)*nv ..] the time mode, dt times the time rate of change (mode 5,
 * Fig. 4).  The paper leaves the body of the pointwise predictor empty; it is
 * read as the Hancock step of MUSCL-Hancock in conserved variables: the time
 * mode is minus the sum over the axes of dt/dx_d times the difference of the
 * physical flux between the zone's two face-centre values U +- S_d/2.
 * With the positivity option, a zone where one of those face-centre values or
 * one of the face states U +- S_d/2 + U5/2 of Fig. 5 is inadmissible falls
 * back to its mean (zero slopes, zero time mode).  Returns 1 for such a zone. */
static int o2_zone(const ocfg *c, const grid_t *g, const double *P, const double *lam, int i, int j, int k,
                   double *q)
{
    int nd = g->nd, nv = g->nv;
    double *U5 = q + (1 + nd) * nv;
    for (int v = 0; v < nv; ++v) {
        q[v] = P[v * g->vs + pidx(g, i, j, k)];
        U5[v] = 0.0;
    }
    int bad = 0;
    for (int d = 0; d < nd; ++d) {
        int o[3] = {0, 0, 0};
        o[d] = 1;
        double *S = q + (1 + d) * nv;
        double Um[MAXV], Up[MAXV], Fm[MAXV], Fp[MAXV];
        for (int v = 0; v < nv; ++v) {
            double lo = P[v * g->vs + pidx(g, i - o[0], j - o[1], k - o[2])];
            double hi = P[v * g->vs + pidx(g, i + o[0], j + o[1], k + o[2])];
            S[v] = oracle_mc(hi - q[v], q[v] - lo, o2_cfac(v));
            Um[v] = q[v] - 0.5 * S[v];
            Up[v] = q[v] + 0.5 * S[v];
        }
        if (!admissible(c, Um) || !admissible(c, Up)) bad = 1;
        phys_flux(c, d, Um, Fm);
        phys_flux(c, d, Up, Fp);
        for (int v = 0; v < nv; ++v) U5[v] -= lam[d] * (Fp[v] - Fm[v]);
    }
    for (int d = 0; d < nd && !bad; ++d)
        for (int side = 0; side < 2 && !bad; ++side) {
            double W[MAXV];
            for (int v = 0; v < nv; ++v)
                W[v] = q[v] + (side ? 0.5 : -0.5) * q[(1 + d) * nv + v] + 0.5 * U5[v];
            if (!admissible(c, W)) bad = 1;
        }
    if (!c->positivity || !bad) return 0;
    for (int t = nv; t < (2 + nd) * nv; ++t) q[t] = 0.0;
    return 1;
}

/* Face flux of Fig. 5 between zone qa (lower index) and qb along dir: the
 * Riemann solver at the face centre and half time step, with the states
 * U + S/2 + U5/2 from qa and U - S/2 + U5/2 from qb. */
static void o2_face_flux(const ocfg *c, int dir, const double *qa, const double *qb, double *F)
{
    int nd = c->ndim, nv = nd + 2;
    double UL[MAXV], UR[MAXV];
    for (int v = 0; v < nv; ++v) {
        UL[v] = qa[v] + 0.5 * qa[(1 + dir) * nv + v] + 0.5 * qa[(1 + nd) * nv + v];
        UR[v] = qb[v] - 0.5 * qb[(1 + dir) * nv + v] + 0.5 * qb[(1 + nd) * nv + v];
    }
    oracle_riemann(c, dir, UL, UR, F);
}

/* Increment of Fig. 6 for one zone: -dt (F_d(+) - F_d(-)) / dx_d summed over
 * the axes, then added to the zone mean (Fig. 7). */
static void o2_update(int nd, const double *u, double dt, const double *h, double (*Fm)[MAXV],
                      double (*Fp)[MAXV], double *out)
{
    int nv = nd + 2;
    for (int v = 0; v < nv; ++v) {
        double du = 0.0;
        for (int d = 0; d < nd; ++d) du -= dt * (Fp[d][v] - Fm[d][v]) / h[d];
        out[v] = u[v] + du;
    }
}

/* One second-order step of the whole grid, in the stage order of Fig. 1:
 * ghost zones, limiter (Fig. 3) and predictor (Fig. 4) on the interior grown
 * by one zone per active axis, face fluxes (Fig. 5), update (Figs. 6-7).
 * Same arguments as oracle_step_count. */
static int o2_step(const ocfg *c, const double *U, double dt, double *Unew, long long *ntroubled)
{
    grid_t g;
    grid_init(c, &g);
    int nd = g.nd, nv = g.nv;
    double h[3] = {c->dx, c->dy, c->dz};
    double lam[3] = {dt / h[0], dt / h[1], dt / h[2]};
    double *P = make_padded(c, &g, U);
    if (!P) return -1;
    int e[3] = {g.n[0] + 2, g.n[1] + 2, (nd == 3) ? g.n[2] + 2 : 1};
    size_t ne = (size_t)e[0] * e[1] * e[2];
    size_t qs = (size_t)(2 + nd) * nv;
    double *Q = (double *)malloc(sizeof(double) * ne * qs);
    if (!Q) { free(P); return -1; }
    int o3 = (nd == 3) ? 1 : 0;
    long long nbad = 0;
#pragma omp parallel for schedule(static) collapse(2) reduction(+ : nbad)
    for (int k = 0; k < e[2]; ++k)
        for (int j = 0; j < e[1]; ++j)
            for (int i = 0; i < e[0]; ++i)
                nbad += o2_zone(c, &g, P, lam, i - 1, j - 1, k - o3, Q + (((size_t)k * e[1] + j) * e[0] + i) * qs);
    *ntroubled = nbad;
#define QAT(i, j, k) (Q + (((size_t)((k) + o3) * e[1] + ((j) + 1)) * e[0] + ((i) + 1)) * qs)
    size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
#pragma omp parallel for schedule(static) collapse(2)
    for (int k = 0; k < g.n[2]; ++k)
        for (int j = 0; j < g.n[1]; ++j)
            for (int i = 0; i < g.n[0]; ++i) {
                double Fm[3][MAXV], Fp[3][MAXV], u[MAXV], un[MAXV] = {0};
                for (int d = 0; d < nd; ++d) {
                    int o[3] = {0, 0, 0};
                    o[d] = 1;
                    o2_face_flux(c, d, QAT(i - o[0], j - o[1], k - o[2]), QAT(i, j, k), Fm[d]);
                    o2_face_flux(c, d, QAT(i, j, k), QAT(i + o[0], j + o[1], k + o[2]), Fp[d]);
                }
                size_t z = ((size_t)k * g.n[1] + j) * g.n[0] + i;
                for (int v = 0; v < nv; ++v) u[v] = U[v * N + z];
                o2_update(nd, u, dt, h, Fm, Fp, un);
                for (int v = 0; v < nv; ++v) Unew[v * N + z] = un[v];
            }
#undef QAT
    free(Q);
    free(P);
    return 0;
}

/* Second-order update of a list of zones, each recomputed from scratch. */
static int o2_step_zones(const ocfg *c, const double *U, double dt, int nlist, const int *ijk, double *out)
{
    grid_t g;
    grid_init(c, &g);
    int nd = g.nd, nv = g.nv;
    double h[3] = {c->dx, c->dy, c->dz};
    double lam[3] = {dt / h[0], dt / h[1], dt / h[2]};
    double *P = make_padded(c, &g, U);
    if (!P) return -1;
    size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
#pragma omp parallel for schedule(static)
    for (int s = 0; s < nlist; ++s) {
        int i = ijk[3 * s], j = ijk[3 * s + 1], k = (nd == 3) ? ijk[3 * s + 2] : 0;
        double qc[5 * MAXV], qm[5 * MAXV], qp[5 * MAXV];
        double Fm[3][MAXV], Fp[3][MAXV], u[MAXV];
        o2_zone(c, &g, P, lam, i, j, k, qc);
        for (int d = 0; d < nd; ++d) {
            int o[3] = {0, 0, 0};
            o[d] = 1;
            o2_zone(c, &g, P, lam, i - o[0], j - o[1], k - o[2], qm);
            o2_zone(c, &g, P, lam, i + o[0], j + o[1], k + o[2], qp);
            o2_face_flux(c, d, qm, qc, Fm[d]);
            o2_face_flux(c, d, qc, qp, Fp[d]);
        }
        size_t z = ((size_t)k * g.n[1] + j) * g.n[0] + i;
        for (int v = 0; v < nv; ++v) u[v] = U[v * N + z];
        o2_update(nd, u, dt, h, Fm, Fp, out + (size_t)s * nv);
    }
    free(P);
    return 0;
}

/* Second-order stage taps: W [zone][1+nd][nv] (mean and limited slopes) and
 * q [zone][2+nd][nv] (with the time mode) of every interior zone. */
static int o2_stage_modes(const ocfg *c, const double *U, double dt, double *Wout, double *qout)
{
    grid_t g;
    grid_init(c, &g);
    int nd = g.nd, nv = g.nv;
    double h[3] = {c->dx, c->dy, c->dz};
    double lam[3] = {dt / h[0], dt / h[1], dt / h[2]};
    double *P = make_padded(c, &g, U);
    if (!P) return -1;
    size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
    for (size_t z = 0; z < N; ++z) {
        int i = (int)(z % g.n[0]), j = (int)((z / g.n[0]) % g.n[1]), k = (int)(z / ((size_t)g.n[0] * g.n[1]));
        double q[5 * MAXV];
        o2_zone(c, &g, P, lam, i, j, k, q);
        if (Wout) memcpy(Wout + z * (1 + nd) * nv, q, sizeof(double) * (1 + nd) * nv);
        if (qout) memcpy(qout + z * (2 + nd) * nv, q, sizeof(double) * (2 + nd) * nv);
    }
    free(P);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Runge-Kutta time stepping (Sec. I.1; Sec. III.1, Table IV)                */
/* ------------------------------------------------------------------------ */
/* The paper compares its ADER step with multi-stage Runge-Kutta schemes built
 * from the same reconstruction and Riemann solver: two stages at second order,
 * three at third, five at fourth.  They are read as the strong-stability-
 * preserving schemes of that shape: SSP-RK(2,2) and SSP-RK(3,3) of Shu and
 * Osher, and SSP-RK(5,4) of Spiteri and Ruuth, in Shu-Osher form
 *   u(i) = sum_{k<i} ( alpha_ik u(k) + beta_ik dt L(u(k)) ),  u(0) = U^n,
 * with the published coefficients (the fourth-order conditions are checked in
 * the tests).  L is the method-of-lines operator: the spatial polynomial of
 * every zone (WENO at third/fourth order, mean + MC slopes at second order),
 * the Riemann solver at the face points in space only (2-point Gauss per
 * tangential axis; the face centre at second order), and the flux
 * difference. */
typedef struct { int i, k; double alpha, beta; } rk_term;

static int rk_table(int stepper, const rk_term **t)
{
    static const rk_term rk2[] = {{1, 0, 1.0, 1.0}, {2, 0, 0.5, 0.0}, {2, 1, 0.5, 0.5}};
    static const rk_term rk3[] = {{1, 0, 1.0, 1.0},
                                  {2, 0, 0.75, 0.0}, {2, 1, 0.25, 0.25},
                                  {3, 0, 1.0 / 3.0, 0.0}, {3, 2, 2.0 / 3.0, 2.0 / 3.0}};
    static const rk_term rk54[] = {{1, 0, 1.0, 0.391752226571890},
                                   {2, 0, 0.444370493651235, 0.0}, {2, 1, 0.555629506348765, 0.368410593050371},
                                   {3, 0, 0.620101851488403, 0.0}, {3, 2, 0.379898148511597, 0.251891774271694},
                                   {4, 0, 0.178079954393132, 0.0}, {4, 3, 0.821920045606868, 0.544974750228521},
                                   {5, 2, 0.517231671970585, 0.0}, {5, 3, 0.096059710526147, 0.063692468666290},
                                   {5, 4, 0.386708617503269, 0.226007483236906}};
    if (stepper == 2) { *t = rk2; return (int)(sizeof rk2 / sizeof rk2[0]); }
    if (stepper == 3) { *t = rk3; return (int)(sizeof rk3 / sizeof rk3[0]); }
    if (stepper == 4) { *t = rk54; return (int)(sizeof rk54 / sizeof rk54[0]); }
    return 0;
}
static int rk_stages(int stepper) { return stepper == 2 ? 2 : (stepper == 3 ? 3 : (stepper == 4 ? 5 : 0)); }

/* Coefficient table for the tests: n terms of (i, k, alpha, beta). */
int oracle_rk_table(int stepper, int *ik, double *ab)
{
    const rk_term *t;
    int n = rk_table(stepper, &t);
    for (int s = 0; s < n && ik; ++s) {
        ik[2 * s] = t[s].i; ik[2 * s + 1] = t[s].k;
        ab[2 * s] = t[s].alpha; ab[2 * s + 1] = t[s].beta;
    }
    return n;
}

/* Spatial modes W [1 + nd or ms][nv] (st_modes order, e = 0 block) of zone
 * (i, j, k) for the method of lines: WENO at third/fourth order, the mean and
 * MC slopes of Fig. 3 at second order.  With the positivity option a zone whose
 * polynomial is inadmissible at one of its face points keeps only its mean.
 * Returns 1 for such a zone. */
static int rk_zone_modes(const ocfg *c, const grid_t *g, const double *P, int i, int j, int k, double *W,
                         int *ms_out)
{
    int nd = g->nd, nv = g->nv, ms;
    mode4 m[MAXST];
    if (c->order == 2) {
        ms = 1 + nd;
        st_modes(nd, 1, m);
        for (int v = 0; v < nv; ++v) W[v] = P[v * g->vs + pidx(g, i, j, k)];
        for (int d = 0; d < nd; ++d) {
            int o[3] = {0, 0, 0};
            o[d] = 1;
            for (int v = 0; v < nv; ++v) {
                double lo = P[v * g->vs + pidx(g, i - o[0], j - o[1], k - o[2])];
                double hi = P[v * g->vs + pidx(g, i + o[0], j + o[1], k + o[2])];
                W[(1 + d) * nv + v] = oracle_mc(hi - W[v], W[v] - lo, o2_cfac(v));
            }
        }
    } else {
        double blk[MAXV * 125];
        unsigned char fl[25];
        int nst = st_modes(nd, c->order - 1, m);
        ms = 0;
        for (int t = 0; t < nst; ++t) ms += (m[t].e == 0);
        gather_block(g, P, i, j, k, blk);
        memset(fl, 0, sizeof fl);
        oracle_recon_block_ex(c, blk, W, fl, NULL);
    }
    *ms_out = ms;
    if (!c->positivity) return 0;
    double s = 0.5 / sqrt(3.0);
    int npt = (c->order == 2) ? 1 : (nd == 3 ? 4 : 2);
    int bad = 0;
    for (int dir = 0; dir < nd && !bad; ++dir)
        for (int side = 0; side < 2 && !bad; ++side)
            for (int pt = 0; pt < npt && !bad; ++pt) {
                double x[3] = {0, 0, 0}, U[MAXV];
                int t1 = (dir == 0) ? 1 : 0, t2 = (nd == 3) ? ((dir == 2) ? 1 : 2) : -1;
                x[dir] = side ? 0.5 : -0.5;
                if (c->order != 2) {
                    x[t1] = (pt & 1) ? s : -s;
                    if (t2 >= 0) x[t2] = (pt & 2) ? s : -s;
                }
                eval_modes(nv, ms, m, W, x[0], x[1], x[2], 0.0, U);
                if (!admissible(c, U)) bad = 1;
            }
    if (!bad) return 0;
    for (int t = nv; t < ms * nv; ++t) W[t] = 0.0;
    return 1;
}

/* Face flux between zones Wa (lower) and Wb along dir in space only: the
 * Riemann solver at 2-point Gauss points of the tangential axes (weights 1/2
 * each, first tangential axis outer), or at the face centre at second order. */
static void rk_face_flux(const ocfg *c, int dir, const double *Wa, const double *Wb, int ms, double *F)
{
    int nd = c->ndim, nv = nd + 2;
    mode4 m[MAXST];
    st_modes(nd, (c->order == 2) ? 1 : c->order - 1, m);
    double s = 0.5 / sqrt(3.0);
    int t1 = (dir == 0) ? 1 : 0, t2 = (nd == 3) ? ((dir == 2) ? 1 : 2) : -1;
    int n1 = (c->order == 2) ? 1 : 2, n2 = (c->order == 2 || nd == 2) ? 1 : 2;
    double w = 1.0 / (n1 * n2);
    for (int v = 0; v < nv; ++v) F[v] = 0.0;
    for (int a1 = 0; a1 < n1; ++a1)
        for (int a2 = 0; a2 < n2; ++a2) {
            double xl[3] = {0, 0, 0}, xr[3] = {0, 0, 0}, UL[MAXV], UR[MAXV], Fp[MAXV];
            xl[dir] = 0.5;
            xr[dir] = -0.5;
            if (n1 == 2) xl[t1] = xr[t1] = a1 ? s : -s;
            if (n2 == 2) xl[t2] = xr[t2] = a2 ? s : -s;
            eval_modes(nv, ms, m, Wa, xl[0], xl[1], xl[2], 0.0, UL);
            eval_modes(nv, ms, m, Wb, xr[0], xr[1], xr[2], 0.0, UR);
            oracle_riemann(c, dir, UL, UR, Fp);
            for (int v = 0; v < nv; ++v) F[v] += w * Fp[v];
        }
}

/* dU = dt L(U) = -dt sum_d (F_d(+) - F_d(-)) / dx_d on the interior. */
static int rk_operator(const ocfg *c, const double *U, double dt, double *dU, long long *ntroubled)
{
    grid_t g;
    grid_init(c, &g);
    int nd = g.nd, nv = g.nv;
    double h[3] = {c->dx, c->dy, c->dz};
    double *P = make_padded(c, &g, U);
    if (!P) return -1;
    int e[3] = {g.n[0] + 2, g.n[1] + 2, (nd == 3) ? g.n[2] + 2 : 1};
    size_t ne = (size_t)e[0] * e[1] * e[2];
    size_t ws = (size_t)MAXST * nv;
    double *Wz = (double *)malloc(sizeof(double) * ne * ws);
    if (!Wz) { free(P); return -1; }
    int o3 = (nd == 3) ? 1 : 0, ms = 1;
    long long nbad = 0;
#pragma omp parallel for schedule(dynamic, 1) collapse(2) reduction(+ : nbad) reduction(max : ms)
    for (int k = 0; k < e[2]; ++k)
        for (int j = 0; j < e[1]; ++j)
            for (int i = 0; i < e[0]; ++i) {
                int msz;
                nbad += rk_zone_modes(c, &g, P, i - 1, j - 1, k - o3, Wz + (((size_t)k * e[1] + j) * e[0] + i) * ws,
                                      &msz);
                if (msz > ms) ms = msz;
            }
    if (ntroubled) *ntroubled += nbad;
#define WAT(i, j, k) (Wz + (((size_t)((k) + o3) * e[1] + ((j) + 1)) * e[0] + ((i) + 1)) * ws)
    size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
#pragma omp parallel for schedule(static) collapse(2)
    for (int k = 0; k < g.n[2]; ++k)
        for (int j = 0; j < g.n[1]; ++j)
            for (int i = 0; i < g.n[0]; ++i) {
                size_t z = ((size_t)k * g.n[1] + j) * g.n[0] + i;
                double du[MAXV] = {0};
                for (int d = 0; d < nd; ++d) {
                    int o[3] = {0, 0, 0};
                    o[d] = 1;
                    double Fm[MAXV], Fp[MAXV];
                    rk_face_flux(c, d, WAT(i - o[0], j - o[1], k - o[2]), WAT(i, j, k), ms, Fm);
                    rk_face_flux(c, d, WAT(i, j, k), WAT(i + o[0], j + o[1], k + o[2]), ms, Fp);
                    for (int v = 0; v < nv; ++v) du[v] -= dt * (Fp[v] - Fm[v]) / h[d];
                }
                for (int v = 0; v < nv; ++v) dU[v * N + z] = du[v];
            }
#undef WAT
    free(Wz);
    free(P);
    return 0;
}

/* One Runge-Kutta step of the whole grid; *ntroubled receives the fallback
 * zones summed over the stages. */
static int rk_step(const ocfg *c, const double *U, double dt, double *Unew, long long *ntroubled)
{
    const rk_term *t;
    int nt = rk_table(c->stepper, &t), s = rk_stages(c->stepper);
    if (!nt) return -2;
    int nd = c->ndim, nv = nd + 2;
    size_t N = (size_t)c->nx * c->ny * ((nd == 3) ? c->nz : 1), nn = N * nv;
    double *u = (double *)malloc(sizeof(double) * nn * (s + 1));   /* u(0) .. u(s) */
    double *L = (double *)malloc(sizeof(double) * nn * s);         /* dt L(u(k)) */
    if (!u || !L) { free(u); free(L); return -1; }
    memcpy(u, U, sizeof(double) * nn);
    *ntroubled = 0;
    for (int i = 1; i <= s; ++i) {
        if (rk_operator(c, u + (size_t)(i - 1) * nn, dt, L + (size_t)(i - 1) * nn, ntroubled)) {
            free(u); free(L); return -1;
        }
        double *ui = u + (size_t)i * nn;
        for (size_t q = 0; q < nn; ++q) ui[q] = 0.0;
        for (int r = 0; r < nt; ++r) {
            if (t[r].i != i) continue;
            const double *uk = u + (size_t)t[r].k * nn, *Lk = L + (size_t)t[r].k * nn;
            for (size_t q = 0; q < nn; ++q) {
                ui[q] += t[r].alpha * uk[q];
                if (t[r].beta != 0.0) ui[q] += t[r].beta * Lk[q];
            }
        }
    }
    memcpy(Unew, u + (size_t)s * nn, sizeof(double) * nn);
    free(u);
    free(L);
    return 0;
}

/* dt L(U) for the tests (method-of-lines operator of the configured order). */
int oracle_rk_operator(const ocfg *c, const double *U, double dt, double *dU)
{
    long long n = 0;
    return rk_operator(c, U, dt, dU, &n);
}

/* ------------------------------------------------------------------------ */
/* Public entry points                                                       */
/* ------------------------------------------------------------------------ */
/* CFL time step of a state (interior SoA): dt = cfl / max_zones sum_d
 * (|u_d| + c) / dx_d.  Returns -1 and sets *bad to the first non-physical
 * zone (rho <= 0, p <= 0 or non-finite) if there is one. */
double oracle_cfl_dt(const ocfg *c, const double *U, long long *bad)
{
    int nd = c->ndim, nv = nd + 2;
    size_t N = (size_t)c->nx * c->ny * ((nd == 3) ? c->nz : 1);
    double h[3] = {c->dx, c->dy, c->dz};
    double smax = 0.0;
    *bad = -1;
    for (size_t z = 0; z < N; ++z) {
        double Uz[MAXV];
        for (int v = 0; v < nv; ++v) Uz[v] = U[v * N + z];
        double rho = Uz[0];
        double p = pressure(c, Uz);
        if (!(rho > 0.0) || !(p > 0.0) || !isfinite(rho) || !isfinite(p)) { *bad = (long long)z; return -1.0; }
        double cs = sqrt(c->gamma * p / rho);
        double s = 0.0;
        for (int d = 0; d < nd; ++d) s += (fabs(Uz[1 + d] / rho) + cs) / h[d];
        if (s > smax) smax = s;
    }
    return c->cfl / smax;
}

/* One ADER-WENO step of the whole grid with time step dt.  U, Unew: interior
 * SoA [nv][nz][ny][nx] (may not alias).  Returns 0, or -1 on allocation failure. */
int oracle_step_gated(const ocfg *c, const double *U, double dt, const unsigned char *gate, double *Unew,
                      long long *ntroubled);
int oracle_step(const ocfg *c, const double *U, double dt, double *Unew)
{
    long long n;
    return oracle_step_gated(c, U, dt, NULL, Unew, &n);
}
int oracle_step_count(const ocfg *c, const double *U, double dt, double *Unew, long long *ntroubled)
{
    return oracle_step_gated(c, U, dt, NULL, Unew, ntroubled);
}

/* One step; gate (may be NULL) as for zone_q; *ntroubled receives the number
 * of zones of the predictor box (interior grown by one zone per active axis)
 * that used the positivity fallback. */
int oracle_step_gated(const ocfg *c, const double *U, double dt, const unsigned char *gate, double *Unew,
                      long long *ntroubled)
{
    if (c->stepper != 0) return gate ? -2 : rk_step(c, U, dt, Unew, ntroubled);
    if (c->order == 2) return gate ? -2 : o2_step(c, U, dt, Unew, ntroubled);
    grid_t g;
    grid_init(c, &g);
    int nd = g.nd, nv = g.nv, p = c->order - 1;
    mode4 m[MAXST];
    int nst = st_modes(nd, p, m);
    double h[3] = {c->dx, c->dy, c->dz};
    double lam[3] = {dt / h[0], dt / h[1], dt / h[2]};
    double *P = make_padded(c, &g, U);
    if (!P) return -1;
    /* predictor on the interior box grown by one zone per active axis */
    int e[3] = {g.n[0] + 2, g.n[1] + 2, (nd == 3) ? g.n[2] + 2 : 1};
    size_t ne = (size_t)e[0] * e[1] * e[2];
    size_t qs = (size_t)nst * nv;
    double *Q = (double *)malloc(sizeof(double) * ne * qs);
    if (!Q) { free(P); return -1; }
    int o3 = (nd == 3) ? 1 : 0;
    long long nbad = 0;
#pragma omp parallel for schedule(dynamic, 1) collapse(2) reduction(+ : nbad)
    for (int k = 0; k < e[2]; ++k)
        for (int j = 0; j < e[1]; ++j)
            for (int i = 0; i < e[0]; ++i)
                nbad += zone_q(c, &g, P, lam, gate, i - 1, j - 1, k - o3, Q + (((size_t)k * e[1] + j) * e[0] + i) * qs);
    *ntroubled = nbad;
#define QAT(i, j, k) (Q + (((size_t)((k) + o3) * e[1] + ((j) + 1)) * e[0] + ((i) + 1)) * qs)
    size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
#pragma omp parallel for schedule(static) collapse(2)
    for (int k = 0; k < g.n[2]; ++k)
        for (int j = 0; j < g.n[1]; ++j)
            for (int i = 0; i < g.n[0]; ++i) {
                double Fm[3][MAXV], Fp[3][MAXV];
                face_flux(c, 0, QAT(i - 1, j, k), QAT(i, j, k), Fm[0]);
                face_flux(c, 0, QAT(i, j, k), QAT(i + 1, j, k), Fp[0]);
                face_flux(c, 1, QAT(i, j - 1, k), QAT(i, j, k), Fm[1]);
                face_flux(c, 1, QAT(i, j, k), QAT(i, j + 1, k), Fp[1]);
                if (nd == 3) {
                    face_flux(c, 2, QAT(i, j, k - 1), QAT(i, j, k), Fm[2]);
                    face_flux(c, 2, QAT(i, j, k), QAT(i, j, k + 1), Fp[2]);
                }
                size_t z = ((size_t)k * g.n[1] + j) * g.n[0] + i;
                for (int v = 0; v < nv; ++v) {
                    double u = U[v * N + z];
                    for (int d = 0; d < nd; ++d) u = u - lam[d] * (Fp[d][v] - Fm[d][v]);
                    Unew[v * N + z] = u;
                }
            }
#undef QAT
    free(Q);
    free(P);
    return 0;
}

/* Same update for a list of zones only (each recomputed from scratch, for
 * spot checks of large grids).  ijk: nlist triples; out: [nlist][nv]. */
int oracle_step_zones(const ocfg *c, const double *U, double dt, int nlist, const int *ijk, double *out)
{
    if (c->stepper != 0) return -2;   /* a Runge-Kutta step is not local to a zone's stencil */
    if (c->order == 2) return o2_step_zones(c, U, dt, nlist, ijk, out);
    grid_t g;
    grid_init(c, &g);
    int nd = g.nd, nv = g.nv, p = c->order - 1;
    mode4 m[MAXST];
    int nst = st_modes(nd, p, m);
    size_t qs = (size_t)nst * nv;
    double h[3] = {c->dx, c->dy, c->dz};
    double lam[3] = {dt / h[0], dt / h[1], dt / h[2]};
    double *P = make_padded(c, &g, U);
    if (!P) return -1;
    size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < nlist; ++s) {
        int i = ijk[3 * s], j = ijk[3 * s + 1], k = (nd == 3) ? ijk[3 * s + 2] : 0;
        double qc[MAXST * MAXV], qm[MAXST * MAXV], qp[MAXST * MAXV];
        double Fm[MAXV], Fp[MAXV];
        size_t z = ((size_t)k * g.n[1] + j) * g.n[0] + i;
        double u[MAXV];
        for (int v = 0; v < nv; ++v) u[v] = U[v * N + z];
        zone_q(c, &g, P, lam, NULL, i, j, k, qc);
        for (int d = 0; d < nd; ++d) {
            int o[3] = {0, 0, 0};
            o[d] = 1;
            zone_q(c, &g, P, lam, NULL, i - o[0], j - o[1], k - o[2], qm);
            zone_q(c, &g, P, lam, NULL, i + o[0], j + o[1], k + o[2], qp);
            face_flux(c, d, qm, qc, Fm);
            face_flux(c, d, qc, qp, Fp);
            for (int v = 0; v < nv; ++v) u[v] = u[v] - lam[d] * (Fp[v] - Fm[v]);
        }
        (void)qs;
        for (int v = 0; v < nv; ++v) out[s * nv + v] = u[v];
    }
    free(P);
    return 0;
}

/* Time loop: dt from the CFL condition of the current state each step (the
 * paper's dt_next, Fig. 1/Fig. 7); if t_end > 0 the last step is clipped so
 * the run ends at t_end, else exactly nsteps steps are taken.  U is updated
 * in place.  Returns the number of steps taken, or -1 on a non-physical state. */
int oracle_run(const ocfg *c, double *U, int nsteps, double t_end, double *t_out, double *dts)
{
    int nd = c->ndim, nv = nd + 2;
    size_t N = (size_t)c->nx * c->ny * ((nd == 3) ? c->nz : 1);
    double *tmp = (double *)malloc(sizeof(double) * N * nv);
    if (!tmp) return -1;
    double t = 0.0;
    int s = 0;
    for (;;) {
        if (t_end > 0.0) { if (t >= t_end * (1.0 - 1e-14)) break; }
        else if (s >= nsteps) break;
        long long bad;
        double dt = oracle_cfl_dt(c, U, &bad);
        if (dt < 0.0) { free(tmp); return -1; }
        if (t_end > 0.0 && t + dt > t_end) dt = t_end - t;
        if (oracle_step(c, U, dt, tmp) != 0) { free(tmp); return -1; }
        memcpy(U, tmp, sizeof(double) * N * nv);
        if (dts) dts[s] = dt;
        t += dt;
        ++s;
    }
    *t_out = t;
    free(tmp);
    return s;
}

/* Stage taps for parity checks: spatial modes W [zone][ms][nv] and space-time
 * modes q [zone][nst][nv] of every interior zone (ignoring zones beyond). */
int oracle_stage_modes(const ocfg *c, const double *U, double dt, double *Wout, double *qout)
{
    if (c->stepper != 0) return -2;
    if (c->order == 2) return o2_stage_modes(c, U, dt, Wout, qout);
    grid_t g;
    grid_init(c, &g);
    int nd = g.nd, nv = g.nv, p = c->order - 1;
    mode4 m[MAXST];
    int nst = st_modes(nd, p, m);
    int ms = 0;
    for (int i = 0; i < nst; ++i) ms += (m[i].e == 0);
    double h[3] = {c->dx, c->dy, c->dz};
    double lam[3] = {dt / h[0], dt / h[1], dt / h[2]};
    double *P = make_padded(c, &g, U);
    if (!P) return -1;
    size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
#pragma omp parallel for schedule(dynamic, 4)
    for (long long z = 0; z < (long long)N; ++z) {
        int i = (int)(z % g.n[0]), j = (int)((z / g.n[0]) % g.n[1]), k = (int)(z / ((size_t)g.n[0] * g.n[1]));
        double blk[MAXV * 125], W[MAXST * MAXV], q[MAXST * MAXV];
        gather_block(&g, P, i, j, k, blk);
        oracle_recon_block(c, blk, W);
        if (Wout) memcpy(Wout + (size_t)z * ms * nv, W, sizeof(double) * ms * nv);
        if (qout) {
            oracle_predict(c, lam, W, q);
            memcpy(qout + (size_t)z * nst * nv, q, sizeof(double) * nst * nv);
        }
    }
    free(P);
    return 0;
}

/* Per interior zone: max_k |omega_k/gamma_k - 1| over the variables and the
 * 1D applications centred at the zone (full nonlinear weights). */
int oracle_zone_maxdev(const ocfg *c, const double *U, double *out)
{
    if (c->order == 2) return -2;   /* no WENO weights at second order */
    grid_t g;
    grid_init(c, &g);
    double *P = make_padded(c, &g, U);
    if (!P) return -1;
    size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
#pragma omp parallel for schedule(dynamic, 16)
    for (long long z = 0; z < (long long)N; ++z) {
        int i = (int)(z % g.n[0]), j = (int)((z / g.n[0]) % g.n[1]), k = (int)(z / ((size_t)g.n[0] * g.n[1]));
        double blk[MAXV * 125], W[MAXST * MAXV], d;
        gather_block(&g, P, i, j, k, blk);
        oracle_recon_block_ex(c, blk, W, NULL, &d);
        out[z] = d;
    }
    free(P);
    return 0;
}

/* Number of spatial / space-time modes and the mode list (for tests). */
int oracle_modes(int ndim, int p, int *abce)
{
    mode4 m[MAXST];
    int n = st_modes(ndim, p, m);
    if (abce)
        for (int i = 0; i < n; ++i) { abce[4 * i] = m[i].a; abce[4 * i + 1] = m[i].b; abce[4 * i + 2] = m[i].c; abce[4 * i + 3] = m[i].e; }
    return n;
}

/* Basis and quadrature accessors for the pins. */
double oracle_leg(int a, double x) { return leg(a, x); }
double oracle_sleg(int e, double t) { return sleg(e, t); }
double oracle_dleg(int a, int ap) { return dleg(a, ap); }
double oracle_tint(int e, int ep) { return tint(e, ep); }
void oracle_gauss(int n, double *x, double *w) { gauss(n, x, w); }

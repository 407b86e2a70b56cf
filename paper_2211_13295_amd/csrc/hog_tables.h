// hog_tables.h -- compile-time bases, quadrature rules and mode lists of the
// ADER-WENO zone update on gfx950.
//
// Everything here is derived at compile time from three facts: the
// Gauss-Legendre nodes/weights, the three-term recurrence of the monic
// Legendre polynomials on the reference zone [-1/2, 1/2], and the recurrence
// of the Legendre polynomials shifted to the time interval [0, 1].  Norms,
// derivative maps and time-integral maps are obtained by exact quadrature or
// exact polynomial algebra on top of them, so every coefficient folds into an
// instruction literal in the fully unrolled kernels.
#pragma once

namespace hog {

// ---------------------------------------------------------------------------
// Gauss-Legendre rules on [-1/2, 1/2] with n = 2, 3, 4 points (weights sum to 1).
// ---------------------------------------------------------------------------
constexpr double gl_node(int n, int i)
{
    if (n == 2) return i == 0 ? -0.28867513459481288225 : 0.28867513459481288225;
    if (n == 3) return i == 0 ? -0.38729833462074168852 : (i == 1 ? 0.0 : 0.38729833462074168852);
    const double a = 0.16999052179242813240, b = 0.43056815579702628761;
    return i == 0 ? -b : (i == 1 ? -a : (i == 2 ? a : b));
}
constexpr double gl_weight(int n, int i)
{
    if (n == 2) return 0.5;
    if (n == 3) return i == 1 ? 4.0 / 9.0 : 5.0 / 18.0;
    const double wa = 0.32607257743127307131, wb = 0.17392742256872692869;
    return (i == 1 || i == 2) ? wa : wb;
}

// Monic Legendre polynomial of degree a on [-1/2, 1/2] and its derivative,
// from  P_{n+1} = x P_n - n^2 / (4 (4 n^2 - 1)) P_{n-1}.
constexpr double mleg(int a, double x)
{
    double pm = 1.0, p = x;
    if (a == 0) return 1.0;
    for (int n = 1; n < a; ++n) {
        double pn = x * p - (double)(n * n) / (4.0 * (4.0 * n * n - 1.0)) * pm;
        pm = p;
        p = pn;
    }
    return p;
}
constexpr double dmleg(int a, double x)
{
    if (a == 0) return 0.0;
    double pm = 1.0, p = x, dpm = 0.0, dp = 1.0;
    for (int n = 1; n < a; ++n) {
        double c = (double)(n * n) / (4.0 * (4.0 * n * n - 1.0));
        double pn = x * p - c * pm;
        double dpn = p + x * dp - c * dpm;
        pm = p; p = pn;
        dpm = dp; dp = dpn;
    }
    return dp;
}
// Shifted Legendre polynomial on [0, 1]:  (e+1) L_{e+1} = (2e+1)(2t-1) L_e - e L_{e-1}.
constexpr double tleg(int e, double t)
{
    double lm = 1.0, l = 2.0 * t - 1.0;
    if (e == 0) return 1.0;
    for (int n = 1; n < e; ++n) {
        double ln = ((2.0 * n + 1.0) * (2.0 * t - 1.0) * l - n * lm) / (n + 1.0);
        lm = l;
        l = ln;
    }
    return l;
}

// ---------------------------------------------------------------------------
// 1D tables for polynomial degree P (P + 1 Gauss points per axis).
// ---------------------------------------------------------------------------
template <int P>
struct Rules {
    static constexpr int N = P + 1;
    double x[N], w[N], t[N];
    double px[P + 1][N];      // P_a(x_i)
    double pn[P + 1];         // int P_a^2
    double lt[P + 1][N];      // L_e(t_l)
    double ln[P + 1];         // int_0^1 L_e^2
    double proj[P + 1][N];    // w_i P_a(x_i) / pn[a]   (L2 projection weights)
    double tproj[P + 1][N];   // w_l L_e(t_l) / ln[e]
    double tpow[N][P + 1];    // t_l^e
    double D[P + 1][P + 1];   // d/dx P_a = sum_{a'} D[a][a'] P_{a'}
    double I[P + 1][P + 2];   // int_0^tau L_e = sum_k I[e][k] tau^k
    constexpr Rules() : x{}, w{}, t{}, px{}, pn{}, lt{}, ln{}, proj{}, tproj{}, tpow{}, D{}, I{}
    {
        for (int i = 0; i < N; ++i) {
            x[i] = gl_node(N, i);
            w[i] = gl_weight(N, i);
            t[i] = 0.5 + x[i];
        }
        for (int a = 0; a <= P; ++a) {
            double s = 0.0, st = 0.0;
            for (int i = 0; i < N; ++i) {
                px[a][i] = mleg(a, x[i]);
                lt[a][i] = tleg(a, t[i]);
                s += w[i] * px[a][i] * px[a][i];     // exact: degree 2a <= 2N - 1
                st += w[i] * lt[a][i] * lt[a][i];
            }
            pn[a] = s;
            ln[a] = st;
        }
        for (int a = 0; a <= P; ++a)
            for (int i = 0; i < N; ++i) {
                proj[a][i] = w[i] * px[a][i] / pn[a];
                tproj[a][i] = w[i] * lt[a][i] / ln[a];
            }
        for (int l = 0; l < N; ++l) {
            double v = 1.0;
            for (int e = 0; e <= P; ++e) { tpow[l][e] = v; v *= t[l]; }
        }
        // derivative map by exact projection of dP_a onto P_{a'}
        for (int a = 0; a <= P; ++a)
            for (int ap = 0; ap <= P; ++ap) {
                double s = 0.0;
                for (int i = 0; i < N; ++i) s += w[i] * dmleg(a, x[i]) * px[ap][i];
                D[a][ap] = (ap < a) ? s / pn[ap] : 0.0;
            }
        // monomial coefficients of L_e by the recurrence, then integrate
        double c[P + 2][P + 2] = {};
        c[0][0] = 1.0;
        if (P >= 1) { c[1][0] = -1.0; c[1][1] = 2.0; }
        for (int n = 1; n < P; ++n)
            for (int k = 0; k <= n + 1; ++k) {
                double two_t_l = (k >= 1 ? 2.0 * c[n][k - 1] : 0.0) - c[n][k];
                c[n + 1][k] = ((2.0 * n + 1.0) * two_t_l - n * c[n - 1][k]) / (n + 1.0);
            }
        for (int e = 0; e <= P; ++e)
            for (int k = 0; k <= P; ++k) I[e][k + 1] = c[e][k] / (k + 1.0);
    }
};

// ---------------------------------------------------------------------------
// Mode lists.  Space-time modes (a, b, c, e) with a + b + c + e <= P in the
// canonical order: e outermost, then c, then b, then a innermost (c = 0 in
// 2D).  The e = 0 block is the list of spatial modes.
// ---------------------------------------------------------------------------
constexpr int binom(int n, int k)
{
    int r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}
constexpr int ipow_c(int b, int e)
{
    int r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

template <int D, int P>
struct Modes {
    static constexpr int NS = binom(P + D, D);          // spatial modes
    static constexpr int NST = binom(P + D + 1, D + 1); // space-time modes
    int a[NST], b[NST], c[NST], e[NST];
    int at[P + 1][P + 1][P + 1][P + 1];   // index of (a, b, c, e), -1 if not a mode
    constexpr Modes() : a{}, b{}, c{}, e{}, at{}
    {
        for (int i0 = 0; i0 <= P; ++i0)
            for (int i1 = 0; i1 <= P; ++i1)
                for (int i2 = 0; i2 <= P; ++i2)
                    for (int i3 = 0; i3 <= P; ++i3) at[i0][i1][i2][i3] = -1;
        int n = 0;
        for (int ee = 0; ee <= P; ++ee)
            for (int cc = 0; cc <= (D == 3 ? P : 0); ++cc)
                for (int bb = 0; bb <= P; ++bb)
                    for (int aa = 0; aa <= P; ++aa)
                        if (aa + bb + cc + ee <= P) {
                            a[n] = aa; b[n] = bb; c[n] = cc; e[n] = ee;
                            at[aa][bb][cc][ee] = n;
                            ++n;
                        }
    }
    constexpr int find(int aa, int bb, int cc, int ee) const
    {
        for (int i = 0; i < NST; ++i)
            if (a[i] == aa && b[i] == bb && c[i] == cc && e[i] == ee) return i;
        return -1;
    }
    constexpr int idx(int d, int m) const { return d == 0 ? a[m] : (d == 1 ? b[m] : c[m]); }
};

// Pair index of (a, b) with a + b <= P in the same order (b outer, a inner):
// the spatial-mode order in 2D and the layout of the y-sweep output in 3D.
template <int P>
struct Pairs {
    int at[P + 1][P + 1];
    constexpr Pairs() : at{}
    {
        int n = 0;
        for (int bb = 0; bb <= P; ++bb)
            for (int aa = 0; aa <= P; ++aa) at[aa][bb] = -1;
        for (int bb = 0; bb <= P; ++bb)
            for (int aa = 0; aa + bb <= P; ++aa) at[aa][bb] = n++;
    }
};

} // namespace hog

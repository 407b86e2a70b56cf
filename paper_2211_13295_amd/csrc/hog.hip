// hog.hip -- C ABI of the gfx950 ADER-WENO Euler zone update: workspace
// planning, argument checks and the per-step launch sequence on the caller's
// HIP stream.  The kernels are in hog_kernels.h.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "hog.h"
#include "hog_kernels.h"
#include "hog_gate.h"
#include "hog_o2.h"
#include "hog_rk.h"
#include "hog_char.h"

using namespace hog;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) return fail(HOG_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Plan {
    int nd, nv, p;
    int es;          // bytes per element of the reconstruction / predictor arrays
    int n[3];
    Pad pad;
    Box I, AX, BY, R, FB[3];
    Box E;           // interior extended by the ghost layers of an external last axis (else I)
    int ms, mst;
    // byte offsets in the workspace
    size_t off_info, off_U[2], off_A, off_B, off_W, off_FP, off_F[3], off_Q, off_stage;
    size_t off_gate, off_flags, off_logits, total;
    // Runge-Kutta: stage states u(1) .. u(s-1) (padded) and dt L(u(k)) (interior)
    int nstages;
    size_t off_S[6], off_L[6];
};

int nmodes(int d, int p) { int r = 1; for (int i = 1; i <= d; ++i) r = r * (p + i) / i; return r; }

int check_cfg(const hog_config* c)
{
    if (!c) return fail(HOG_EINVAL, "config is NULL");
    if (c->ndim != 2 && c->ndim != 3) return fail(HOG_EINVAL, "ndim must be 2 or 3 (got %d)", c->ndim);
    if (c->order < 2 || c->order > 4) return fail(HOG_EINVAL, "order must be 2, 3 or 4 (got %d)", c->order);
    if (c->order == 2 && c->precision != HOG_FP64)
        return fail(HOG_EINVAL, "the second-order scheme runs on the FP64 path only");
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return fail(HOG_EINVAL, "zone counts must be >= 1");
    if (c->ndim == 2 && c->nz != 1) return fail(HOG_EINVAL, "nz must be 1 in 2D");
    if (c->riemann < 0 || c->riemann > 4) return fail(HOG_EINVAL, "unknown Riemann solver %d", c->riemann);
    for (int d = 0; d < 3; ++d)
        if (c->bc[d] != HOG_PERIODIC && c->bc[d] != HOG_OUTFLOW && c->bc[d] != HOG_EXTERNAL)
            return fail(HOG_EINVAL, "bad boundary type on axis %d", d);
    for (int d = 0; d < 3; ++d)
        if (c->bc[d] == HOG_EXTERNAL && d >= c->ndim)
            return fail(HOG_EINVAL, "axis %d is not active in %dD and cannot be external", d, c->ndim);
    for (int d = 0; d < c->ndim; ++d)
        if (c->bc[d] == HOG_EXTERNAL && c->stepper != HOG_ADER)
            return fail(HOG_EINVAL, "an external boundary needs the one-exchange ADER step (Runge-Kutta stages would "
                                    "need new ghost layers each)");
    if (c->precision != HOG_FP64 && c->precision != HOG_MIXED)
        return fail(HOG_EINVAL, "precision %d not supported", c->precision);
    if (c->precision == HOG_MIXED && c->debug)
        return fail(HOG_EINVAL, "space-time mode taps are kept on the FP64 path only");
    if (c->reserved != 0) return fail(HOG_EINVAL, "reserved fields must be 0");
    if (c->characteristic != 0 && c->characteristic != 1) return fail(HOG_EINVAL, "characteristic must be 0 or 1");
    if (c->characteristic && (c->order < 3 || c->precision != HOG_FP64))
        return fail(HOG_EINVAL, "characteristic reconstruction runs at orders 3 and 4 on the FP64 path");
    if (c->stepper != HOG_ADER && !rk_nstages(c->stepper)) return fail(HOG_EINVAL, "unknown stepper %d", c->stepper);
    if (c->stepper != HOG_ADER && (c->precision != HOG_FP64 || c->debug))
        return fail(HOG_EINVAL, "Runge-Kutta stepping runs on the FP64 path without debug taps");
    if (c->positivity != 0 && c->positivity != 1) return fail(HOG_EINVAL, "positivity must be 0 or 1");
    if (!(c->gamma > 1.0) || !std::isfinite(c->gamma)) return fail(HOG_EINVAL, "gamma must be > 1");
    const double h[3] = {c->dx, c->dy, c->dz};
    for (int d = 0; d < c->ndim; ++d)
        if (!(h[d] > 0.0) || !std::isfinite(h[d])) return fail(HOG_EINVAL, "zone width on axis %d must be > 0", d);
    if (!(c->cfl > 0.0) || !(c->cfl <= 1.0)) return fail(HOG_EINVAL, "cfl must be in (0, 1]");
    // periodic wrap of a 5-zone stencil plus one face neighbour needs n >= 3 on periodic axes
    const int n[3] = {c->nx, c->ny, c->nz};
    for (int d = 0; d < c->ndim; ++d)
        if (c->bc[d] == HOG_PERIODIC && n[d] < 3) return fail(HOG_EINVAL, "periodic axis %d needs >= 3 zones", d);
    long long N = (long long)c->nx * c->ny * c->nz;
    if (N > (1ll << 31)) return fail(HOG_EINVAL, "too many zones (%lld)", N);
    return HOG_OK;
}

Box make_box(int l0, int l1, int l2, int n0, int n1, int n2)
{
    Box b;
    b.lo[0] = l0; b.lo[1] = l1; b.lo[2] = l2;
    b.n[0] = n0; b.n[1] = n1; b.n[2] = n2;
    return b;
}

void plan(const hog_config* c, Plan* P)
{
    const int nd = c->ndim, p = c->order - 1, nv = nd + 2;
    P->nd = nd; P->nv = nv; P->p = p;
    const size_t es = (c->precision == HOG_MIXED) ? sizeof(float) : sizeof(double);
    P->es = (int)es;
    P->n[0] = c->nx; P->n[1] = c->ny; P->n[2] = (nd == 3) ? c->nz : 1;
    const int g3 = (nd == 3) ? kGhostZones : 0;
    P->pad.np[0] = P->n[0] + 2 * kGhostZones;
    P->pad.np[1] = P->n[1] + 2 * kGhostZones;
    P->pad.np[2] = P->n[2] + 2 * g3;
    P->pad.off[0] = kGhostZones; P->pad.off[1] = kGhostZones; P->pad.off[2] = g3;
    P->pad.vs = (long long)P->pad.np[0] * P->pad.np[1] * P->pad.np[2];
    const int nx = P->n[0], ny = P->n[1], nz = P->n[2];
    P->I = make_box(0, 0, 0, nx, ny, nz);
    // the zones a caller supplies: the interior grown by the ghost layers
    // along every external axis (edges and corners between external axes too)
    {
        int lo[3] = {0, 0, 0}, ext[3] = {nx, ny, nz};
        for (int d = 0; d < nd; ++d)
            if (c->bc[d] == HOG_EXTERNAL) { lo[d] = -kGhostZones; ext[d] += 2 * kGhostZones; }
        P->E = make_box(lo[0], lo[1], lo[2], ext[0], ext[1], ext[2]);
    }
    if (nd == 3) {
        P->AX = make_box(-1, -3, -3, nx + 2, ny + 6, nz + 6);
        P->BY = make_box(-1, -1, -3, nx + 2, ny + 2, nz + 6);
        P->R = make_box(-1, -1, -1, nx + 2, ny + 2, nz + 2);
        P->FB[2] = make_box(0, 0, -1, nx, ny, nz + 1);
    } else {
        P->AX = make_box(-1, -3, 0, nx + 2, ny + 6, 1);
        P->BY = make_box(-1, -1, 0, nx + 2, ny + 2, 1);
        P->R = P->BY;
        P->FB[2] = make_box(0, 0, 0, 0, 0, 0);
    }
    P->FB[0] = make_box(-1, 0, 0, nx + 1, ny, nz);
    P->FB[1] = make_box(0, -1, 0, nx, ny + 1, nz);
    P->ms = nmodes(nd, p);
    P->mst = nmodes(nd + 1, p);
    const int npairs = (p + 1) * (p + 2) / 2;
    const int npt = 1 << nd;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    P->off_info = take(sizeof(StepInfo));
    P->off_U[0] = take(sizeof(double) * nv * P->pad.vs);
    P->off_U[1] = take(sizeof(double) * nv * P->pad.vs);
    // the second-order kernel keeps its modes, face states and fluxes on chip;
    // face fluxes are stored only for the debug taps
    const bool o2 = (p == 1);
    P->off_A = o2 ? 0 : take(es * (p + 1) * nv * box_size(P->AX));
    P->off_B = o2 ? 0 : take(es * npairs * nv * box_size(P->BY));
    P->off_W = o2 ? 0 : ((nd == 3) ? take(es * P->ms * nv * box_size(P->R)) : P->off_B);
    P->off_FP = o2 ? 0 : take(es * nd * 2 * npt * nv * box_size(P->R));
    for (int d = 0; d < 3; ++d)
        P->off_F[d] = (d < nd && (!o2 || c->debug)) ? take(sizeof(double) * nv * box_size(P->FB[d])) : 0;
    P->off_Q = c->debug ? take(sizeof(double) * P->mst * nv * box_size(P->R)) : 0;
    P->off_stage = take(sizeof(double) * nv * box_size(P->E));
    P->nstages = rk_nstages(c->stepper);
    for (int k = 0; k < 6; ++k) { P->off_S[k] = 0; P->off_L[k] = 0; }
    for (int k = 1; k < P->nstages; ++k) P->off_S[k] = take(sizeof(double) * nv * P->pad.vs);
    for (int k = 0; k < P->nstages; ++k) P->off_L[k] = take(sizeof(double) * nv * box_size(P->I));
    P->off_gate = take(nd == 3 ? sizeof(GateParams<3>) : sizeof(GateParams<2>));
    P->off_flags = take(box_size(P->I));
    P->off_logits = take(sizeof(float) * box_size(P->I));
    P->total = o;
}

} // namespace

struct hog_grid {
    hog_config cfg;
    Plan P;
    hipStream_t stream;
    char* ws;
    size_t ws_bytes;
    int cur;
    bool have_state, have_step, smax_valid;
    long long last_bad;
    WenoArgs wa;
    double h[3];
    int cus;          // compute units of the device (workgroup scheduling of the fused kernels)
    StepInfo* info;
    double* U[2];
    void *A, *B, *W, *FP, *Q;     // element type: double (FP64) or float (mixed)
    double *F[3], *stage;
    double *S[6], *Lb[6];          // Runge-Kutta stage states and dt L buffers
    // learned gate (device copy of the parameters, per-zone flags and logits);
    // gate_on: flags are used by the steps; gate_fixed: they were set by the
    // caller (no inference); gate_net: a network is loaded
    bool gate_on, gate_fixed, gate_net;
    void* gate;
    unsigned char* flags;
    float* logits;
    // stage timing: pairs of events per recorded stage launch, evaluated on read
    bool profiling;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
};

namespace {

inline unsigned nblocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }
// Thread counts of the marching sweeps (one thread per line, chunk, mode, variable).
template <int D, int P>
long long recon_y_threads(const Box& BY)
{
    return (long long)BY.n[0] * BY.n[2] * ((BY.n[1] + kRecChunk - 1) / kRecChunk) * (P + 1) * (D + 2);
}
template <int P>
long long recon_z_threads(const Box& R)
{
    return (long long)R.n[0] * R.n[1] * ((R.n[2] + kRecChunk - 1) / kRecChunk) * ((P + 1) * (P + 2) / 2) * 5;
}

hipEvent_t take_event(hog_grid* g)
{
    if (!g->ev_pool.empty()) {
        hipEvent_t e = g->ev_pool.back();
        g->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// RAII marker: records a start event now and an end event when it goes out
// of scope, both on the handle's stream, if profiling is on.
struct StageMark {
    hog_grid* g;
    int stage;
    hipEvent_t a = nullptr, b = nullptr;
    StageMark(hog_grid* g_, int s) : g(g_), stage(s)
    {
        if (!g->profiling) return;
        a = take_event(g);
        b = take_event(g);
        if (a && b) (void)hipEventRecord(a, g->stream);
    }
    ~StageMark()
    {
        if (!g->profiling || !a || !b) return;
        (void)hipEventRecord(b, g->stream);
        g->ev_used.push_back({stage, {a, b}});
    }
};

int launch_check(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HOG_EDEVICE, "launch of %s failed: %s", what, hipGetErrorString(e));
    return HOG_OK;
}

// The x -> y -> z reconstruction sweeps of the padded state Uc into the
// spatial modes W (component-wise, or on characteristic fields).
template <int D, int P, typename T>
void enqueue_recon(hog_grid* g, const double* Uc, T* A, T* B, T* W, const unsigned char* gf)
{
    const Plan& L = g->P;
    hipStream_t s = g->stream;
    if constexpr (sizeof(T) == 8) {
        if (g->cfg.characteristic) {
            const double gam = g->cfg.gamma;
            k_recon_x_char<D, P><<<nblocks(box_size(L.AX), 256), 256, 0, s>>>(Uc, L.pad, L.AX, A, g->wa, gam, gf,
                                                                              L.I);
            k_recon_y_char<D, P><<<nblocks(recon_y_threads<D, P>(L.BY) / (D + 2), 256), 256, 0, s>>>(
                A, L.AX, L.BY, B, g->wa, gam, gf, L.I);
            if constexpr (D == 3)
                k_recon_z_char<P><<<nblocks(recon_z_threads<P>(L.R) / 5, 256), 256, 0, s>>>(B, L.BY, L.R, W, g->wa,
                                                                                             gam, gf, L.I);
            return;
        }
    }
    k_recon_x<D, P, T><<<nblocks(box_size(L.AX), 256), 256, 0, s>>>(Uc, L.pad, L.AX, A, g->wa, gf, L.I);
    k_recon_y<D, P, T><<<nblocks(recon_y_threads<D, P>(L.BY), 256), 256, 0, s>>>(A, L.AX, L.BY, B, g->wa, gf, L.I);
    if constexpr (D == 3)
        k_recon_z<P, T><<<nblocks(recon_z_threads<P>(L.R), 256), 256, 0, s>>>(B, L.BY, L.R, W, g->wa, gf, L.I);
}

template <int D, int P, typename T>
int enqueue_step_t(hog_grid* g, double dt_user)
{
    T* A = static_cast<T*>(g->A);
    T* B = static_cast<T*>(g->B);
    T* W = static_cast<T*>(g->W);
    T* FPa = static_cast<T*>(g->FP);
    T* Q = static_cast<T*>(g->Q);
    const Plan& L = g->P;
    hipStream_t s = g->stream;
    const double* h = g->h;
    double* Uc = g->U[g->cur];
    double* Un = g->U[g->cur ^ 1];
    k_begin_step<<<1, 1, 0, s>>>(g->info, dt_user, g->cfg.cfl, h[0], h[1], h[2]);
    {
        StageMark m(g, 0);
        const long long npad = (long long)L.pad.np[0] * L.pad.np[1] * L.pad.np[2];
        k_ghost<D><<<nblocks(npad, 256), 256, 0, s>>>(Uc, L.pad, L.n[0], L.n[1], L.n[2], g->cfg.bc[0],
                                                       g->cfg.bc[1], g->cfg.bc[2]);
    }
    {
        const unsigned char* gf = nullptr;
        if (g->gate_on && !g->gate_fixed) {
            StageMark mg(g, 5);
            k_gate_infer<D><<<gate_blocks(box_size(L.I), g->cus), 64 * kGateWaves, 0, s>>>(
                Uc, L.pad, L.I, static_cast<const GateParams<D>*>(g->gate), g->flags, nullptr);
        }
        if (g->gate_on) gf = g->flags;
        StageMark m(g, 1);
        enqueue_recon<D, P, T>(g, Uc, A, B, W, gf);
    }
    {
        StageMark m(g, 2);
        using S = PredShape<D, P>;
        const long long ngroups = (box_size(L.R) + S::ZPW - 1) / S::ZPW;
        k_predict<D, P, T><<<xcd_blocks(ngroups), 64, 0, s>>>(W, L.R, g->info, g->cfg.gamma, g->cfg.positivity,
                                                               FPa, Q);
    }
    {
        StageMark m(g, 3);
        for (int d = 0; d < D; ++d)
            launch_riemann<D, T>(g->cfg.riemann, nblocks(box_size(L.FB[d]), 256), s, FPa, L.R, L.FB[d], d,
                                 g->cfg.gamma, g->F[d]);
    }
    {
        StageMark m(g, 4);
        k_update<D><<<nblocks(box_size(L.I), 256), 256, 0, s>>>(Uc, Un, L.pad, L.I, g->F[0], L.FB[0], g->F[1],
                                                               L.FB[1], g->F[2], L.FB[2], g->info, g->cfg.gamma,
                                                               1.0 / h[0], 1.0 / h[1], 1.0 / h[2]);
    }
    return launch_check("step");
}

// Planes of the march axis per workgroup of the second-order kernel.  MINB
// workgroups are resident per compute unit; the march is cut into as many
// chunks as fill whole rounds of resident workgroups (a partial last round
// leaves compute units idle), using as few rounds as keep the chunks at about
// 32 planes or less (each chunk recomputes two extra planes of modes).
template <int D>
int o2_chunk(const Plan& L, int cus)
{
    using S = O2Shape<D>;
    const long long cols = (long long)((L.n[0] + S::TX - 3) / (S::TX - 2)) *
                           (D == 3 ? (L.n[1] + S::TY - 3) / (S::TY - 2) : 1);
    const long long nm = L.n[D - 1];
    const long long slots = (long long)S::MINB * cus;
    const long long rounds = std::max(1ll, (nm * cols + slots * 32 - 1) / (slots * 32));
    const long long chunks = std::max(1ll, rounds * slots / cols);
    return (int)std::min(nm, (nm + chunks - 1) / chunks);
}

template <int D>
int enqueue_o2(hog_grid* g, double dt_user)
{
    using S = O2Shape<D>;
    const Plan& L = g->P;
    hipStream_t s = g->stream;
    const double* h = g->h;
    k_begin_step<<<1, 1, 0, s>>>(g->info, dt_user, g->cfg.cfl, h[0], h[1], h[2]);
    O2Args a;
    for (int d = 0; d < 3; ++d) { a.n[d] = L.n[d]; a.bc[d] = g->cfg.bc[d]; a.ih[d] = 1.0 / h[d]; }
    a.zc = o2_chunk<D>(L, g->cus);
    a.positivity = g->cfg.positivity;
    a.gamma = g->cfg.gamma;
    const long long nb = (long long)((L.n[0] + S::TX - 3) / (S::TX - 2)) *
                         (D == 3 ? (L.n[1] + S::TY - 3) / (S::TY - 2) : 1) * ((L.n[D - 1] + a.zc - 1) / a.zc);
    {
        StageMark m(g, 2);
        O2Taps tp;
        tp.Q = static_cast<double*>(g->Q);
        tp.R = L.R;
        for (int d = 0; d < 3; ++d) { tp.F[d] = g->F[d]; tp.FB[d] = L.FB[d]; }
        auto launch = [&](auto kernel) {
            kernel<<<xcd_blocks(nb), S::TX * S::TY, 0, s>>>(g->U[g->cur], g->U[g->cur ^ 1], L.pad, a, g->info, tp,
                                                           nullptr);
        };
        const bool taps = g->Q != nullptr;
        if (g->cfg.riemann == HOG_HLLC)
            taps ? launch(k_o2_step<D, HOG_HLLC, true, false>) : launch(k_o2_step<D, HOG_HLLC, false, false>);
        else if (g->cfg.riemann == HOG_HLL)
            taps ? launch(k_o2_step<D, HOG_HLL, true, false>) : launch(k_o2_step<D, HOG_HLL, false, false>);
        else if (g->cfg.riemann == HOG_HLLEM)
            taps ? launch(k_o2_step<D, HOG_HLLEM, true, false>) : launch(k_o2_step<D, HOG_HLLEM, false, false>);
        else if (g->cfg.riemann == HOG_HLLI)
            taps ? launch(k_o2_step<D, HOG_HLLI, true, false>) : launch(k_o2_step<D, HOG_HLLI, false, false>);
        else taps ? launch(k_o2_step<D, HOG_RUSANOV, true, false>) : launch(k_o2_step<D, HOG_RUSANOV, false, false>);
    }
    return launch_check("second-order step");
}

// Runge-Kutta step: per stage, dt L of the previous stage state (reconstruction,
// face points, Riemann solver; at second order the fused kernel) and the
// Shu-Osher combination; the last stage writes the other state buffer and the
// CFL reduction of the new state.
template <int D, int P>
int enqueue_rk(hog_grid* g, double dt_user)
{
    const Plan& L = g->P;
    hipStream_t s = g->stream;
    const double* h = g->h;
    const int st = g->cfg.stepper, ns = L.nstages;
    const RkRow* rows;
    const int nrows = rk_rows(st, &rows);
    k_begin_step<<<1, 1, 0, s>>>(g->info, dt_user, g->cfg.cfl, h[0], h[1], h[2]);
    auto state = [&](int k) -> double* { return k == 0 ? g->U[g->cur] : (k == ns ? g->U[g->cur ^ 1] : g->S[k]); };
    for (int i = 1; i <= ns; ++i) {
        double* src = state(i - 1);
        const bool keep = rk_keep_L(st, i - 1);
        if constexpr (P == 1) {
            using S = O2Shape<D>;
            O2Args a;
            for (int d = 0; d < 3; ++d) { a.n[d] = L.n[d]; a.bc[d] = g->cfg.bc[d]; a.ih[d] = 1.0 / h[d]; }
            a.zc = o2_chunk<D>(L, g->cus);
            a.positivity = g->cfg.positivity;
            a.gamma = g->cfg.gamma;
            const long long nb = (long long)((L.n[0] + S::TX - 3) / (S::TX - 2)) *
                                 (D == 3 ? (L.n[1] + S::TY - 3) / (S::TY - 2) : 1) *
                                 ((L.n[D - 1] + a.zc - 1) / a.zc);
            O2Taps tp;
            std::memset(&tp, 0, sizeof tp);
            StageMark m(g, 2);
            auto launch = [&](auto kernel) {
                kernel<<<xcd_blocks(nb), S::TX * S::TY, 0, s>>>(src, nullptr, L.pad, a, g->info, tp, g->Lb[i - 1]);
            };
            if (g->cfg.riemann == HOG_HLLC) launch(k_o2_step<D, HOG_HLLC, false, true>);
            else if (g->cfg.riemann == HOG_HLL) launch(k_o2_step<D, HOG_HLL, false, true>);
            else if (g->cfg.riemann == HOG_HLLEM) launch(k_o2_step<D, HOG_HLLEM, false, true>);
            else if (g->cfg.riemann == HOG_HLLI) launch(k_o2_step<D, HOG_HLLI, false, true>);
            else launch(k_o2_step<D, HOG_RUSANOV, false, true>);
        } else {
            double* A = static_cast<double*>(g->A);
            double* B = static_cast<double*>(g->B);
            double* W = static_cast<double*>(g->W);
            double* FPa = static_cast<double*>(g->FP);
            {
                StageMark m(g, 0);
                const long long npad = (long long)L.pad.np[0] * L.pad.np[1] * L.pad.np[2];
                k_ghost<D><<<nblocks(npad, 256), 256, 0, s>>>(src, L.pad, L.n[0], L.n[1], L.n[2], g->cfg.bc[0],
                                                               g->cfg.bc[1], g->cfg.bc[2]);
            }
            {
                StageMark m(g, 1);
                enqueue_recon<D, P, double>(g, src, A, B, W, nullptr);
            }
            {
                StageMark m(g, 2);
                k_face_points<D, P><<<nblocks(box_size(L.R), 256), 256, 0, s>>>(
                    W, L.R, g->info, g->cfg.gamma, g->cfg.positivity, FPa);
            }
            {
                StageMark m(g, 3);
                for (int d = 0; d < D; ++d)
                    launch_riemann<D, double, (1 << (D - 1))>(g->cfg.riemann, nblocks(box_size(L.FB[d]), 256), s,
                                                              FPa, L.R, L.FB[d], d, g->cfg.gamma, g->F[d]);
            }
        }
        RkStage sg;
        sg.n = 0;
        for (int r = 0; r < nrows; ++r) {
            if (rows[r].i != i) continue;
            sg.src[sg.n] = state(rows[r].k);
            sg.padded[sg.n] = 1;
            sg.coef[sg.n] = rows[r].alpha;
            ++sg.n;
            if (rows[r].beta != 0.0) {
                sg.src[sg.n] = (rows[r].k == i - 1) ? nullptr : g->Lb[rows[r].k];
                sg.padded[sg.n] = 0;
                sg.coef[sg.n] = rows[r].beta;
                ++sg.n;
            }
        }
        StageMark m(g, 4);
        const bool o2 = (P == 1);
        k_rk_combine<D><<<nblocks(box_size(L.I), 256), 256, 0, s>>>(
            L.pad, L.I, g->F[0], L.FB[0], g->F[1], L.FB[1], g->F[2], L.FB[2], o2 ? g->Lb[i - 1] : nullptr,
            (!o2 && keep) ? g->Lb[i - 1] : nullptr, sg, state(i), g->info, i == ns ? 1 : 0, g->cfg.gamma,
            1.0 / h[0], 1.0 / h[1], 1.0 / h[2]);
    }
    return launch_check("Runge-Kutta step");
}

int enqueue_step(hog_grid* g, double dt_user)
{
    if (g->cfg.stepper != HOG_ADER) {
        switch (g->P.nd * 10 + g->P.p) {
        case 21: return enqueue_rk<2, 1>(g, dt_user);
        case 22: return enqueue_rk<2, 2>(g, dt_user);
        case 23: return enqueue_rk<2, 3>(g, dt_user);
        case 31: return enqueue_rk<3, 1>(g, dt_user);
        case 32: return enqueue_rk<3, 2>(g, dt_user);
        case 33: return enqueue_rk<3, 3>(g, dt_user);
        }
        return fail(HOG_EINVAL, "unsupported dimension/order");
    }
    if (g->P.p == 1) return g->P.nd == 3 ? enqueue_o2<3>(g, dt_user) : enqueue_o2<2>(g, dt_user);
    const int key = (g->cfg.precision == HOG_MIXED ? 100 : 0) + g->P.nd * 10 + g->P.p;
    switch (key) {
    case 22: return enqueue_step_t<2, 2, double>(g, dt_user);
    case 23: return enqueue_step_t<2, 3, double>(g, dt_user);
    case 32: return enqueue_step_t<3, 2, double>(g, dt_user);
    case 33: return enqueue_step_t<3, 3, double>(g, dt_user);
    case 122: return enqueue_step_t<2, 2, float>(g, dt_user);
    case 123: return enqueue_step_t<2, 3, float>(g, dt_user);
    case 132: return enqueue_step_t<3, 2, float>(g, dt_user);
    case 133: return enqueue_step_t<3, 3, float>(g, dt_user);
    }
    return fail(HOG_EINVAL, "unsupported dimension/order");
}

int enqueue_cfl(hog_grid* g, int which)
{
    const Plan& L = g->P;
    k_reset<<<1, 1, 0, g->stream>>>(g->info, 0.0, 0);
    if (L.nd == 3)
        k_cfl<3><<<nblocks(box_size(L.I), 256), 256, 0, g->stream>>>(g->U[which], L.pad, L.I, g->info,
                                                                      g->cfg.gamma, 1.0 / g->h[0], 1.0 / g->h[1],
                                                                      1.0 / g->h[2]);
    else
        k_cfl<2><<<nblocks(box_size(L.I), 256), 256, 0, g->stream>>>(g->U[which], L.pad, L.I, g->info,
                                                                      g->cfg.gamma, 1.0 / g->h[0], 1.0 / g->h[1],
                                                                      1.0 / g->h[2]);
    return launch_check("cfl");
}

int read_info(hog_grid* g, StepInfo* out)
{
    HIP_TRY(hipMemcpyAsync(out, g->info, sizeof(StepInfo), hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    return HOG_OK;
}

double smax_of(const StepInfo& si)
{
    double s;
    std::memcpy(&s, &si.smax_bits, sizeof s);
    return s;
}

// The current device must be a gfx950 GPU; *cus receives its compute units.
int device_check(int* cus)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(HOG_EDEVICE, "device %d is %s, this library is built for gfx950", dev, prop.gcnArchName);
    *cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    return HOG_OK;
}

// Point a handle at the pieces of a workspace laid out by plan() and set its
// scheme constants.  Enqueues nothing and allocates nothing.
void bind_grid(hog_grid* g, const hog_config* cfg, const Plan& P, char* ws, size_t bytes, hipStream_t stream,
               int cus)
{
    g->cfg = *cfg;
    g->P = P;
    g->cus = cus;
    g->stream = stream;
    g->ws = ws;
    g->ws_bytes = bytes;
    g->cur = 0;
    g->have_state = g->have_step = g->smax_valid = false;
    g->profiling = false;
    g->last_bad = -1;
    g->h[0] = cfg->dx; g->h[1] = cfg->dy; g->h[2] = (P.nd == 3) ? cfg->dz : 1.0;
    g->wa.eps = cfg->weno_eps > 0.0 ? cfg->weno_eps : 1e-12;
    const bool g3zero = cfg->g3[0] == 0.0 && cfg->g3[1] == 0.0 && cfg->g3[2] == 0.0;
    const bool g4zero = cfg->g4[0] == 0.0 && cfg->g4[1] == 0.0 && cfg->g4[2] == 0.0 && cfg->g4[3] == 0.0;
    if (P.p == 2) {
        const double d3[3] = {0.075, 0.85, 0.075};
        for (int i = 0; i < 3; ++i) g->wa.g[i] = g3zero ? d3[i] : cfg->g3[i];
        g->wa.g[3] = 0.0;
    } else {
        const double d4[4] = {0.85, 0.01125, 0.1275, 0.01125};
        for (int i = 0; i < 4; ++i) g->wa.g[i] = g4zero ? d4[i] : cfg->g4[i];
    }
    g->wa.linear = cfg->linear_weno ? 1 : 0;
    g->info = reinterpret_cast<StepInfo*>(ws + P.off_info);
    g->U[0] = reinterpret_cast<double*>(ws + P.off_U[0]);
    g->U[1] = reinterpret_cast<double*>(ws + P.off_U[1]);
    g->A = (P.p > 1) ? ws + P.off_A : nullptr;
    g->B = (P.p > 1) ? ws + P.off_B : nullptr;
    g->W = (P.p > 1) ? ws + P.off_W : nullptr;
    g->FP = (P.p > 1) ? ws + P.off_FP : nullptr;
    for (int d = 0; d < 3; ++d)
        g->F[d] = (d < P.nd && (P.p > 1 || cfg->debug)) ? reinterpret_cast<double*>(ws + P.off_F[d]) : nullptr;
    g->Q = cfg->debug ? static_cast<void*>(ws + P.off_Q) : nullptr;
    g->stage = reinterpret_cast<double*>(ws + P.off_stage);
    for (int k = 0; k < 6; ++k) {
        g->S[k] = (k >= 1 && k < P.nstages) ? reinterpret_cast<double*>(ws + P.off_S[k]) : nullptr;
        g->Lb[k] = (k < P.nstages) ? reinterpret_cast<double*>(ws + P.off_L[k]) : nullptr;
    }
    g->gate_on = g->gate_fixed = g->gate_net = false;
    g->gate = ws + P.off_gate;
    g->flags = reinterpret_cast<unsigned char*>(ws + P.off_flags);
    g->logits = reinterpret_cast<float*>(ws + P.off_logits);
}

} // namespace

extern "C" {

int hog_abi_version(void) { return HOG_ABI_VERSION; }

const char* hog_last_error(void) { return g_err; }

int hog_workspace_size(const hog_config* cfg, size_t* bytes)
{
    int rc = check_cfg(cfg);
    if (rc) return rc;
    if (!bytes) return fail(HOG_EINVAL, "bytes is NULL");
    Plan P;
    plan(cfg, &P);
    *bytes = P.total;
    return HOG_OK;
}

int hog_create(const hog_config* cfg, void* workspace, size_t bytes, void* hip_stream, hog_grid** out)
{
    g_err[0] = 0;
    int rc = check_cfg(cfg);
    if (rc) return rc;
    if (!out) return fail(HOG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!workspace) return fail(HOG_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(HOG_EINVAL, "workspace must be 256-byte aligned");
    Plan P;
    plan(cfg, &P);
    if (bytes < P.total) return fail(HOG_ENOMEM, "workspace too small: %zu < %zu bytes", bytes, P.total);
    int cus = 0;
    rc = device_check(&cus);
    if (rc) return rc;
    hog_grid* g = new (std::nothrow) hog_grid();
    if (!g) return fail(HOG_ENOMEM, "host allocation failed");
    bind_grid(g, cfg, P, static_cast<char*>(workspace), bytes, static_cast<hipStream_t>(hip_stream), cus);
    k_reset<<<1, 1, 0, g->stream>>>(g->info, 0.0, 1);
    rc = launch_check("reset");
    if (rc) { delete g; return rc; }
    *out = g;
    return HOG_OK;
}

int hog_destroy(hog_grid* g)
{
    if (!g) return HOG_OK;
    if (!g->ev_used.empty()) (void)hipStreamSynchronize(g->stream);
    for (auto& u : g->ev_used) {
        (void)hipEventDestroy(u.second.first);
        (void)hipEventDestroy(u.second.second);
    }
    for (auto e : g->ev_pool) (void)hipEventDestroy(e);
    delete g;
    return HOG_OK;
}

int hog_profile_enable(hog_grid* g, int enable)
{
    if (!g) return fail(HOG_EINVAL, "NULL handle");
    g->profiling = enable != 0;
    return HOG_OK;
}

int hog_profile_read(hog_grid* g, double* ms, int* launches, int nstages)
{
    if (!g || !ms || !launches || nstages < HOG_NSTAGES) return fail(HOG_EINVAL, "bad arguments");
    for (int i = 0; i < nstages; ++i) { ms[i] = 0.0; launches[i] = 0; }
    HIP_TRY(hipStreamSynchronize(g->stream));
    for (auto& u : g->ev_used) {
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, u.second.first, u.second.second));
        ms[u.first] += t;
        launches[u.first] += 1;
        g->ev_pool.push_back(u.second.first);
        g->ev_pool.push_back(u.second.second);
    }
    g->ev_used.clear();
    return HOG_OK;
}

int hog_set_state(hog_grid* g, const double* U, int layout, int where)
{
    if (!g || !U) return fail(HOG_EINVAL, "NULL argument");
    if (layout != HOG_SOA && layout != HOG_AOS) return fail(HOG_EINVAL, "unknown layout %d", layout);
    if (where != HOG_HOST && where != HOG_DEVICE) return fail(HOG_EINVAL, "unknown location %d", where);
    const Plan& L = g->P;
    const long long N = box_size(L.I);
    const double* src = U;
    if (where == HOG_HOST) {
        HIP_TRY(hipMemcpyAsync(g->stage, U, sizeof(double) * L.nv * N, hipMemcpyHostToDevice, g->stream));
        HIP_TRY(hipStreamSynchronize(g->stream));
        src = g->stage;
    }
    const int aos = layout == HOG_AOS;
    if (L.nd == 3) k_pack<3><<<nblocks(N, 256), 256, 0, g->stream>>>(src, g->U[g->cur], L.pad, L.I, aos);
    else k_pack<2><<<nblocks(N, 256), 256, 0, g->stream>>>(src, g->U[g->cur], L.pad, L.I, aos);
    int rc = launch_check("pack");
    if (rc) return rc;
    rc = enqueue_cfl(g, g->cur);
    if (rc) return rc;
    g->have_state = true;
    g->smax_valid = true;
    g->have_step = false;
    return HOG_OK;
}

int hog_set_state_ext(hog_grid* g, const double* U, int where)
{
    if (!g || !U) return fail(HOG_EINVAL, "NULL argument");
    if (where != HOG_HOST && where != HOG_DEVICE) return fail(HOG_EINVAL, "unknown location %d", where);
    const Plan& L = g->P;
    bool any = false;
    for (int d = 0; d < L.nd; ++d) any = any || g->cfg.bc[d] == HOG_EXTERNAL;
    if (!any) return fail(HOG_EINVAL, "no axis is external");
    const long long NE = box_size(L.E);
    const double* src = U;
    if (where == HOG_HOST) {
        HIP_TRY(hipMemcpyAsync(g->stage, U, sizeof(double) * L.nv * NE, hipMemcpyHostToDevice, g->stream));
        HIP_TRY(hipStreamSynchronize(g->stream));
        src = g->stage;
    }
    if (L.nd == 3) k_pack<3><<<nblocks(NE, 256), 256, 0, g->stream>>>(src, g->U[g->cur], L.pad, L.E, 0);
    else k_pack<2><<<nblocks(NE, 256), 256, 0, g->stream>>>(src, g->U[g->cur], L.pad, L.E, 0);
    int rc = launch_check("pack");
    if (rc) return rc;
    rc = enqueue_cfl(g, g->cur);
    if (rc) return rc;
    g->have_state = true;
    g->smax_valid = true;
    g->have_step = false;
    return HOG_OK;
}

int hog_get_state(hog_grid* g, double* U, int layout, int where)
{
    if (!g || !U) return fail(HOG_EINVAL, "NULL argument");
    if (layout != HOG_SOA && layout != HOG_AOS) return fail(HOG_EINVAL, "unknown layout %d", layout);
    if (where != HOG_HOST && where != HOG_DEVICE) return fail(HOG_EINVAL, "unknown location %d", where);
    if (!g->have_state) return fail(HOG_ESTATE, "no state set");
    const Plan& L = g->P;
    const long long N = box_size(L.I);
    double* dst = (where == HOG_DEVICE) ? U : g->stage;
    const int aos = layout == HOG_AOS;
    if (L.nd == 3) k_unpack<3><<<nblocks(N, 256), 256, 0, g->stream>>>(g->U[g->cur], dst, L.pad, L.I, aos);
    else k_unpack<2><<<nblocks(N, 256), 256, 0, g->stream>>>(g->U[g->cur], dst, L.pad, L.I, aos);
    int rc = launch_check("unpack");
    if (rc) return rc;
    if (where == HOG_HOST) {
        HIP_TRY(hipMemcpyAsync(U, g->stage, sizeof(double) * L.nv * N, hipMemcpyDeviceToHost, g->stream));
        HIP_TRY(hipStreamSynchronize(g->stream));
    }
    return HOG_OK;
}

int hog_compute_dt(hog_grid* g, double* dt)
{
    if (!g || !dt) return fail(HOG_EINVAL, "NULL argument");
    if (!g->have_state) return fail(HOG_ESTATE, "no state set");
    int rc;
    if (!g->smax_valid) {
        rc = enqueue_cfl(g, g->cur);
        if (rc) return rc;
        g->smax_valid = true;
    }
    StepInfo si;
    rc = read_info(g, &si);
    if (rc) return rc;
    if (si.bad != ULLONG_MAX) {
        g->last_bad = (long long)si.bad;
        return fail(HOG_ENONPHYS, "non-physical state in zone %lld", g->last_bad);
    }
    g->last_bad = -1;
    *dt = g->cfg.cfl / smax_of(si);
    return HOG_OK;
}

int hog_step(hog_grid* g, double dt, double* dt_next)
{
    if (!g) return fail(HOG_EINVAL, "NULL handle");
    if (!g->have_state) return fail(HOG_ESTATE, "no state set");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(HOG_EINVAL, "dt must be finite and > 0 (got %g)", dt);
    int rc = enqueue_step(g, dt);
    if (rc) return rc;
    g->have_step = true;
    if (!dt_next) {
        g->cur ^= 1;
        g->smax_valid = true;
        return HOG_OK;
    }
    StepInfo si;
    rc = read_info(g, &si);
    if (rc) return rc;
    if (si.bad != ULLONG_MAX) {
        g->last_bad = (long long)si.bad;
        // keep the pre-step state; its CFL reduction is recomputed on demand
        g->smax_valid = false;
        return fail(HOG_ENONPHYS, "step produced a non-physical state in zone %lld", g->last_bad);
    }
    g->last_bad = -1;
    g->cur ^= 1;
    g->smax_valid = true;
    *dt_next = g->cfg.cfl / smax_of(si);
    return HOG_OK;
}

int hog_advance(hog_grid* g, int nsteps, double t_end, double* t_out)
{
    if (!g) return fail(HOG_EINVAL, "NULL handle");
    if (!g->have_state) return fail(HOG_ESTATE, "no state set");
    if (nsteps < 0 || !std::isfinite(t_end)) return fail(HOG_EINVAL, "bad nsteps / t_end");
    int rc;
    if (!g->smax_valid) {
        rc = enqueue_cfl(g, g->cur);
        if (rc) return rc;
        g->smax_valid = true;
    }
    // reset the time accumulator without touching the CFL reduction, and make
    // a non-physical state halt the run (later steps of it write no new state)
    {
        StepInfo si;
        rc = read_info(g, &si);
        if (rc) return rc;
        if (si.bad != ULLONG_MAX) {
            g->last_bad = (long long)si.bad;
            return fail(HOG_ENONPHYS, "non-physical state in zone %lld", g->last_bad);
        }
        si.t = 0.0;
        si.t_end = t_end > 0.0 ? t_end : 0.0;
        si.nstep = 0ull;
        si.sticky = 1;
        si.halted = 0;
        HIP_TRY(hipMemcpyAsync(g->info, &si, sizeof si, hipMemcpyHostToDevice, g->stream));
        HIP_TRY(hipStreamSynchronize(g->stream));
    }
    const int cur0 = g->cur;
    StepInfo si;
    for (int s = 0; s < nsteps; ++s) {
        rc = enqueue_step(g, -1.0);
        if (rc) return rc;
        g->cur ^= 1;
        g->have_step = true;
        if (t_end > 0.0) {
            rc = read_info(g, &si);
            if (rc) return rc;
            if (si.bad != ULLONG_MAX) break;
            if (si.t >= t_end * (1.0 - 1e-14) || si.dt <= 0.0) break;
        }
    }
    rc = read_info(g, &si);
    if (rc) return rc;
    k_arm<<<1, 1, 0, g->stream>>>(g->info, 0);
    rc = launch_check("arm");
    if (rc) return rc;
    if (si.bad != ULLONG_MAX) {
        // step nstep - 1 (counted from 0) made the non-physical state; its
        // input, the last admissible state, is still in its buffer
        const unsigned long long f = si.nstep > 0 ? si.nstep - 1 : 0;
        g->cur = cur0 ^ (int)(f & 1ull);
        g->smax_valid = false;
        g->last_bad = (long long)si.bad;
        return fail(HOG_ENONPHYS, "step %llu of the run produced a non-physical state in zone %lld; the state "
                                  "before that step is kept", f + 1, g->last_bad);
    }
    g->last_bad = -1;
    if (t_out) *t_out = si.t;
    return HOG_OK;
}

long long hog_last_bad_zone(hog_grid* g) { return g ? g->last_bad : -1; }

int hog_stats(hog_grid* g, double* t, double* dt, long long* fallback_zones)
{
    if (!g) return fail(HOG_EINVAL, "NULL handle");
    StepInfo si;
    int rc = read_info(g, &si);
    if (rc) return rc;
    if (t) *t = si.t;
    if (dt) *dt = si.dt;
    if (fallback_zones) *fallback_zones = (long long)si.fallback;
    return HOG_OK;
}

int hog_debug_tap(hog_grid* g, int tap, void* dst, size_t bytes)
{
    if (!g || !dst) return fail(HOG_EINVAL, "NULL argument");
    if (!g->have_step) return fail(HOG_ESTATE, "no step taken yet");
    const Plan& L = g->P;
    const long long N = box_size(L.I), nR = box_size(L.R);
    const int nv = L.nv;
    if (tap == HOG_TAP_MODES || tap == HOG_TAP_STMODES) {
        const int nm = (tap == HOG_TAP_MODES) ? L.ms : L.mst;
        // at second order the mean and slopes are the first 1 + nd space-time modes
        const void* src = (tap == HOG_TAP_MODES && L.p > 1) ? g->W : g->Q;
        if (!src) return fail(HOG_EINVAL, "space-time modes are kept only with debug = 1");
        if (bytes < sizeof(double) * N * nm * nv) return fail(HOG_EINVAL, "tap buffer too small");
        const size_t n = (size_t)nm * nv * nR;
        std::vector<char> h(n * L.es);
        HIP_TRY(hipMemcpyAsync(h.data(), src, h.size(), hipMemcpyDeviceToHost, g->stream));
        HIP_TRY(hipStreamSynchronize(g->stream));
        auto at = [&](size_t i) {
            return L.es == 8 ? reinterpret_cast<const double*>(h.data())[i]
                             : (double)reinterpret_cast<const float*>(h.data())[i];
        };
        double* out = static_cast<double*>(dst);
        for (int k = 0; k < L.n[2]; ++k)
            for (int j = 0; j < L.n[1]; ++j)
                for (int i = 0; i < L.n[0]; ++i) {
                    const long long z = ((long long)k * L.n[1] + j) * L.n[0] + i;
                    const long long r = ((long long)(k - L.R.lo[2]) * L.R.n[1] + (j - L.R.lo[1])) * L.R.n[0] +
                                        (i - L.R.lo[0]);
                    for (int m = 0; m < nm; ++m)
                        for (int v = 0; v < nv; ++v) out[(z * nm + m) * nv + v] = at(((size_t)m * nv + v) * nR + r);
                }
        return HOG_OK;
    }
    if (tap >= HOG_TAP_FLUX_X && tap <= HOG_TAP_FLUX_Z) {
        const int d = tap - HOG_TAP_FLUX_X;
        if (d >= L.nd) return fail(HOG_EINVAL, "no z faces in 2D");
        const long long nF = box_size(L.FB[d]);
        if (bytes < sizeof(double) * nv * nF) return fail(HOG_EINVAL, "tap buffer too small");
        HIP_TRY(hipMemcpyAsync(dst, g->F[d], sizeof(double) * nv * nF, hipMemcpyDeviceToHost, g->stream));
        HIP_TRY(hipStreamSynchronize(g->stream));
        return HOG_OK;
    }
    return fail(HOG_EINVAL, "unknown tap %d", tap);
}

// ------------------------------------------------------------------------
// Learned gate
// ------------------------------------------------------------------------
static uint16_t host_bf16(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

int hog_gate_param_count(int ndim, int* count)
{
    if ((ndim != 2 && ndim != 3) || !count) return fail(HOG_EINVAL, "bad arguments");
    *count = (ndim == 3) ? GateShape<3>::NPARAM : GateShape<2>::NPARAM;
    return HOG_OK;
}

extern "C++" {
template <int D>
static int set_gate_t(hog_grid* g, const float* prm, double theta)
{
    using G = GateShape<D>;
    using O = MlpOffsets<G::NF>;
    GateParams<D> h;
    std::memset(&h, 0, sizeof h);
    for (int o = 0; o < kHidden; ++o)
        for (int f = 0; f < G::NF; ++f)   // device feature layout: variable blocks of NCB columns
            h.W1[o][(f / G::NC) * G::NCB + f % G::NC] = host_bf16(prm[O::W1 + o * G::NF + f]);
    // the inputs of layers 2 and 3 in the order the inference kernel's
    // fragments hold them: position q carries hidden unit gate_unit(q)
    for (int o = 0; o < kHidden; ++o) {
        h.b1[o] = prm[O::B1 + o];
        h.b2[o] = prm[O::B2 + o];
        h.w3[o] = host_bf16(prm[O::W3 + gate_unit(o)]);
        for (int q = 0; q < kHidden; ++q) h.W2[o][q] = host_bf16(prm[O::W2 + o * kHidden + gate_unit(q)]);
    }
    h.b3 = prm[O::B3];
    h.logit_thr = (float)std::log(theta / (1.0 - theta));
    HIP_TRY(hipMemcpyAsync(g->gate, &h, sizeof h, hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    return HOG_OK;
}
} // extern "C++"

int hog_set_gate(hog_grid* g, const float* params, double theta)
{
    if (!g) return fail(HOG_EINVAL, "NULL handle");
    g->gate_fixed = false;
    if (!params) { g->gate_on = g->gate_net = false; return HOG_OK; }
    if (g->P.p == 1) return fail(HOG_EINVAL, "the second-order scheme has no WENO weights to gate");
    if (g->cfg.stepper != HOG_ADER) return fail(HOG_EINVAL, "the gate runs with the ADER step only");
    if (!(theta > 0.0 && theta < 1.0)) return fail(HOG_EINVAL, "theta must be in (0, 1)");
    const int rc = (g->P.nd == 3) ? set_gate_t<3>(g, params, theta) : set_gate_t<2>(g, params, theta);
    if (rc) { g->gate_on = g->gate_net = false; return rc; }
    g->gate_on = g->gate_net = true;
    return HOG_OK;
}

int hog_set_gate_flags(hog_grid* g, const unsigned char* flags)
{
    if (!g) return fail(HOG_EINVAL, "NULL handle");
    if (!flags) {
        g->gate_fixed = false;
        g->gate_on = g->gate_net;
        return HOG_OK;
    }
    if (g->P.p == 1) return fail(HOG_EINVAL, "the second-order scheme has no WENO weights to gate");
    if (g->cfg.stepper != HOG_ADER) return fail(HOG_EINVAL, "the gate runs with the ADER step only");
    const long long N = box_size(g->P.I);
    for (long long i = 0; i < N; ++i)
        if (flags[i] > 1) return fail(HOG_EINVAL, "flags must be 0 or 1 (zone %lld)", i);
    HIP_TRY(hipMemcpyAsync(g->flags, flags, N, hipMemcpyHostToDevice, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    g->gate_fixed = g->gate_on = true;
    return HOG_OK;
}

static void enqueue_ghost(hog_grid* g)
{
    const Plan& L = g->P;
    const long long npad = (long long)L.pad.np[0] * L.pad.np[1] * L.pad.np[2];
    if (L.nd == 3)
        k_ghost<3><<<nblocks(npad, 256), 256, 0, g->stream>>>(g->U[g->cur], L.pad, L.n[0], L.n[1], L.n[2],
                                                               g->cfg.bc[0], g->cfg.bc[1], g->cfg.bc[2]);
    else
        k_ghost<2><<<nblocks(npad, 256), 256, 0, g->stream>>>(g->U[g->cur], L.pad, L.n[0], L.n[1], L.n[2],
                                                               g->cfg.bc[0], g->cfg.bc[1], g->cfg.bc[2]);
}

int hog_gate_eval(hog_grid* g, float* logits, unsigned char* flags)
{
    if (!g) return fail(HOG_EINVAL, "NULL handle");
    if (!g->gate_net) return fail(HOG_ESTATE, "no gate network set");
    if (g->gate_fixed) return fail(HOG_ESTATE, "fixed gate flags are set");
    if (!g->have_state) return fail(HOG_ESTATE, "no state set");
    const Plan& L = g->P;
    const long long N = box_size(L.I);
    enqueue_ghost(g);
    if (L.nd == 3)
        k_gate_infer<3><<<gate_blocks(N, g->cus), 64 * kGateWaves, 0, g->stream>>>(g->U[g->cur], L.pad, L.I,
                                                               static_cast<const GateParams<3>*>(g->gate), g->flags,
                                                               g->logits);
    else
        k_gate_infer<2><<<gate_blocks(N, g->cus), 64 * kGateWaves, 0, g->stream>>>(g->U[g->cur], L.pad, L.I,
                                                               static_cast<const GateParams<2>*>(g->gate), g->flags,
                                                               g->logits);
    int rc = launch_check("gate");
    if (rc) return rc;
    if (logits) HIP_TRY(hipMemcpyAsync(logits, g->logits, sizeof(float) * N, hipMemcpyDeviceToHost, g->stream));
    if (flags) HIP_TRY(hipMemcpyAsync(flags, g->flags, N, hipMemcpyDeviceToHost, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    return HOG_OK;
}

extern "C++" {
template <int D, int P>
static void enqueue_harvest(hog_grid* g, const long long* zones, long long n, float* feat, float* maxdev)
{
    const Plan& L = g->P;
    hipStream_t s = g->stream;
    double* Uc = g->U[g->cur];
    double* A = static_cast<double*>(g->A);
    double* B = static_cast<double*>(g->B);
    k_recon_x<D, P, double><<<nblocks(box_size(L.AX), 256), 256, 0, s>>>(Uc, L.pad, L.AX, A, g->wa, nullptr, L.I);
    k_recon_y<D, P, double><<<nblocks(recon_y_threads<D, P>(L.BY), 256), 256, 0, s>>>(A, L.AX, L.BY, B, g->wa,
                                                                                       nullptr, L.I);
    k_harvest<D, P><<<nblocks(n, 256), 256, 0, s>>>(Uc, L.pad, L.I, A, L.AX, B, L.BY, zones, n, g->wa, feat, maxdev);
}
} // extern "C++"

int hog_harvest(hog_grid* g, const long long* zones, long long n, float* features, float* maxdev)
{
    if (!g || !zones || !features || !maxdev || n < 0) return fail(HOG_EINVAL, "bad arguments");
    if (!g->have_state) return fail(HOG_ESTATE, "no state set");
    if (g->cfg.precision != HOG_FP64) return fail(HOG_EINVAL, "harvest runs on the FP64 path");
    if (g->P.p == 1) return fail(HOG_EINVAL, "the second-order scheme has no WENO weights to harvest");
    if (n == 0) return HOG_OK;
    enqueue_ghost(g);
    switch (g->P.nd * 10 + g->P.p) {
    case 22: enqueue_harvest<2, 2>(g, zones, n, features, maxdev); break;
    case 23: enqueue_harvest<2, 3>(g, zones, n, features, maxdev); break;
    case 32: enqueue_harvest<3, 2>(g, zones, n, features, maxdev); break;
    case 33: enqueue_harvest<3, 3>(g, zones, n, features, maxdev); break;
    }
    return launch_check("harvest");
}

} // extern "C"

// ------------------------------------------------------------------------
// Gate training
// ------------------------------------------------------------------------
struct hog_mlp {
    int nf, batch_max, np, t, nbmax;
    hipStream_t stream;
    float *prm, *m, *v, *grad, *lsum, *partial;
    MlpBatch bt;
};

static int mlp_nparam(int nf) { return kHidden * nf + kHidden + kHidden * kHidden + kHidden + kHidden + 1; }
static int mlp_nb(int n) { return (n + 255) / 256 * 256; }

// Workspace: FP32 parameters, Adam moments and gradient; the per-batch BF16
// arrays (transposed, [row][sample]) and FP32 per-sample values; the partial
// gradient tiles of each 256-sample chunk.
static size_t mlp_bytes(int nf, int batch_max, int np, size_t off[12])
{
    const int nb = mlp_nb(batch_max);
    const int nfp = (nf + 15) / 16 * 16;
    const int ntile = 4 * (nfp / 16) + 16;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    off[0] = take(sizeof(float) * np);                       // prm
    off[1] = take(sizeof(float) * np);                       // m
    off[2] = take(sizeof(float) * np);                       // v
    off[3] = take(sizeof(float) * np);                       // grad
    off[4] = take(sizeof(uint16_t) * (size_t)nfp * nb);      // XT
    off[5] = take(sizeof(uint16_t) * (size_t)kHidden * nb);  // H1T
    off[6] = take(sizeof(uint16_t) * (size_t)kHidden * nb);  // H2T
    off[7] = take(sizeof(uint16_t) * 2 * (size_t)kHidden * nb);   // D1T (hi, lo)
    off[8] = take(sizeof(uint16_t) * 2 * (size_t)kHidden * nb);   // D2T (hi, lo)
    off[9] = take(sizeof(float) * 3 * (size_t)nb + 64);      // dz, loss, logit, loss sum
    off[10] = take(sizeof(float) * (size_t)(nb / 256) * ntile * 256);   // partial tiles
    return o;
}

extern "C" {

int hog_mlp_workspace_size(int nf, int batch_max, size_t* bytes)
{
    if ((nf != 36 && nf != 65) || batch_max < 1 || !bytes) return fail(HOG_EINVAL, "nf must be 36 or 65");
    size_t off[12];
    *bytes = mlp_bytes(nf, batch_max, mlp_nparam(nf), off);
    return HOG_OK;
}

int hog_mlp_create(int nf, int batch_max, void* ws, size_t bytes, void* stream, hog_mlp** out)
{
    size_t need = 0;
    int rc = hog_mlp_workspace_size(nf, batch_max, &need);
    if (rc) return rc;
    if (!ws || !out) return fail(HOG_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(HOG_EINVAL, "workspace must be 256-byte aligned");
    if (bytes < need) return fail(HOG_ENOMEM, "workspace too small: %zu < %zu", bytes, need);
    hog_mlp* m = new (std::nothrow) hog_mlp();
    if (!m) return fail(HOG_ENOMEM, "host allocation failed");
    m->nf = nf; m->batch_max = batch_max; m->np = mlp_nparam(nf); m->t = 0;
    m->nbmax = mlp_nb(batch_max);
    m->stream = static_cast<hipStream_t>(stream);
    size_t off[12];
    mlp_bytes(nf, batch_max, m->np, off);
    char* w = static_cast<char*>(ws);
    m->prm = reinterpret_cast<float*>(w + off[0]);
    m->m = reinterpret_cast<float*>(w + off[1]);
    m->v = reinterpret_cast<float*>(w + off[2]);
    m->grad = reinterpret_cast<float*>(w + off[3]);
    m->bt.XT = reinterpret_cast<uint16_t*>(w + off[4]);
    m->bt.H1T = reinterpret_cast<uint16_t*>(w + off[5]);
    m->bt.H2T = reinterpret_cast<uint16_t*>(w + off[6]);
    m->bt.D1T = reinterpret_cast<uint16_t*>(w + off[7]);
    m->bt.D2T = reinterpret_cast<uint16_t*>(w + off[8]);
    float* f = reinterpret_cast<float*>(w + off[9]);
    m->bt.dz = f;
    m->bt.loss = f + m->nbmax;
    m->bt.logit = f + 2 * (size_t)m->nbmax;
    m->lsum = f + 3 * (size_t)m->nbmax;
    m->partial = reinterpret_cast<float*>(w + off[10]);
    m->bt.nb = m->nbmax;
    HIP_TRY(hipMemsetAsync(ws, 0, need, m->stream));
    *out = m;
    return HOG_OK;
}

int hog_mlp_destroy(hog_mlp* m)
{
    delete m;
    return HOG_OK;
}

int hog_mlp_set_params(hog_mlp* m, const float* params)
{
    if (!m || !params) return fail(HOG_EINVAL, "NULL argument");
    HIP_TRY(hipMemcpyAsync(m->prm, params, sizeof(float) * m->np, hipMemcpyHostToDevice, m->stream));
    HIP_TRY(hipMemsetAsync(m->m, 0, sizeof(float) * m->np, m->stream));
    HIP_TRY(hipMemsetAsync(m->v, 0, sizeof(float) * m->np, m->stream));
    HIP_TRY(hipStreamSynchronize(m->stream));
    m->t = 0;
    return HOG_OK;
}

int hog_mlp_get_params(hog_mlp* m, float* params)
{
    if (!m || !params) return fail(HOG_EINVAL, "NULL argument");
    HIP_TRY(hipMemcpyAsync(params, m->prm, sizeof(float) * m->np, hipMemcpyDeviceToHost, m->stream));
    HIP_TRY(hipStreamSynchronize(m->stream));
    return HOG_OK;
}

static int mlp_backward(hog_mlp* m, const float* X, const float* y, const float* w, int n)
{
    if (n < 1 || n > m->batch_max || !X || !y) return fail(HOG_EINVAL, "batch must be 1..%d", m->batch_max);
    MlpBatch bt = m->bt;
    bt.nb = mlp_nb(n);
    const int nchunk = bt.nb / 256;
    if (m->nf == 65) {
        using S = MlpShape<65>;
        k_mlp_fwd_bwd<65><<<bt.nb / 64, 64, 0, m->stream>>>(X, y, w, n, m->prm, bt, nullptr);
        k_mlp_wgrad<65><<<dim3(S::NTILE, nchunk), 64, 0, m->stream>>>(bt, m->partial);
        k_mlp_reduce<65><<<(S::NTILE * 256 + 63) / 64 + 193, 64, 0, m->stream>>>(bt, m->partial, nchunk, m->grad);
    } else {
        using S = MlpShape<36>;
        k_mlp_fwd_bwd<36><<<bt.nb / 64, 64, 0, m->stream>>>(X, y, w, n, m->prm, bt, nullptr);
        k_mlp_wgrad<36><<<dim3(S::NTILE, nchunk), 64, 0, m->stream>>>(bt, m->partial);
        k_mlp_reduce<36><<<(S::NTILE * 256 + 63) / 64 + 193, 64, 0, m->stream>>>(bt, m->partial, nchunk, m->grad);
    }
    k_sum_fixed<<<1, 256, 0, m->stream>>>(bt.loss, n, m->lsum);
    return launch_check("mlp backward");
}

int hog_mlp_grads(hog_mlp* m, const float* X, const float* y, const float* w, int n, float* grads, float* loss)
{
    if (!m) return fail(HOG_EINVAL, "NULL handle");
    int rc = mlp_backward(m, X, y, w, n);
    if (rc) return rc;
    if (grads) HIP_TRY(hipMemcpyAsync(grads, m->grad, sizeof(float) * m->np, hipMemcpyDeviceToHost, m->stream));
    if (loss) HIP_TRY(hipMemcpyAsync(loss, m->lsum, sizeof(float), hipMemcpyDeviceToHost, m->stream));
    HIP_TRY(hipStreamSynchronize(m->stream));
    return HOG_OK;
}

int hog_mlp_step(hog_mlp* m, const float* X, const float* y, const float* w, int n, float lr, float* loss)
{
    if (!m) return fail(HOG_EINVAL, "NULL handle");
    if (!(lr > 0.0f)) return fail(HOG_EINVAL, "lr must be > 0");
    int rc = mlp_backward(m, X, y, w, n);
    if (rc) return rc;
    m->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)m->t), c2 = 1.0f - std::pow(b2, (float)m->t);
    k_mlp_adam<<<nblocks(m->np, 256), 256, 0, m->stream>>>(m->prm, m->m, m->v, m->grad, m->np, lr, b1, b2, 1e-8f,
                                                            c1, c2);
    rc = launch_check("adam");
    if (rc) return rc;
    if (loss) {
        HIP_TRY(hipMemcpyAsync(loss, m->lsum, sizeof(float), hipMemcpyDeviceToHost, m->stream));
        HIP_TRY(hipStreamSynchronize(m->stream));
    }
    return HOG_OK;
}

int hog_mlp_predict(hog_mlp* m, const float* X, int n, float* logits)
{
    if (!m || !X || !logits || n < 1) return fail(HOG_EINVAL, "bad arguments");
    for (int s0 = 0; s0 < n; s0 += m->batch_max) {
        const int b = (n - s0 < m->batch_max) ? n - s0 : m->batch_max;
        MlpBatch bt = m->bt;
        bt.nb = mlp_nb(b);
        if (m->nf == 65)
            k_mlp_fwd_bwd<65><<<bt.nb / 64, 64, 0, m->stream>>>(X + (size_t)s0 * 65, nullptr, nullptr, b, m->prm, bt,
                                                              logits + s0);
        else
            k_mlp_fwd_bwd<36><<<bt.nb / 64, 64, 0, m->stream>>>(X + (size_t)s0 * 36, nullptr, nullptr, b, m->prm, bt,
                                                              logits + s0);
    }
    return launch_check("mlp predict");
}

} // extern "C"

// ------------------------------------------------------------------------
// Slab streaming of a host-resident mesh.  The paper keeps each patch of a
// large mesh in host memory and moves it to the GPU every time step (Sec.
// II.2 and Sec. V, Tables I-II); here a mesh of any size along its last axis
// lives in two pinned host buffers (current and next state) and is stepped
// slab by slab through two patch grids on the device: while one slab is
// computed on the compute stream, the next one is copied in and the previous
// one copied out on the copy stream.  Each slab carries the three ghost
// layers of its neighbours (an HOG_EXTERNAL last axis), so the result equals
// the in-core step zone for zone.  One exchange per step is what the ADER
// step needs; Runge-Kutta stages would need one each, so they are rejected.
// ------------------------------------------------------------------------
namespace {

// fold one slab's step info into the accumulator: max signal speed, first bad
// zone (in mesh numbering), fallback count
__global__ void k_fold_info(const StepInfo* __restrict__ src, StepInfo* acc, long long zone_offset, int reset)
{
    if (reset) { acc->smax_bits = 0ull; acc->bad = ULLONG_MAX; acc->fallback = 0ull; }
    if (src->smax_bits > acc->smax_bits) acc->smax_bits = src->smax_bits;
    if (src->bad != ULLONG_MAX) {
        const unsigned long long b = src->bad + (unsigned long long)zone_offset;
        if (b < acc->bad) acc->bad = b;
    }
    acc->fallback += src->fallback;
}

} // namespace

struct hog_stream {
    hog_config mesh;
    int nd, nv, nlast, pn, npatch;
    long long plane, nmesh;        // zones per plane of the last axis; zones of the mesh
    double* host[2];               // pinned, caller-owned: current / next state, SoA [v][nlast][plane]
    int cur;
    hipStream_t cs, xs, xo;        // compute, copy in (caller's), copy out (own, default priority)
    hog_grid* g[3];                // slab grids: two of pn planes, one for a shorter last slab
    double* in[2];                 // device staging, [v][pn + 6][plane]
    double* out[2];                // device staging, [v][pn][plane]
    StepInfo* acc;                 // folded step info of the whole mesh
    hipEvent_t h2d[2], comp[2], done[2];
    double smax;                   // max signal speed of the current state (< 0: unknown)
    long long last_bad;
};

namespace {

struct StreamPlan {
    hog_config pcfg, tcfg;   // slab configs (full and last)
    int npatch, tail;        // planes of the last slab if shorter, else 0
    size_t off_g[3], bytes_g[3], off_in[2], off_out[2], off_acc, total;
};

int stream_plan(const hog_config* m, int pn, StreamPlan* S)
{
    int rc = check_cfg(m);
    if (rc) return rc;
    const int nd = m->ndim;
    const int nlast = (nd == 3) ? m->nz : m->ny;
    for (int d = 0; d < nd; ++d)
        if (m->bc[d] == HOG_EXTERNAL) return fail(HOG_EINVAL, "the mesh's own boundaries must be periodic or outflow");
    if (m->stepper != HOG_ADER) return fail(HOG_EINVAL, "streaming needs the one-exchange ADER step");
    if (m->debug) return fail(HOG_EINVAL, "no debug taps when streaming");
    if (pn < 1 || pn > nlast) return fail(HOG_EINVAL, "slab planes must be in [1, %d]", nlast);
    S->npatch = (nlast + pn - 1) / pn;
    S->tail = (nlast % pn) ? nlast % pn : 0;
    S->pcfg = *m;
    S->pcfg.bc[nd - 1] = HOG_EXTERNAL;
    if (nd == 3) S->pcfg.nz = pn; else S->pcfg.ny = pn;
    S->tcfg = S->pcfg;
    if (S->tail) { if (nd == 3) S->tcfg.nz = S->tail; else S->tcfg.ny = S->tail; }
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
    for (int k = 0; k < 3; ++k) {
        S->bytes_g[k] = 0;
        S->off_g[k] = 0;
        if (k == 2 && !S->tail) continue;
        rc = hog_workspace_size(k == 2 ? &S->tcfg : &S->pcfg, &S->bytes_g[k]);
        if (rc) return rc;
        S->off_g[k] = take(S->bytes_g[k]);
    }
    const long long plane = (long long)m->nx * (nd == 3 ? m->ny : 1);
    const int nv = nd + 2;
    for (int k = 0; k < 2; ++k) {
        S->off_in[k] = take(sizeof(double) * nv * (pn + 2 * kGhostZones) * plane);
        S->off_out[k] = take(sizeof(double) * nv * pn * plane);
    }
    S->off_acc = take(sizeof(StepInfo));
    S->total = o;
    return HOG_OK;
}

// mesh plane that supplies plane z of the padded last axis (ghosts by the mesh's boundary type)
int mesh_plane(int z, int n, int bc)
{
    if (z >= 0 && z < n) return z;
    if (bc == HOG_PERIODIC) return ((z % n) + n) % n;
    return z < 0 ? 0 : n - 1;
}

// enqueue the copy of slab p (planes [z0 - 3, z0 + np + 3) of the current host state) into in[slot],
// laid out [v][np + 6][plane] as the slab grid's extended box wants it
int stream_h2d(hog_stream* s, int p, int slot)
{
    const int z0 = p * s->pn, np = std::min(s->pn, s->nlast - z0), G = kGhostZones;
    const int bc = s->mesh.bc[s->nd - 1];
    const size_t pb = sizeof(double) * s->plane;
    int z = -G;
    while (z < np + G) {
        // longest run of consecutive mesh planes starting at z
        const int m0 = mesh_plane(z0 + z, s->nlast, bc);
        int len = 1;
        while (z + len < np + G && mesh_plane(z0 + z + len, s->nlast, bc) == m0 + len) ++len;
        for (int v = 0; v < s->nv; ++v)
            HIP_TRY(hipMemcpyAsync(s->in[slot] + ((long long)v * (np + 2 * G) + (z + G)) * s->plane,
                                   s->host[s->cur] + ((long long)v * s->nlast + m0) * s->plane, pb * len,
                                   hipMemcpyHostToDevice, s->xs));
        z += len;
    }
    return HOG_OK;
}

// staged slab -> the slab grid's padded state, ghost layers of the external axis included
int stream_pack(hog_stream* s, hog_grid* g, int slot)
{
    const Plan& L = g->P;
    const long long NE = box_size(L.E);
    const double* src = s->in[slot];
    if (L.nd == 3) k_pack<3><<<nblocks(NE, 256), 256, 0, s->cs>>>(src, g->U[g->cur], L.pad, L.E, 0);
    else k_pack<2><<<nblocks(NE, 256), 256, 0, s->cs>>>(src, g->U[g->cur], L.pad, L.E, 0);
    return launch_check("slab pack");
}

} // namespace

extern "C" {

int hog_stream_workspace_size(const hog_config* mesh, int slab_planes, size_t* bytes)
{
    if (!bytes) return fail(HOG_EINVAL, "bytes is NULL");
    StreamPlan S;
    int rc = stream_plan(mesh, slab_planes, &S);
    if (rc) return rc;
    *bytes = S.total;
    return HOG_OK;
}

int hog_stream_create(const hog_config* mesh, int slab_planes, void* workspace, size_t bytes, double* host_a,
                      double* host_b, void* compute_stream, void* copy_stream, hog_stream** out)
{
    g_err[0] = 0;
    if (!out || !host_a || !host_b || !workspace) return fail(HOG_EINVAL, "NULL argument");
    *out = nullptr;
    if (compute_stream == copy_stream) return fail(HOG_EINVAL, "the compute and copy streams must differ");
    if (host_a == host_b) return fail(HOG_EINVAL, "the two host state buffers must differ");
    StreamPlan S;
    int rc = stream_plan(mesh, slab_planes, &S);
    if (rc) return rc;
    if (bytes < S.total) return fail(HOG_ENOMEM, "workspace too small: %zu < %zu bytes", bytes, S.total);
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(HOG_EINVAL, "workspace must be 256-byte aligned");
    hog_stream* s = new (std::nothrow) hog_stream();
    if (!s) return fail(HOG_ENOMEM, "host allocation failed");
    char* ws = static_cast<char*>(workspace);
    s->mesh = *mesh;
    s->nd = mesh->ndim;
    s->nv = s->nd + 2;
    s->nlast = (s->nd == 3) ? mesh->nz : mesh->ny;
    s->pn = slab_planes;
    s->npatch = S.npatch;
    s->plane = (long long)mesh->nx * (s->nd == 3 ? mesh->ny : 1);
    s->nmesh = s->plane * s->nlast;
    s->host[0] = host_a;
    s->host[1] = host_b;
    s->cur = 0;
    s->cs = static_cast<hipStream_t>(compute_stream);
    s->xs = static_cast<hipStream_t>(copy_stream);
    s->smax = -1.0;
    s->last_bad = -1;
    for (int k = 0; k < 3; ++k) s->g[k] = nullptr;
    for (int k = 0; k < 2; ++k) s->h2d[k] = s->comp[k] = s->done[k] = nullptr;
    s->xo = nullptr;
    auto cleanup = [&](int code) {
        for (int k = 0; k < 3; ++k) hog_destroy(s->g[k]);
        if (s->xo) (void)hipStreamDestroy(s->xo);
        for (int k = 0; k < 2; ++k) {
            if (s->h2d[k]) (void)hipEventDestroy(s->h2d[k]);
            if (s->comp[k]) (void)hipEventDestroy(s->comp[k]);
            if (s->done[k]) (void)hipEventDestroy(s->done[k]);
        }
        delete s;
        return code;
    };
    for (int k = 0; k < 3; ++k) {
        if (!S.bytes_g[k]) continue;
        rc = hog_create(k == 2 ? &S.tcfg : &S.pcfg, ws + S.off_g[k], S.bytes_g[k], compute_stream, &s->g[k]);
        if (rc) return cleanup(rc);
    }
    if (hipStreamCreateWithFlags(&s->xo, hipStreamNonBlocking) != hipSuccess)
        return cleanup(fail(HOG_EDEVICE, "stream creation failed"));
    for (int k = 0; k < 2; ++k) {
        s->in[k] = reinterpret_cast<double*>(ws + S.off_in[k]);
        s->out[k] = reinterpret_cast<double*>(ws + S.off_out[k]);
        if (hipEventCreateWithFlags(&s->h2d[k], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&s->comp[k], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&s->done[k], hipEventDisableTiming) != hipSuccess)
            return cleanup(fail(HOG_EDEVICE, "event creation failed"));
        if (hipEventRecord(s->done[k], s->xs) != hipSuccess) return cleanup(fail(HOG_EDEVICE, "event record failed"));
    }
    s->acc = reinterpret_cast<StepInfo*>(ws + S.off_acc);
    *out = s;
    return HOG_OK;
}

int hog_stream_destroy(hog_stream* s)
{
    if (!s) return HOG_OK;
    (void)hipStreamSynchronize(s->cs);
    (void)hipStreamSynchronize(s->xs);
    (void)hipStreamSynchronize(s->xo);
    for (int k = 0; k < 3; ++k) hog_destroy(s->g[k]);
    for (int k = 0; k < 2; ++k) {
        (void)hipEventDestroy(s->h2d[k]);
        (void)hipEventDestroy(s->comp[k]);
        (void)hipEventDestroy(s->done[k]);
    }
    (void)hipStreamDestroy(s->xo);
    delete s;
    return HOG_OK;
}

int hog_stream_state(hog_stream* s, double** host_state)
{
    if (!s || !host_state) return fail(HOG_EINVAL, "NULL argument");
    *host_state = s->host[s->cur];
    return HOG_OK;
}

// One pass over the slabs: with step = 0 the CFL reduction of the current
// state, else one step of every slab with dt, new state into the other buffer.
// Software pipeline: the copy-in of slab p+1 is queued before slab p is
// computed, and the copy-out of slab p runs on its own stream, so both PCIe
// directions overlap the computation of the neighbouring slabs.
static int stream_pass(hog_stream* s, double dt, int step)
{
    auto copy_in = [&](int p) -> int {
        const int slot = p & 1;
        HIP_TRY(hipStreamWaitEvent(s->xs, s->done[slot], 0));   // slot free: slab p-2 copied out
        int rc = stream_h2d(s, p, slot);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(s->h2d[slot], s->xs));
        return HOG_OK;
    };
    int rc = copy_in(0);
    if (rc) return rc;
    for (int p = 0; p < s->npatch; ++p) {
        const int slot = p & 1;
        const int z0 = p * s->pn, np = std::min(s->pn, s->nlast - z0);
        hog_grid* g = (np == s->pn) ? s->g[slot] : s->g[2];
        if (p + 1 < s->npatch) {
            rc = copy_in(p + 1);
            if (rc) return rc;
        }
        HIP_TRY(hipStreamWaitEvent(s->cs, s->h2d[slot], 0));
        rc = stream_pack(s, g, slot);
        if (rc) return rc;
        const Plan& L = g->P;
        if (step) {
            rc = enqueue_step(g, dt);
            if (rc) return rc;
            g->cur ^= 1;
            const long long N = box_size(L.I);
            if (L.nd == 3) k_unpack<3><<<nblocks(N, 256), 256, 0, s->cs>>>(g->U[g->cur], s->out[slot], L.pad, L.I, 0);
            else k_unpack<2><<<nblocks(N, 256), 256, 0, s->cs>>>(g->U[g->cur], s->out[slot], L.pad, L.I, 0);
        } else {
            rc = enqueue_cfl(g, g->cur);
            if (rc) return rc;
        }
        k_fold_info<<<1, 1, 0, s->cs>>>(g->info, s->acc, (long long)z0 * s->plane, p == 0 ? 1 : 0);
        rc = launch_check("slab step");
        if (rc) return rc;
        HIP_TRY(hipEventRecord(s->comp[slot], s->cs));
        HIP_TRY(hipStreamWaitEvent(s->xo, s->comp[slot], 0));
        if (step) {
            const size_t bytes = sizeof(double) * (size_t)np * s->plane;
            for (int v = 0; v < s->nv; ++v)
                HIP_TRY(hipMemcpyAsync(s->host[s->cur ^ 1] + ((long long)v * s->nlast + z0) * s->plane,
                                       s->out[slot] + (long long)v * np * s->plane, bytes, hipMemcpyDeviceToHost, s->xo));
        }
        HIP_TRY(hipEventRecord(s->done[slot], s->xo));
    }
    HIP_TRY(hipStreamSynchronize(s->cs));
    HIP_TRY(hipStreamSynchronize(s->xs));
    HIP_TRY(hipStreamSynchronize(s->xo));
    return HOG_OK;
}

int hog_stream_compute_dt(hog_stream* s, double* dt)
{
    if (!s || !dt) return fail(HOG_EINVAL, "NULL argument");
    int rc = stream_pass(s, 0.0, 0);
    if (rc) return rc;
    StepInfo si;
    HIP_TRY(hipMemcpy(&si, s->acc, sizeof si, hipMemcpyDeviceToHost));
    if (si.bad != ULLONG_MAX) {
        s->last_bad = (long long)si.bad;
        return fail(HOG_ENONPHYS, "non-physical state in zone %lld", s->last_bad);
    }
    s->smax = smax_of(si);
    *dt = s->mesh.cfl / s->smax;
    return HOG_OK;
}

int hog_stream_step(hog_stream* s, double dt, double* dt_next)
{
    if (!s) return fail(HOG_EINVAL, "NULL handle");
    if (!(dt > 0.0) || !std::isfinite(dt)) {
        if (dt != 0.0) return fail(HOG_EINVAL, "dt must be finite and > 0, or 0 for the CFL dt (got %g)", dt);
        if (!(s->smax > 0.0)) {
            double d;
            int rc = hog_stream_compute_dt(s, &d);
            if (rc) return rc;
        }
        dt = s->mesh.cfl / s->smax;
    }
    int rc = stream_pass(s, dt, 1);
    if (rc) return rc;
    StepInfo si;
    HIP_TRY(hipMemcpy(&si, s->acc, sizeof si, hipMemcpyDeviceToHost));
    if (si.bad != ULLONG_MAX) {
        s->last_bad = (long long)si.bad;
        return fail(HOG_ENONPHYS, "step produced a non-physical state in zone %lld", s->last_bad);
    }
    s->cur ^= 1;
    s->smax = smax_of(si);
    if (dt_next) *dt_next = s->mesh.cfl / s->smax;
    return HOG_OK;
}

} // extern "C"

// ------------------------------------------------------------------------
// One step with no device allocation: the workspace is a file-scope device
// array of a fixed size instead of a caller's buffer.  Each GPU the library
// runs on holds its own copy of the array from the module load to the end of
// the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the array's name is a host-side
// stand-in, not a device address).
// ------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices];   // device address of scratch per device (null: not looked up yet)
int g_scratch_cus[kMaxDevices];

// Device address of the scratch array on the current device, looked up (and
// the device checked) on the first call on that device.
int scratch_on_current_device(char** ptr, int* cus)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(HOG_EDEVICE, "device index %d is out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int c = 0;
        int rc = device_check(&c);
        if (rc) return rc;
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || reinterpret_cast<uintptr_t>(p) % kAlign)
            return fail(HOG_EDEVICE, "scratch array of device %d is not 256-byte aligned", dev);
        g_scratch_ptr[dev] = static_cast<char*>(p);
        g_scratch_cus[dev] = c;
    }
    *ptr = g_scratch_ptr[dev];
    *cus = g_scratch_cus[dev];
    return HOG_OK;
}

} // namespace

extern "C" {

size_t hog_step_static_capacity(void) { return kScratchBytes; }

int hog_step_static(const hog_config* cfg, const double* U_in, double* U_out, double dt, double* dt_next,
                    void* hip_stream)
{
    g_err[0] = 0;
    int rc = check_cfg(cfg);
    if (rc) return rc;
    if (!U_in || !U_out) return fail(HOG_EINVAL, "NULL state pointer");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(HOG_EINVAL, "dt must be finite and > 0 (got %g)", dt);
    for (int d = 0; d < 3; ++d)
        if (cfg->bc[d] == HOG_EXTERNAL)
            return fail(HOG_EINVAL, "an external boundary needs hog_set_state_ext on a handle");
    if (cfg->debug) return fail(HOG_EINVAL, "debug taps need a handle (hog_create)");
    Plan P;
    plan(cfg, &P);
    if (P.total > kScratchBytes)
        return fail(HOG_ENOMEM, "this grid needs %zu workspace bytes; hog_step_static holds at most %zu "
                                "(use hog_create with a caller workspace)", P.total, kScratchBytes);
    char* ws = nullptr;
    int cus = 0;
    rc = scratch_on_current_device(&ws, &cus);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hog_grid g{};
    bind_grid(&g, cfg, P, ws, kScratchBytes, s, cus);
    // the array keeps the previous call's contents: reset the step scalars
    k_reset<<<1, 1, 0, s>>>(g.info, 0.0, 1);
    const long long N = box_size(P.I);
    if (P.nd == 3) k_pack<3><<<nblocks(N, 256), 256, 0, s>>>(U_in, g.U[0], P.pad, P.I, 0);
    else k_pack<2><<<nblocks(N, 256), 256, 0, s>>>(U_in, g.U[0], P.pad, P.I, 0);
    rc = launch_check("pack");
    if (rc) return rc;
    rc = enqueue_step(&g, dt);
    if (rc) return rc;
    if (dt_next) {
        StepInfo si;
        rc = read_info(&g, &si);
        if (rc) return rc;
        if (si.bad != ULLONG_MAX)
            return fail(HOG_ENONPHYS, "step produced a non-physical state in zone %lld", (long long)si.bad);
        *dt_next = cfg->cfl / smax_of(si);
    }
    if (P.nd == 3) k_unpack<3><<<nblocks(N, 256), 256, 0, s>>>(g.U[1], U_out, P.pad, P.I, 0);
    else k_unpack<2><<<nblocks(N, 256), 256, 0, s>>>(g.U[1], U_out, P.pad, P.I, 0);
    return launch_check("unpack");
}

} // extern "C"

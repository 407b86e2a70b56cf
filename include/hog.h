/*
 * hog.h -- C ABI of the MI355X (gfx950) ADER-WENO zone update for the 2D/3D
 * compressible Euler equations of an ideal gas.
 *
 * One call of hog_step() performs the three-stage update the paper builds its
 * GPU codes on (arXiv 2211.13295, Sec. I.1 and Sec. II.2, Figs. 1-7):
 *   WENO reconstruction of the conserved variables in every zone,
 *   an ADER predictor that extends each zone polynomial in time,
 *   a Riemann-solver (HLLC/HLL/Rusanov) corrector with a conservative
 *   flux-difference update, and the CFL time step of the new state.
 * With order = 2 the step is instead the paper's own second-order scheme
 * (Sec. II.2, Figs. 3-7): slopes of the conserved variables from a
 * monotonised-central limiter with compression factor 2 for the density and
 * 1.5 for the other variables (Fig. 3), a pointwise predictor of the time
 * mode (Fig. 4; its body is not printed and is read as the Hancock step:
 * minus dt/dx_d times the flux difference between the zone's face-centre
 * values U +- S_d/2, summed over the axes), one Riemann problem per face at
 * the face centre and half time step with the states U +- S_d/2 + U5/2
 * (Fig. 5), and the flux-difference update (Figs. 6-7).  It runs as one fused
 * kernel per step on the FP64 path.
 * The state lives in device memory between calls: the paper's per-step host
 * round trip of the zone means (its "U_skinny" transfer, Sec. II.2, Fig. 1)
 * only happens when the caller asks for it with hog_get_state().
 *
 * Conventions
 *  - Every call returns an int status: HOG_OK (0) or a negative HOG_E* code;
 *    hog_last_error() gives a message (thread-local, static storage).
 *    Nothing is printed and nothing aborts.
 *  - State layout HOG_SOA: double U[nv][nz][ny][nx] (x fastest), nv = ndim+2,
 *    variables rho, rho*u, rho*v, [rho*w], E; in 2D nz = 1.  HOG_AOS:
 *    double U[nz][ny][nx][nv] (the paper's zone-mean array order).
 *  - Device memory: the caller allocates one workspace of
 *    hog_workspace_size() bytes (e.g. a torch uint8 tensor) and keeps it alive
 *    as long as the handle; the library allocates no device memory itself
 *    (hog_step_static instead uses a fixed array that every GPU the library
 *    runs on holds from the library's load).
 *  - Stream: all work is enqueued on the hipStream_t given at hog_create();
 *    calls return without synchronising unless stated.  One handle must not
 *    be used from two threads at once.
 */
#ifndef HOG_H
#define HOG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HOG_ABI_VERSION 1

enum {
    HOG_OK = 0,
    HOG_EINVAL = -1,     /* bad argument or configuration */
    HOG_ENOMEM = -2,     /* workspace too small */
    HOG_EDEVICE = -3,    /* HIP runtime error or unsupported device */
    HOG_ENONPHYS = -4,   /* rho <= 0, p <= 0 or non-finite value in a zone */
    HOG_ESTATE = -5      /* call out of order (e.g. step before set_state) */
};

/* Per-axis boundary.  HOG_EXTERNAL (any active axis, ADER stepping only):
 * the caller supplies the three ghost layers below and above the interior
 * along that axis with hog_set_state_ext -- from the neighbouring slabs of a
 * larger mesh (see hog_stream_*, which makes the last axis external), or, for
 * one block of a mesh split over devices, from the neighbouring blocks
 * (every axis external: the one exchange per step of Sec. I.1). */
enum { HOG_PERIODIC = 0, HOG_OUTFLOW = 1, HOG_EXTERNAL = 2 };
/* Riemann solver.  HOG_HLLEM and HOG_HLLI: the HLL flux with the dissipation
 * of the entropy and shear waves of Roe's linearisation reduced by Einfeldt's
 * factor c/(c+|u_n|) (HLLEM) or by Dumbser and Balsara's factor
 * 1 - min(u_n,0)/S_L - max(u_n,0)/S_R (HLLI); all Roe-averaged. */
enum { HOG_HLLC = 0, HOG_HLL = 1, HOG_RUSANOV = 2, HOG_HLLEM = 3, HOG_HLLI = 4 };
/* Arithmetic of the path.  HOG_FP64: everything in FP64.  HOG_MIXED: the
 * reconstruction coefficients, predictor, face states and Riemann solver in
 * FP32; the stencil differences, smoothness indicators, epsilon division and
 * nonlinear weights, the face-flux Gauss sum, the conservative update and the
 * CFL reduction in FP64.  The state is FP64 on both paths. */
enum { HOG_FP64 = 0, HOG_MIXED = 1 };
/* Time stepping (hog_config.stepper).  The Runge-Kutta schemes are the
 * strong-stability-preserving ones in Shu-Osher form: SSP-RK(2,2) and
 * SSP-RK(3,3) of Shu and Osher, SSP-RK(5,4) of Spiteri and Ruuth. */
enum { HOG_ADER = 0, HOG_SSPRK2 = 2, HOG_SSPRK3 = 3, HOG_SSPRK54 = 4 };
enum { HOG_SOA = 0, HOG_AOS = 1 };                     /* state layouts */
enum { HOG_HOST = 0, HOG_DEVICE = 1 };                 /* where a user buffer lives */

/* Debug taps (hog_debug_tap): intermediates of the last hog_step(). */
enum {
    HOG_TAP_MODES = 1,   /* spatial modes after reconstruction: double [N][ns][nv]
                            (at order 2: mean and limited undivided slopes, debug = 1) */
    HOG_TAP_STMODES = 2, /* space-time modes after the predictor: double [N][nst][nv]
                            (needs debug = 1 in the config; at order 2 the last
                            mode is the time mode U5 = dt dU/dt of Fig. 4) */
    HOG_TAP_FLUX_X = 3,  /* face fluxes: double [nv][nz][ny][nx+1] (x faces)      */
    HOG_TAP_FLUX_Y = 4,  /*              double [nv][nz][ny+1][nx]                */
    HOG_TAP_FLUX_Z = 5   /*              double [nv][nz+1][ny][nx]                */
};
/* N = nx*ny*nz interior zones in x-fastest order; modes are listed in the
 * canonical order: space-time modes (a,b,c,e) with a+b+c+e <= p, e outermost,
 * then c, then b, then a innermost (c = 0 in 2D); the spatial modes are the
 * e = 0 block.  Mode (a,b,c,e) multiplies P_a(xi) P_b(eta) P_c(zeta) tau^e,
 * P_k the monic Legendre polynomials on the zone [-1/2,1/2] and tau in [0,1]
 * the fraction of the time step. */

typedef struct hog_config {
    int ndim;            /* 2 or 3 */
    int nx, ny, nz;      /* interior zones per axis (nz = 1 in 2D), each >= 1 */
    int order;           /* 2, 3 or 4 (polynomial degree p = order - 1); 2 is the
                            scheme of Figs. 3-7 and needs precision HOG_FP64 */
    int riemann;         /* HOG_HLLC | HOG_HLL | HOG_RUSANOV | HOG_HLLEM | HOG_HLLI */
    int bc[3];           /* per axis HOG_PERIODIC | HOG_OUTFLOW | HOG_EXTERNAL (last axis) */
    int precision;       /* HOG_FP64 | HOG_MIXED */
    int linear_weno;     /* 1: WENO nonlinear weights replaced by the linear ones */
    int debug;           /* 1: keep the space-time modes for HOG_TAP_STMODES */
    int positivity;      /* 1: a zone whose predictor meets rho <= 0, p <= 0 or a
                            non-finite state at any quadrature node or face point
                            falls back to its zone mean (first order) for that step;
                            at order 2 the points checked are the face-centre values
                            U +- S_d/2 and the face states U +- S_d/2 + U5/2 */
    int stepper;         /* HOG_ADER (0): the one-step ADER predictor-corrector (at order 2
                            the Hancock step of Fig. 4); HOG_SSPRK2 / HOG_SSPRK3 /
                            HOG_SSPRK54: Runge-Kutta with 2, 3 or 5 stages (Table IV), each
                            stage the same reconstruction and Riemann solver with
                            face points in space only; FP64, no debug taps, no gate */
    int characteristic;  /* 1: every 1D WENO application on the characteristic fields of
                            the flux Jacobian along its axis at the mean of its centre
                            zone instead of on the conserved variables (orders 3 and 4,
                            FP64; the alternative to Sec. I.1's component-wise choice) */
    int reserved;        /* must be 0 */
    double gamma;        /* ratio of specific heats, > 1 */
    double dx, dy, dz;   /* zone widths (dz ignored in 2D), > 0 */
    double cfl;          /* CFL number of hog_compute_dt / dt_next, in (0, 1] */
    double weno_eps;     /* epsilon of the nonlinear weights; <= 0 selects 1e-12 */
    double g3[3];        /* O3 linear weights L, C, R; all 0 selects (0.075, 0.85, 0.075) */
    double g4[4];        /* O4 linear weights H, L, C, R; all 0 selects
                            (0.85, 0.01125, 0.1275, 0.01125) */
} hog_config;

typedef struct hog_grid hog_grid;

/* ABI version of the loaded library (HOG_ABI_VERSION). */
int hog_abi_version(void);

/* Device bytes the caller must provide to hog_create() for this config.
 * Errors: HOG_EINVAL for an invalid config or NULL pointer. */
int hog_workspace_size(const hog_config* cfg, size_t* bytes);

/* Bind a config, a device workspace (>= hog_workspace_size bytes, 256-byte
 * aligned) and a HIP stream (NULL = default stream) to a new handle.  The
 * handle borrows the workspace and the stream; both must outlive it.  The
 * current HIP device must be a gfx950 GPU.
 * Errors: HOG_EINVAL, HOG_ENOMEM (workspace too small), HOG_EDEVICE. */
int hog_create(const hog_config* cfg, void* workspace, size_t bytes, void* hip_stream,
               hog_grid** out);

/* Release the handle (not the workspace or stream).  NULL is allowed. */
int hog_destroy(hog_grid* g);

/* Copy the interior state in (layout HOG_SOA | HOG_AOS, buffer on HOG_HOST |
 * HOG_DEVICE, nv*nx*ny*nz doubles): the `update device(U_skinny)` and
 * U_Skinny_to_U of Fig. 1 (Sec. II.2), done once instead of every step.
 * Stream-ordered; host buffers are copied before return.  Also evaluates the
 * CFL reduction of the new state.
 * Errors: HOG_EINVAL, HOG_EDEVICE. */
int hog_set_state(hog_grid* g, const double* U, int layout, int where);

/* Copy the current interior state out (same layouts): the `update
 * host(U_skinny)` of Fig. 1 (Sec. II.2), only when the caller asks for it.
 * For a host buffer the call synchronises the stream.  Errors: HOG_EINVAL, HOG_ESTATE, HOG_EDEVICE. */
int hog_get_state(hog_grid* g, double* U, int layout, int where);

/* Like hog_set_state (SoA only) for a grid with HOG_EXTERNAL axes: U holds
 * the interior grown by the three ghost layers below and above along every
 * external axis, [nv][mz][my][mx] with m = n + 6 on an external axis and m = n
 * otherwise (index 0 is the lowest ghost layer; edges and corners between
 * external axes included).  The supplied ghost zones are used as given by the
 * next step; the remaining ghosts are filled from their axes' boundary types
 * (from the supplied values where they meet an external axis).
 * Errors: HOG_EINVAL (NULL, or no axis external), HOG_EDEVICE. */
int hog_set_state_ext(hog_grid* g, const double* U, int where);

/* CFL time step of the current state, dt = cfl / max_zones sum_d
 * (|u_d| + c) / dx_d (Fig. 7 of Sec. II.2: Eval_Tstep_Ptwise per zone with a
 * min reduction into dt_next; its body is not printed, the sum form is used).
 * Synchronises.  Errors: HOG_ENONPHYS (see hog_last_bad_zone), HOG_ESTATE. */
int hog_compute_dt(hog_grid* g, double* dt);

/* One ADER-WENO step with time step dt > 0.  If dt_next is not NULL the call
 * synchronises, checks the new state and returns its CFL time step; on a
 * non-physical new state it returns HOG_ENONPHYS and keeps the pre-step
 * state as the current one.  If dt_next is NULL nothing is checked and the
 * call does not synchronise.
 * Errors: HOG_EINVAL (dt <= 0 or not finite), HOG_ESTATE, HOG_ENONPHYS. */
int hog_step(hog_grid* g, double dt, double* dt_next);

/* The time loop of Fig. 1 (Sec. II.2: DO i_timestep, dt = dt_next) run on the
 * device: advance with the CFL time step computed on the device from each
 * state (no host round trip per step).  t_end <= 0: exactly nsteps steps.  t_end > 0:
 * steps until the accumulated time reaches t_end, clipping the last step
 * (this mode synchronises once per step); nsteps is then an upper bound.
 * *t_out (may be NULL) receives the time advanced.  Synchronises at the end
 * and checks the final state.  If a step produces a non-physical state the
 * later steps of the run write nothing, and the call returns HOG_ENONPHYS
 * with the state before that step as the current one (as hog_step does) and
 * the first non-physical zone of that step in hog_last_bad_zone().
 * Errors: HOG_EINVAL, HOG_ESTATE, HOG_ENONPHYS. */
int hog_advance(hog_grid* g, int nsteps, double t_end, double* t_out);

/* Copy an intermediate of the last step to host memory dst (HOG_TAP_*): the
 * spatial modes the reconstruction (Limiter of Figs. 1 and 3) leaves in
 * U(:,:,:,:,1:4), the space-time modes of the predictor (Figs. 1 and 4) and
 * the face fluxes of Make_Flux_X/Y/Z (Fig. 5), for tests.
 * Synchronises.  Errors: HOG_EINVAL (unknown tap, bytes too small, tap not
 * kept), HOG_ESTATE (no step yet). */
int hog_debug_tap(hog_grid* g, int tap, void* dst, size_t bytes);

/* Stage timing with HIP events recorded on the handle's stream around every
 * stage of every subsequent step: 0 ghost fill, 1 reconstruction sweeps,
 * 2 ADER predictor, 3 Riemann solver, 4 update + CFL, 5 learned-gate
 * inference (only with a gate set) (HOG_NSTAGES).  At order 2 the fused
 * kernel is recorded as stage 2; with Runge-Kutta stepping stage 2 holds the
 * face-point evaluation (or the fused kernel at order 2) and stage 4 the
 * stage combination, summed over the stages of a step.  Used to
 * split step time the way the paper splits out the predictor (Sec. III.1,
 * Table III).  enable = 0 stops recording.  Errors: HOG_EINVAL, HOG_EDEVICE. */
#define HOG_NSTAGES 6
int hog_profile_enable(hog_grid* g, int enable);

/* Total milliseconds and launch count per stage since the last enable/read
 * (arrays of nstages >= HOG_NSTAGES entries); synchronises and resets the
 * counters.  Errors: HOG_EINVAL, HOG_EDEVICE. */
int hog_profile_read(hog_grid* g, double* ms, int* launches, int nstages);

/* Device-side counters of the last step (synchronises): *t time advanced
 * since the last hog_advance/hog_set_state, *dt the last time step,
 * *fallback_zones the predictor zones (interior grown by one zone per axis)
 * that used the positivity fallback in the last step (summed over the stages
 * of a Runge-Kutta step).  Pointers may be NULL.
 * Errors: HOG_EINVAL, HOG_EDEVICE. */
int hog_stats(hog_grid* g, double* t, double* dt, long long* fallback_zones);

/* ---------------------------------------------------------------------
 * Slab streaming of a host-resident mesh (Sec. II.1 and Sec. V: each patch of
 * a mesh larger than the GPU's memory is moved to the GPU every step).  The
 * mesh, of any size along its last axis, lives in two pinned host buffers;
 * every step moves it through the GPU in slabs of at most slab_planes planes
 * of the last axis, each with the three ghost layers of its neighbours, on two
 * slab grids: the copies of one slab (in on the copy stream, out after its
 * step) overlap the step of the other.  The result equals the in-core
 * hog_step zone for zone (the fallback count differs: it counts each slab's
 * grown box).  ADER stepping only: a Runge-Kutta stage would need an
 * exchange of its own.
 * --------------------------------------------------------------------- */
typedef struct hog_stream hog_stream;

/* Device bytes for a mesh (its own last-axis boundary periodic or outflow,
 * stepper HOG_ADER, debug 0) streamed in slabs of slab_planes planes
 * (1 <= slab_planes <= the last axis).  Errors: HOG_EINVAL. */
int hog_stream_workspace_size(const hog_config* mesh, int slab_planes, size_t* bytes);

/* Bind a device workspace (256-byte aligned, hog_stream_workspace_size bytes,
 * borrowed), two host buffers of nv*nx*ny*nz doubles each (SoA [v][nz][ny][nx];
 * pinned host memory, e.g. hipHostMalloc or a pinned torch tensor; borrowed;
 * host_a holds the initial state, host_b receives the next one and the two
 * alternate; they must not overlap) and two different HIP streams (compute and copy).
 * Errors: HOG_EINVAL, HOG_ENOMEM (workspace too small), HOG_EDEVICE. */
int hog_stream_create(const hog_config* mesh, int slab_planes, void* workspace, size_t bytes, double* host_a,
                      double* host_b, void* compute_stream, void* copy_stream, hog_stream** out);
int hog_stream_destroy(hog_stream* s);

/* CFL dt of the current state (one pass of the slabs); synchronises.
 * Errors: HOG_ENONPHYS, HOG_EDEVICE. */
int hog_stream_compute_dt(hog_stream* s, double* dt);

/* One step of the whole mesh with dt (dt = 0: the CFL dt of the current
 * state, from the previous step or one extra pass); the new state goes to the
 * other host buffer, which becomes current.  Synchronises; dt_next (may be
 * NULL) receives the CFL dt of the new state.  On HOG_ENONPHYS the current
 * state is kept.  Errors: HOG_EINVAL, HOG_ENONPHYS, HOG_EDEVICE. */
int hog_stream_step(hog_stream* s, double dt, double* dt_next);

/* The host buffer that holds the current state. */
int hog_stream_state(hog_stream* s, double** host_state);

/* ---------------------------------------------------------------------
 * Learned smooth-zone gate (not in the paper; a cheaper reconstruction in
 * zones a small network predicts to be smooth).  Network: features x ->
 * h1 = relu(W1 x + b1) (64) -> h2 = relu(W2 h1 + b2) (64) -> logit =
 * w3 . h2 + b3, with W1, W2, w3 and every layer input rounded to BF16, FP32
 * biases and accumulation.  Features of a zone, per variable: the cross of
 * the zone and its two neighbours on each side along each axis (13 zones in
 * 3D, 9 in 2D) minus the zone value, divided by (max - min + 1e-12 max(1,
 * |zone value|)) over the cross; order [variable][centre, x-2, x-1, x+1,
 * x+2, y-2, ..., z+2]: nf = 65 (3D) or 36 (2D).  Parameter vector (FP32):
 * W1[64][nf], b1[64], W2[64][64], b2[64], w3[64], b3 (row-major).
 * --------------------------------------------------------------------- */

/* Number of FP32 parameters of the gate for ndim (8449 in 3D, 6593 in 2D). */
int hog_gate_param_count(int ndim, int* count);

/* Enable the gate with the given FP32 parameters (copied, rounded to BF16 on
 * the host) and probability threshold theta in (0,1): in every later step,
 * the 1D WENO applications centred at an interior zone whose output
 * probability is >= theta use the linear weights (no smoothness indicators);
 * applications centred outside the interior keep the nonlinear weights.
 * params = NULL disables the gate.  Synchronises.  Errors: HOG_EINVAL (also
 * for a non-NULL params at order 2, which has no WENO weights). */
int hog_set_gate(hog_grid* g, const float* params, double theta);

/* Evaluate the gate on the current state: host arrays of nx*ny*nz logits
 * and/or flags (either may be NULL).  Synchronises.
 * Errors: HOG_ESTATE (no network, fixed flags set, or no state), HOG_EDEVICE. */
int hog_gate_eval(hog_grid* g, float* logits, unsigned char* flags);

/* Use fixed per-zone flags (host array of nx*ny*nz bytes, x fastest, each
 * 0 or 1; copied) in every later step instead of the network's, with the
 * same effect (flag 1: the 1D applications centred at that zone use the
 * linear weights).  For ablations of the gate: all zones linear, or a
 * random selection of the network's smooth fraction.  flags = NULL returns
 * to the network loaded by hog_set_gate, or to no gate; hog_set_gate also
 * clears fixed flags.  Synchronises.  Errors: HOG_EINVAL (a flag not 0/1, or
 * non-NULL flags at order 2). */
int hog_set_gate_flags(hog_grid* g, const unsigned char* flags);

/* Training samples from the current state (FP64 path only): for the n
 * interior zone indices in zones (device array, x fastest) write the features
 * feature-major to features (device, nf*n floats, [feature][sample]) and, to
 * maxdev (device, n floats), the largest |omega_k/gamma_k - 1| of the
 * nonlinear WENO weights over the variables and the 1D applications centred
 * at the zone (a zone is labelled smooth when it is <= 0.25).  An index
 * outside [0, nx*ny*nz) reads nothing and yields NaN features and a NaN
 * maxdev for that sample.  Stream-ordered, no synchronisation.  Errors: HOG_EINVAL (also at order 2), HOG_ESTATE. */
int hog_harvest(hog_grid* g, const long long* zones, long long n, float* features, float* maxdev);

/* Training of the gate network on the GPU (FP32 masters, Adam, BF16-rounded
 * operands in the forward pass as in inference; gradients summed over the
 * batch in a fixed order).  The caller owns a device workspace of
 * hog_mlp_workspace_size() bytes and the batch arrays: X (device, n*nf
 * floats, sample-major), y (device, n labels 0/1), w (device, n per-sample
 * loss weights, or NULL for 1).  Loss: weighted binary cross entropy, mean
 * over the batch. */
typedef struct hog_mlp hog_mlp;
int hog_mlp_workspace_size(int nf, int batch_max, size_t* bytes);
int hog_mlp_create(int nf, int batch_max, void* workspace, size_t bytes, void* hip_stream, hog_mlp** out);
int hog_mlp_destroy(hog_mlp* m);
/* Copy the FP32 parameter vector in (resets the Adam moments) / out. */
int hog_mlp_set_params(hog_mlp* m, const float* params);
int hog_mlp_get_params(hog_mlp* m, float* params);
/* Loss and gradient (host outputs, either may be NULL), no update; synchronises. */
int hog_mlp_grads(hog_mlp* m, const float* X, const float* y, const float* w, int n, float* grads, float* loss);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with learning rate lr; *loss
 * (host, may be NULL: then no synchronisation) receives the pre-step loss. */
int hog_mlp_step(hog_mlp* m, const float* X, const float* y, const float* w, int n, float lr, float* loss);
/* Logits of n samples (device output). */
int hog_mlp_predict(hog_mlp* m, const float* X, int n, float* logits);

/* ---------------------------------------------------------------------
 * One step without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels as hog_step, with the workspace in a
 * fixed-size device array inside the library instead of a caller's buffer.
 * U_in and U_out are device arrays of the interior state, SoA
 * [nv][nz][ny][nx] doubles, owned by the caller; they may be the same array
 * (U_in is copied in before anything is written).  The step is enqueued on
 * hip_stream (NULL = default stream).  If dt_next is not NULL the call
 * synchronises, checks the new state and returns its CFL time step; on a
 * non-physical new state it returns HOG_ENONPHYS and leaves U_out untouched.
 * If dt_next is NULL nothing is checked and the call does not synchronise.
 * The config may not use HOG_EXTERNAL boundaries or debug taps; no gate.
 * Limit: hog_workspace_size(cfg) must not exceed hog_step_static_capacity()
 * bytes (256 MiB: up to 40^3 zones at fourth order in 3D FP64, 520^2 at
 * third order in 2D); larger grids get HOG_ENOMEM and need hog_create.
 * Each GPU holds one copy of the array from the library's load to the end of
 * the process, shared by every call on that GPU: calls that overlap on one
 * GPU (two streams or threads at once) race and must be serialised by the
 * caller.  No host or device memory is allocated by the call.
 * Errors: HOG_EINVAL, HOG_ENOMEM (grid too large), HOG_ENONPHYS, HOG_EDEVICE.
 * --------------------------------------------------------------------- */
size_t hog_step_static_capacity(void);
int hog_step_static(const hog_config* cfg, const double* U_in, double* U_out, double dt, double* dt_next,
                    void* hip_stream);

/* Zone index (x fastest) of the first non-physical zone found by the last
 * check, or -1. */
long long hog_last_bad_zone(hog_grid* g);

/* Message of the last error on this thread ("" if none). */
const char* hog_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HOG_H */

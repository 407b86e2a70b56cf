"""FP64 CPU oracle of the ADER-WENO Euler zone update (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2211_13295_amd``); the only common dependency is the seeded input
generator package ``icgen``.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc into
``liboracle.so``); this module only marshals arguments.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RIEMANN = {"hllc": 0, "hll": 1, "rusanov": 2, "hllem": 3, "hlli": 4}
STEPPER = {"ader": 0, "rk2": 2, "rk3": 3, "rk4": 4}
BC = {"periodic": 0, "outflow": 1}


def build(force=True):
    """Compile liboracle.so with gcc (OpenMP over zones, FP64, -O3)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class OCfg(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("order", C.c_int), ("riemann", C.c_int), ("bc", C.c_int * 3),
        ("linear_weno", C.c_int), ("positivity", C.c_int),
        ("gamma", C.c_double), ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
        ("cfl", C.c_double), ("weno_eps", C.c_double),
        ("g3", C.c_double * 3), ("g4", C.c_double * 4),
        ("stepper", C.c_int), ("char_recon", C.c_int),
    ]


# Linear weights and epsilon of the WENO readings (stated in the design notes).
DEFAULT_G3 = (0.075, 0.85, 0.075)
DEFAULT_G4 = (0.85, 0.01125, 0.1275, 0.01125)   # H, L, C, R
DEFAULT_EPS = 1e-12

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        cp = C.POINTER(OCfg)
        L.oracle_step.argtypes = [cp, dp, C.c_double, dp]
        L.oracle_step.restype = C.c_int
        L.oracle_step_count.argtypes = [cp, dp, C.c_double, dp, C.POINTER(C.c_longlong)]
        L.oracle_step_count.restype = C.c_int
        up = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
        L.oracle_step_gated.argtypes = [cp, dp, C.c_double, up, dp, C.POINTER(C.c_longlong)]
        L.oracle_step_gated.restype = C.c_int
        L.oracle_zone_maxdev.argtypes = [cp, dp, dp]
        L.oracle_zone_maxdev.restype = C.c_int
        L.oracle_step_zones.argtypes = [cp, dp, C.c_double, C.c_int, ip, dp]
        L.oracle_step_zones.restype = C.c_int
        L.oracle_cfl_dt.argtypes = [cp, dp, C.POINTER(C.c_longlong)]
        L.oracle_cfl_dt.restype = C.c_double
        L.oracle_run.argtypes = [cp, dp, C.c_int, C.c_double, C.POINTER(C.c_double), C.c_void_p]
        L.oracle_run.restype = C.c_int
        L.oracle_stage_modes.argtypes = [cp, dp, C.c_double, C.c_void_p, C.c_void_p]
        L.oracle_stage_modes.restype = C.c_int
        L.oracle_weno1d.argtypes = [cp, C.c_int, dp, dp]
        L.oracle_recon_block.argtypes = [cp, dp, dp]
        L.oracle_predict.argtypes = [cp, dp, dp, dp]
        L.oracle_predict.restype = C.c_int
        L.oracle_eval_q.argtypes = [cp, dp, C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.oracle_riemann.argtypes = [cp, C.c_int, dp, dp, dp]
        L.oracle_phys_flux.argtypes = [cp, C.c_int, dp, dp]
        L.oracle_modes.argtypes = [C.c_int, C.c_int, C.c_void_p]
        L.oracle_modes.restype = C.c_int
        for f in ("oracle_leg", "oracle_sleg"):
            getattr(L, f).argtypes = [C.c_int, C.c_double]
            getattr(L, f).restype = C.c_double
        for f in ("oracle_dleg", "oracle_tint"):
            getattr(L, f).argtypes = [C.c_int, C.c_int]
            getattr(L, f).restype = C.c_double
        L.oracle_gauss.argtypes = [C.c_int, dp, dp]
        L.oracle_rk_table.argtypes = [C.c_int, C.c_void_p, C.c_void_p]
        L.oracle_rk_table.restype = C.c_int
        L.oracle_rk_operator.argtypes = [cp, dp, C.c_double, dp]
        L.oracle_rk_operator.restype = C.c_int
        L.oracle_char_eigen.argtypes = [cp, C.c_int, dp, dp, dp]
        L.oracle_mc.argtypes = [C.c_double, C.c_double, C.c_double]
        L.oracle_mc.restype = C.c_double
        _lib = L
    return _lib


def make_cfg(ndim, n, order, h, gamma=1.4, cfl=0.4, riemann="hllc", bc=("periodic",) * 3,
             linear_weno=False, eps=DEFAULT_EPS, g3=DEFAULT_G3, g4=DEFAULT_G4, positivity=True, stepper="ader",
             characteristic=False):
    c = OCfg()
    c.ndim = ndim
    c.nx, c.ny, c.nz = int(n[0]), int(n[1]), int(n[2]) if ndim == 3 else 1
    c.order = order
    c.riemann = RIEMANN[riemann] if isinstance(riemann, str) else int(riemann)
    for d in range(3):
        b = bc[d]
        c.bc[d] = BC[b] if isinstance(b, str) else int(b)
    c.linear_weno = int(bool(linear_weno))
    c.positivity = int(bool(positivity))
    c.gamma = gamma
    c.dx, c.dy, c.dz = h
    c.cfl = cfl
    c.weno_eps = eps
    for i in range(3):
        c.g3[i] = g3[i]
    for i in range(4):
        c.g4[i] = g4[i]
    c.stepper = STEPPER[stepper] if isinstance(stepper, str) else int(stepper)
    c.char_recon = int(bool(characteristic))
    return c


def cfg_from_problem(pb, order, cfl=0.4, riemann="hllc", **kw):
    return make_cfg(pb.ndim, pb.n, order, pb.h, gamma=pb.gamma, cfl=cfl, riemann=riemann,
                    bc=pb.bc, **kw)


def nmodes(ndim, p):
    return lib().oracle_modes(ndim, p, None)


def modes(ndim, p):
    n = nmodes(ndim, p)
    buf = (C.c_int * (4 * n))()
    lib().oracle_modes(ndim, p, buf)
    return np.array(list(buf), dtype=np.int64).reshape(n, 4)


def _state(U):
    return np.ascontiguousarray(U, dtype=np.float64)


def cfl_dt(cfg, U):
    bad = C.c_longlong(-1)
    dt = lib().oracle_cfl_dt(C.byref(cfg), _state(U), C.byref(bad))
    return dt, bad.value


def step(cfg, U, dt):
    U = _state(U)
    out = np.empty_like(U)
    rc = lib().oracle_step(C.byref(cfg), U, float(dt), out)
    if rc != 0:
        raise MemoryError("oracle_step failed")
    return out


def step_count(cfg, U, dt):
    """One step; returns (U_new, number of predictor zones that used the fallback)."""
    U = _state(U)
    out = np.empty_like(U)
    n = C.c_longlong(0)
    rc = lib().oracle_step_count(C.byref(cfg), U, float(dt), out, C.byref(n))
    if rc != 0:
        raise MemoryError("oracle_step failed")
    return out, n.value


def step_gated(cfg, U, dt, gate):
    """One step where the 1D WENO applications centred at zones with gate = 1
    use the linear weights; gate has the interior shape (uint8)."""
    U = _state(U)
    g = np.ascontiguousarray(gate, dtype=np.uint8)
    assert g.size == U[0].size
    out = np.empty_like(U)
    n = C.c_longlong(0)
    rc = lib().oracle_step_gated(C.byref(cfg), U, float(dt), g.reshape(-1), out, C.byref(n))
    if rc != 0:
        raise MemoryError("oracle_step_gated failed")
    return out, n.value


def zone_maxdev(cfg, U):
    """max_k |omega_k/gamma_k - 1| per interior zone (applications centred there)."""
    U = _state(U)
    out = np.empty(U[0].shape, dtype=np.float64)
    rc = lib().oracle_zone_maxdev(C.byref(cfg), U, out.reshape(-1))
    if rc != 0:
        raise MemoryError("oracle_zone_maxdev failed")
    return out


def step_zones(cfg, U, dt, ijk):
    U = _state(U)
    ijk = np.ascontiguousarray(np.asarray(ijk, dtype=np.int32).reshape(-1, 3))
    nv = cfg.ndim + 2
    out = np.empty((ijk.shape[0], nv), dtype=np.float64)
    rc = lib().oracle_step_zones(C.byref(cfg), U, float(dt), ijk.shape[0], ijk, out)
    if rc != 0:
        raise MemoryError("oracle_step_zones failed")
    return out


def run(cfg, U, nsteps=0, t_end=0.0):
    """Advance a copy of U; returns (U_final, t_final, dts)."""
    U = _state(U).copy()
    maxsteps = nsteps if t_end <= 0 else 1000000
    dts = np.zeros(max(maxsteps, 1) if t_end <= 0 else 100000, dtype=np.float64)
    t = C.c_double(0.0)
    s = lib().oracle_run(C.byref(cfg), U, int(nsteps), float(t_end), C.byref(t),
                         dts.ctypes.data_as(C.c_void_p))
    if s < 0:
        raise FloatingPointError("oracle_run: non-physical state")
    return U, t.value, dts[:s].copy()


def stage_modes(cfg, U, dt, want_q=True):
    """Spatial modes W [N, ms, nv] and space-time modes q [N, nst, nv] per interior zone."""
    U = _state(U)
    nd, p = cfg.ndim, cfg.order - 1
    nst = nmodes(nd, p)
    mod = modes(nd, p)
    ms = int((mod[:, 3] == 0).sum())
    nv = nd + 2
    N = cfg.nx * cfg.ny * (cfg.nz if nd == 3 else 1)
    W = np.empty((N, ms, nv))
    q = np.empty((N, nst, nv)) if want_q else None
    rc = lib().oracle_stage_modes(C.byref(cfg), U, float(dt), W.ctypes.data_as(C.c_void_p),
                                  q.ctypes.data_as(C.c_void_p) if want_q else None)
    if rc != 0:
        raise MemoryError("oracle_stage_modes failed")
    return W, q


def weno1d(cfg, p, v5):
    out = np.zeros(4)
    lib().oracle_weno1d(C.byref(cfg), p, _state(v5), out)
    return out


def recon_block(cfg, blk):
    nd, p = cfg.ndim, cfg.order - 1
    mod = modes(nd, p)
    ms = int((mod[:, 3] == 0).sum())
    W = np.zeros((ms, nd + 2))
    lib().oracle_recon_block(C.byref(cfg), _state(blk), W)
    return W


def predict(cfg, lam, W):
    nd, p = cfg.ndim, cfg.order - 1
    nst = nmodes(nd, p)
    q = np.zeros((nst, nd + 2))
    lib().oracle_predict(C.byref(cfg), _state(np.asarray(lam, dtype=np.float64).reshape(3)),
                         _state(W), q)
    return q


def eval_q(cfg, q, xi, eta, zeta, tau):
    out = np.zeros(cfg.ndim + 2)
    lib().oracle_eval_q(C.byref(cfg), _state(q), xi, eta, zeta, tau, out)
    return out


def riemann(cfg, d, UL, UR):
    out = np.zeros(cfg.ndim + 2)
    lib().oracle_riemann(C.byref(cfg), d, _state(UL), _state(UR), out)
    return out


def phys_flux(cfg, d, U):
    out = np.zeros(cfg.ndim + 2)
    lib().oracle_phys_flux(C.byref(cfg), d, _state(U), out)
    return out


def rk_table(stepper):
    """Shu-Osher coefficients of a Runge-Kutta stepper: list of (i, k, alpha, beta)."""
    st = STEPPER[stepper] if isinstance(stepper, str) else int(stepper)
    n = lib().oracle_rk_table(st, None, None)
    ik = (C.c_int * (2 * n))()
    ab = (C.c_double * (2 * n))()
    lib().oracle_rk_table(st, ik, ab)
    return [(ik[2 * s], ik[2 * s + 1], ab[2 * s], ab[2 * s + 1]) for s in range(n)]


def rk_operator(cfg, U, dt):
    """dt L(U) of the method-of-lines operator (interior SoA)."""
    U = _state(U)
    out = np.empty_like(U)
    if lib().oracle_rk_operator(C.byref(cfg), U, float(dt), out) != 0:
        raise MemoryError("oracle_rk_operator failed")
    return out


def mc(a, b, cfac):
    """Limited undivided slope of the second-order scheme (Fig. 3)."""
    return lib().oracle_mc(float(a), float(b), float(cfac))


def gauss(n):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().oracle_gauss(n, x, w)
    return x, w


def leg(a, x):
    return lib().oracle_leg(a, x)


def sleg(e, t):
    return lib().oracle_sleg(e, t)


def dleg(a, ap):
    return lib().oracle_dleg(a, ap)


def tint(e, ep):
    return lib().oracle_tint(e, ep)


def char_eigen(cfg, d, U):
    """Right eigenvectors (columns of R) of the flux Jacobian along axis d at
    the conserved state U, and L = R^-1, as used by the characteristic
    reconstruction."""
    nv = cfg.ndim + 2
    R = np.zeros((nv, nv))
    L = np.zeros((nv, nv))
    lib().oracle_char_eigen(C.byref(cfg), d, _state(U), R, L)
    return R, L

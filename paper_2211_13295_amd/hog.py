"""Thin ctypes binding of the C ABI in include/hog.h (argument marshalling only).

Every step of the update runs in the gfx950 kernels of ``libhog.so``; this
module only fills the config struct, allocates the caller-side workspace with
PyTorch (device memory) and passes pointers and the current HIP stream.  If
the library is missing or cannot be loaded it raises: there is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhog.so")

HOG_OK, HOG_EINVAL, HOG_ENOMEM, HOG_EDEVICE, HOG_ENONPHYS, HOG_ESTATE = 0, -1, -2, -3, -4, -5
SOA, AOS = 0, 1
HOST, DEVICE = 0, 1
TAP_MODES, TAP_STMODES, TAP_FLUX_X, TAP_FLUX_Y, TAP_FLUX_Z = 1, 2, 3, 4, 5
RIEMANN = {"hllc": 0, "hll": 1, "rusanov": 2, "hllem": 3, "hlli": 4}
BC = {"periodic": 0, "outflow": 1, "external": 2}
PRECISION = {"fp64": 0, "mixed": 1}
STEPPER = {"ader": 0, "rk2": 2, "rk3": 3, "rk4": 4}
_ERRNAMES = {HOG_EINVAL: "EINVAL", HOG_ENOMEM: "ENOMEM", HOG_EDEVICE: "EDEVICE",
             HOG_ENONPHYS: "ENONPHYS", HOG_ESTATE: "ESTATE"}


class HogError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hog error {_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class HogConfig(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("order", C.c_int), ("riemann", C.c_int), ("bc", C.c_int * 3),
        ("precision", C.c_int), ("linear_weno", C.c_int), ("debug", C.c_int),
        ("positivity", C.c_int), ("stepper", C.c_int), ("characteristic", C.c_int), ("reserved", C.c_int),
        ("gamma", C.c_double), ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
        ("cfl", C.c_double), ("weno_eps", C.c_double), ("g3", C.c_double * 3), ("g4", C.c_double * 4),
    ]


_lib = None


def load():
    """Load libhog.so (built by paper_2211_13295_amd/build.py); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with `python paper_2211_13295_amd/build.py`")
    # torch first: it carries its own HIP runtime under the same soname, and
    # the library must bind to that one so that both share one runtime (and
    # torch's device memory and streams)
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, cp = C.c_void_p, C.POINTER(HogConfig)
    L.hog_abi_version.restype = C.c_int
    L.hog_last_error.restype = C.c_char_p
    L.hog_workspace_size.argtypes = [cp, C.POINTER(C.c_size_t)]
    L.hog_create.argtypes = [cp, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.hog_destroy.argtypes = [vp]
    L.hog_set_state.argtypes = [vp, vp, C.c_int, C.c_int]
    L.hog_get_state.argtypes = [vp, vp, C.c_int, C.c_int]
    L.hog_set_state_ext.argtypes = [vp, vp, C.c_int]
    L.hog_stream_workspace_size.argtypes = [cp, C.c_int, C.POINTER(C.c_size_t)]
    L.hog_stream_create.argtypes = [cp, C.c_int, vp, C.c_size_t, vp, vp, vp, vp, C.POINTER(vp)]
    L.hog_stream_destroy.argtypes = [vp]
    L.hog_stream_compute_dt.argtypes = [vp, C.POINTER(C.c_double)]
    L.hog_stream_step.argtypes = [vp, C.c_double, C.POINTER(C.c_double)]
    L.hog_stream_state.argtypes = [vp, C.POINTER(vp)]
    L.hog_compute_dt.argtypes = [vp, C.POINTER(C.c_double)]
    L.hog_step.argtypes = [vp, C.c_double, vp]
    L.hog_advance.argtypes = [vp, C.c_int, C.c_double, C.POINTER(C.c_double)]
    L.hog_debug_tap.argtypes = [vp, C.c_int, vp, C.c_size_t]
    L.hog_profile_enable.argtypes = [vp, C.c_int]
    L.hog_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_int]
    L.hog_stats.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_longlong)]
    fp, ip_ = C.POINTER(C.c_float), C.POINTER(C.c_int)
    L.hog_gate_param_count.argtypes = [C.c_int, ip_]
    L.hog_set_gate.argtypes = [vp, vp, C.c_double]
    L.hog_gate_eval.argtypes = [vp, vp, vp]
    L.hog_set_gate_flags.argtypes = [vp, vp]
    L.hog_harvest.argtypes = [vp, vp, C.c_longlong, vp, vp]
    L.hog_mlp_workspace_size.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_size_t)]
    L.hog_mlp_create.argtypes = [C.c_int, C.c_int, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.hog_mlp_destroy.argtypes = [vp]
    L.hog_mlp_set_params.argtypes = [vp, vp]
    L.hog_mlp_get_params.argtypes = [vp, vp]
    L.hog_mlp_grads.argtypes = [vp, vp, vp, vp, C.c_int, vp, vp]
    L.hog_mlp_step.argtypes = [vp, vp, vp, vp, C.c_int, C.c_float, vp]
    L.hog_mlp_predict.argtypes = [vp, vp, C.c_int, vp]
    for f in ("hog_gate_param_count", "hog_set_gate", "hog_gate_eval", "hog_set_gate_flags", "hog_harvest",
              "hog_mlp_workspace_size",
              "hog_mlp_create", "hog_mlp_destroy", "hog_mlp_set_params", "hog_mlp_get_params", "hog_mlp_grads",
              "hog_mlp_step", "hog_mlp_predict"):
        getattr(L, f).restype = C.c_int
    L.hog_step_static.argtypes = [cp, vp, vp, C.c_double, C.POINTER(C.c_double), vp]
    L.hog_step_static.restype = C.c_int
    L.hog_step_static_capacity.restype = C.c_size_t
    L.hog_last_bad_zone.argtypes = [vp]
    L.hog_last_bad_zone.restype = C.c_longlong
    for f in ("hog_set_state_ext", "hog_stream_workspace_size", "hog_stream_create", "hog_stream_destroy",
              "hog_stream_compute_dt", "hog_stream_step", "hog_stream_state"):
        getattr(L, f).restype = C.c_int
    for f in ("hog_workspace_size", "hog_create", "hog_destroy", "hog_set_state", "hog_get_state",
              "hog_compute_dt", "hog_step", "hog_advance", "hog_debug_tap", "hog_profile_enable",
              "hog_profile_read", "hog_stats"):
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


def _check(rc):
    if rc != HOG_OK:
        raise HogError(rc, load().hog_last_error().decode())


def make_config(ndim, n, order, h, gamma=1.4, cfl=0.4, riemann="hllc", bc=("periodic",) * 3,
                linear_weno=False, debug=False, weno_eps=0.0, g3=(0, 0, 0), g4=(0, 0, 0, 0),
                positivity=True, precision="fp64", stepper="ader", characteristic=False):
    c = HogConfig()
    c.ndim = ndim
    c.nx, c.ny = int(n[0]), int(n[1])
    c.nz = int(n[2]) if ndim == 3 else 1
    c.order = order
    c.riemann = RIEMANN[riemann] if isinstance(riemann, str) else int(riemann)
    for d in range(3):
        c.bc[d] = BC[bc[d]] if isinstance(bc[d], str) else int(bc[d])
    c.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    c.linear_weno = int(bool(linear_weno))
    c.debug = int(bool(debug))
    c.positivity = int(bool(positivity))
    c.stepper = STEPPER[stepper] if isinstance(stepper, str) else int(stepper)
    c.characteristic = int(bool(characteristic))
    c.gamma = gamma
    c.dx, c.dy = h[0], h[1]
    c.dz = h[2] if ndim == 3 else 1.0
    c.cfl = cfl
    c.weno_eps = weno_eps
    for i in range(3):
        c.g3[i] = g3[i]
    for i in range(4):
        c.g4[i] = g4[i]
    return c


def workspace_size(cfg):
    n = C.c_size_t(0)
    _check(load().hog_workspace_size(C.byref(cfg), C.byref(n)))
    return n.value


def step_static_capacity():
    """Workspace bytes the no-allocation step holds (hog_step_static_capacity)."""
    return int(load().hog_step_static_capacity())


def step_static(cfg, U_in, U_out, dt, want_next=True):
    """hog_step_static: one step of the interior state U_in (a CUDA float64
    tensor, SoA [nv][nz][ny][nx], contiguous) into U_out (same shape; may be
    U_in) on torch's current stream, with the library's own fixed device
    scratch array as workspace (no allocation).  Returns dt_next, or None
    when want_next is False (then nothing is checked or synchronised)."""
    import torch
    for t in (U_in, U_out):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("U_in and U_out must be contiguous float64 CUDA tensors")
    nv = cfg.ndim + 2
    n = nv * cfg.nx * cfg.ny * (cfg.nz if cfg.ndim == 3 else 1)
    if U_in.numel() != n or U_out.numel() != n:
        raise ValueError(f"state tensors must hold {n} doubles")
    nxt = C.c_double(0.0)
    stream = torch.cuda.current_stream().cuda_stream
    _check(load().hog_step_static(C.byref(cfg), C.c_void_p(U_in.data_ptr()), C.c_void_p(U_out.data_ptr()),
                                  float(dt), C.byref(nxt) if want_next else None, C.c_void_p(stream)))
    return nxt.value if want_next else None


class Grid:
    """One ADER-WENO grid on the current GPU and the current torch stream."""

    def __init__(self, ndim, n, order, h, **kw):
        import torch
        self._torch = torch
        self.cfg = make_config(ndim, n, order, h, **kw)
        self.ndim, self.order = ndim, order
        self.nv = ndim + 2
        self.n = (self.cfg.nx, self.cfg.ny, self.cfg.nz)
        self.shape = (self.nv, self.n[2], self.n[1], self.n[0]) if ndim == 3 else (self.nv, self.n[1], self.n[0])
        self.nzones = self.n[0] * self.n[1] * self.n[2]
        L = load()
        nbytes = workspace_size(self.cfg)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream()
        h_ = C.c_void_p()
        _check(L.hog_create(C.byref(self.cfg), C.c_void_p(aligned), nbytes,
                            C.c_void_p(self.stream.cuda_stream), C.byref(h_)))
        self._h = h_

    @classmethod
    def from_problem(cls, pb, order, **kw):
        kw.setdefault("gamma", pb.gamma)
        kw.setdefault("bc", pb.bc)
        g = cls(pb.ndim, pb.n, order, pb.h, **kw)
        g.set_state(pb.U)
        return g

    def close(self):
        """Destroy the handle and drop the workspace (its device memory goes back
        to torch's allocator once nothing else references it)."""
        if getattr(self, "_h", None) is not None and self._h.value:
            load().hog_destroy(self._h)
            self._h = C.c_void_p()
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, U, layout=SOA):
        torch = self._torch
        if isinstance(U, torch.Tensor) and U.is_cuda:
            t = U.contiguous().to(torch.float64)
            assert t.numel() == self.nv * self.nzones
            _check(load().hog_set_state(self._h, C.c_void_p(t.data_ptr()), layout, DEVICE))
            torch.cuda.current_stream().synchronize()
            return
        a = np.ascontiguousarray(U, dtype=np.float64)
        assert a.size == self.nv * self.nzones
        _check(load().hog_set_state(self._h, a.ctypes.data_as(C.c_void_p), layout, HOST))

    def ext_shape(self):
        """Shape of the array hog_set_state_ext takes: SoA, each external axis
        grown by the three ghost layers on both sides."""
        bc = (self.cfg.bc[0], self.cfg.bc[1], self.cfg.bc[2])
        n = [self.cfg.nx, self.cfg.ny, self.cfg.nz][: self.ndim]
        m = [n[d] + 6 if bc[d] == BC["external"] else n[d] for d in range(self.ndim)]
        return (self.nv,) + tuple(reversed(m))

    def set_state_ext(self, U):
        """Interior plus the three ghost layers below and above along every
        external axis: SoA [v][mz][my][mx] (host array or CUDA tensor)."""
        torch = self._torch
        want = self.ext_shape()
        if tuple(U.shape) != want:
            raise ValueError(f"set_state_ext needs shape {want}, got {tuple(U.shape)}")
        if isinstance(U, torch.Tensor) and U.is_cuda:
            t = U.contiguous().to(torch.float64)
            _check(load().hog_set_state_ext(self._h, C.c_void_p(t.data_ptr()), DEVICE))
            torch.cuda.current_stream().synchronize()
            return
        a = np.ascontiguousarray(U, dtype=np.float64)
        _check(load().hog_set_state_ext(self._h, a.ctypes.data_as(C.c_void_p), HOST))

    def get_state(self, layout=SOA):
        shape = self.shape if layout == SOA else self.shape[1:] + (self.nv,)
        out = np.empty(shape, dtype=np.float64)
        _check(load().hog_get_state(self._h, out.ctypes.data_as(C.c_void_p), layout, HOST))
        return out

    def get_state_device(self, out, layout=SOA):
        _check(load().hog_get_state(self._h, C.c_void_p(out.data_ptr()), layout, DEVICE))
        return out

    def compute_dt(self):
        dt = C.c_double(0.0)
        _check(load().hog_compute_dt(self._h, C.byref(dt)))
        return dt.value

    def step(self, dt, want_next=True):
        nxt = C.c_double(0.0)
        _check(load().hog_step(self._h, float(dt), C.byref(nxt) if want_next else None))
        return nxt.value if want_next else None

    def advance(self, nsteps, t_end=0.0):
        t = C.c_double(0.0)
        _check(load().hog_advance(self._h, int(nsteps), float(t_end), C.byref(t)))
        return t.value

    def tap(self, which):
        nd, nv, p = self.ndim, self.nv, self.order - 1
        from math import comb
        if which == TAP_MODES:
            shape = (self.nzones, comb(p + nd, nd), nv)
        elif which == TAP_STMODES:
            shape = (self.nzones, comb(p + nd + 1, nd + 1), nv)
        else:
            d = which - TAP_FLUX_X
            n = list(self.n)
            n[d] += 1
            shape = (nv, n[2], n[1], n[0])
        out = np.empty(shape, dtype=np.float64)
        _check(load().hog_debug_tap(self._h, which, out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    STAGES = ("ghost", "reconstruction", "predictor", "riemann", "update", "gate")

    def profile(self, enable=True):
        _check(load().hog_profile_enable(self._h, int(bool(enable))))

    def profile_read(self):
        n = len(self.STAGES)
        ms = (C.c_double * n)()
        cnt = (C.c_int * n)()
        _check(load().hog_profile_read(self._h, ms, cnt, n))
        return {s: (ms[i], cnt[i]) for i, s in enumerate(self.STAGES)}

    def stats(self):
        t, dt, nb = C.c_double(0), C.c_double(0), C.c_longlong(0)
        _check(load().hog_stats(self._h, C.byref(t), C.byref(dt), C.byref(nb)))
        return {"t": t.value, "dt": dt.value, "fallback_zones": nb.value}

    # ---- learned gate
    def set_gate(self, params, theta=0.5):
        """params: FP32 vector (pack_params) or None to disable."""
        if params is None:
            _check(load().hog_set_gate(self._h, None, 0.5))
            return
        v = np.ascontiguousarray(params, dtype=np.float32)
        assert v.size == param_count(self.ndim)
        _check(load().hog_set_gate(self._h, v.ctypes.data_as(C.c_void_p), float(theta)))

    def set_gate_flags(self, flags):
        """Fixed per-zone flags (array of the state's zone shape, 0/1) used by
        later steps instead of the network; None returns to the network."""
        if flags is None:
            _check(load().hog_set_gate_flags(self._h, None))
            return
        f = np.ascontiguousarray(flags, dtype=np.uint8).reshape(-1)
        assert f.size == self.nzones
        _check(load().hog_set_gate_flags(self._h, f.ctypes.data_as(C.c_void_p)))

    def gate_eval(self):
        n = self.nzones
        logits = np.empty(n, np.float32)
        flags = np.empty(n, np.uint8)
        _check(load().hog_gate_eval(self._h, logits.ctypes.data_as(C.c_void_p), flags.ctypes.data_as(C.c_void_p)))
        return logits.reshape(self.shape[1:]), flags.reshape(self.shape[1:])

    def harvest(self, zones):
        """Features (n, nf) and max weight deviation (n,) of interior zones (flat indices)."""
        torch = self._torch
        zn = np.asarray(zones, dtype=np.int64)
        if zn.size and (zn.min() < 0 or zn.max() >= self.nzones):
            raise ValueError(f"zone indices must lie in [0, {self.nzones})")
        z = torch.as_tensor(zn, device="cuda")
        n = z.numel()
        nf = (self.ndim + 2) * (4 * self.ndim + 1)
        feat = torch.empty(nf * max(n, 1), dtype=torch.float32, device="cuda")
        dev = torch.empty(max(n, 1), dtype=torch.float32, device="cuda")
        _check(load().hog_harvest(self._h, C.c_void_p(z.data_ptr()), n, C.c_void_p(feat.data_ptr()),
                                  C.c_void_p(dev.data_ptr())))
        torch.cuda.current_stream().synchronize()
        return feat[: nf * n].view(nf, n).t().contiguous(), dev[:n]

    def last_bad_zone(self):
        return load().hog_last_bad_zone(self._h)


class Stream:
    """A host-resident mesh stepped through the GPU in slabs of the last axis
    (hog_stream_*): two pinned host state buffers, one device workspace, the
    current torch stream for compute and a second stream for the copies."""

    def __init__(self, ndim, n, order, h, slab_planes, **kw):
        import torch
        self._torch = torch
        self.cfg = make_config(ndim, n, order, h, **kw)
        self.ndim, self.nv = ndim, ndim + 2
        self.n = (self.cfg.nx, self.cfg.ny, self.cfg.nz)
        self.shape = (self.nv, self.n[2], self.n[1], self.n[0]) if ndim == 3 else (self.nv, self.n[1], self.n[0])
        L = load()
        nb = C.c_size_t(0)
        _check(L.hog_stream_workspace_size(C.byref(self.cfg), int(slab_planes), C.byref(nb)))
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        self.host = [torch.empty(self.shape, dtype=torch.float64, pin_memory=True) for _ in range(2)]
        self.compute = torch.cuda.current_stream()
        self.copy = torch.cuda.Stream()
        h_ = C.c_void_p()
        _check(L.hog_stream_create(C.byref(self.cfg), int(slab_planes), C.c_void_p(aligned), nb.value,
                                   C.c_void_p(self.host[0].data_ptr()), C.c_void_p(self.host[1].data_ptr()),
                                   C.c_void_p(self.compute.cuda_stream), C.c_void_p(self.copy.cuda_stream),
                                   C.byref(h_)))
        self._h = h_

    @classmethod
    def from_problem(cls, pb, order, slab_planes, **kw):
        kw.setdefault("gamma", pb.gamma)
        kw.setdefault("bc", pb.bc)
        s = cls(pb.ndim, pb.n, order, pb.h, slab_planes, **kw)
        s.host[0].copy_(s._torch.from_numpy(np.ascontiguousarray(pb.U)))
        return s

    def _current(self):
        p = C.c_void_p()
        _check(load().hog_stream_state(self._h, C.byref(p)))
        return self.host[0] if p.value == self.host[0].data_ptr() else self.host[1]

    def get_state(self):
        return self._current().numpy().copy()

    def compute_dt(self):
        dt = C.c_double(0.0)
        _check(load().hog_stream_compute_dt(self._h, C.byref(dt)))
        return dt.value

    def step(self, dt=0.0):
        nxt = C.c_double(0.0)
        _check(load().hog_stream_step(self._h, float(dt), C.byref(nxt)))
        return nxt.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().hog_stream_destroy(self._h)
            self._h = C.c_void_p()
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def param_count(ndim):
    n = C.c_int(0)
    _check(load().hog_gate_param_count(ndim, C.byref(n)))
    return n.value


def pack_params(W1, b1, W2, b2, w3, b3):
    """FP32 parameter vector of the gate network in the C ABI's order."""
    return np.concatenate([np.asarray(a, np.float32).reshape(-1) for a in (W1, b1, W2, b2, w3, b3)])


def unpack_params(v, nf, hidden=64):
    v = np.asarray(v, np.float32)
    o = 0
    out = {}
    for k, shp in (("W1", (hidden, nf)), ("b1", (hidden,)), ("W2", (hidden, hidden)), ("b2", (hidden,)),
                   ("w3", (hidden,)), ("b3", (1,))):
        size = int(np.prod(shp))
        out[k] = v[o:o + size].reshape(shp).copy()
        o += size
    return out


class Mlp:
    """Training handle of the gate network (GPU kernels; torch only allocates)."""

    def __init__(self, nf, batch_max=4096):
        import torch
        self._torch = torch
        self.nf, self.batch_max = nf, batch_max
        L = load()
        nb = C.c_size_t(0)
        _check(L.hog_mlp_workspace_size(nf, batch_max, C.byref(nb)))
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
        base = (self.workspace.data_ptr() + 255) // 256 * 256
        h = C.c_void_p()
        _check(L.hog_mlp_create(nf, batch_max, C.c_void_p(base), nb.value,
                                C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(h)))
        self._h = h
        self.np = 64 * nf + 64 + 64 * 64 + 64 + 64 + 1

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().hog_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, vec):
        v = np.ascontiguousarray(vec, dtype=np.float32)
        assert v.size == self.np
        _check(load().hog_mlp_set_params(self._h, v.ctypes.data_as(C.c_void_p)))

    def get_params(self):
        v = np.empty(self.np, np.float32)
        _check(load().hog_mlp_get_params(self._h, v.ctypes.data_as(C.c_void_p)))
        return v

    def _dev(self, a, dtype):
        torch = self._torch
        if isinstance(a, torch.Tensor):
            return a.to(device="cuda", dtype=dtype).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")

    def grads(self, X, y, w=None):
        X, y = self._dev(X, self._torch.float32), self._dev(y, self._torch.float32)
        w = None if w is None else self._dev(w, self._torch.float32)
        g = np.empty(self.np, np.float32)
        loss = np.zeros(1, np.float32)
        _check(load().hog_mlp_grads(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(y.data_ptr()),
                                    None if w is None else C.c_void_p(w.data_ptr()), int(y.numel()),
                                    g.ctypes.data_as(C.c_void_p), loss.ctypes.data_as(C.c_void_p)))
        return float(loss[0]), g

    def step(self, X, y, w=None, lr=1e-3, want_loss=True):
        loss = np.zeros(1, np.float32)
        _check(load().hog_mlp_step(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(y.data_ptr()),
                                   None if w is None else C.c_void_p(w.data_ptr()), int(y.numel()), float(lr),
                                   loss.ctypes.data_as(C.c_void_p) if want_loss else None))
        return float(loss[0]) if want_loss else None

    def predict(self, X):
        torch = self._torch
        X = self._dev(X, torch.float32)
        n = X.numel() // self.nf
        out = torch.empty(n, dtype=torch.float32, device="cuda")
        _check(load().hog_mlp_predict(self._h, C.c_void_p(X.data_ptr()), n, C.c_void_p(out.data_ptr())))
        torch.cuda.current_stream().synchronize()
        return out

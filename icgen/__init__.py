"""Seeded synthetic initial conditions for the compressible Euler workloads.

This module only builds input states (zone averages of the conserved variables)
and the exact solutions that some of them have.  It holds none of the
reconstruction / predictor / Riemann arithmetic of the method, so both the CPU
oracle's tests and the GPU path's tests and benchmark may use it.

Layout of every returned state: float64 array of shape ``(nv, nz, ny, nx)`` in
3D or ``(nv, ny, nx)`` in 2D (structure of arrays, x fastest), conserved
variables ``rho, rho*u, rho*v, [rho*w], E`` for an ideal gas.

The test problems follow the accuracy study of the paper (Sec. IV.1, Table XII:
the isentropic vortex of Balsara and Shu) and the workload shapes of the
throughput tables (Sec. III.1, Tables I-III: 3D single-patch runs).  Smooth
data are averaged over each zone with a 4-point tensor Gauss rule per axis;
discontinuous data are sampled at zone centres (interfaces of the Riemann and
quadrant problems fall on zone faces).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "prim_to_cons", "vortex2d", "vortex3d_perturbed", "multiblast",
    "four_quadrant", "sod", "entropy_wave", "uniform", "vortex_exact_density",
]

_GX, _GW = np.polynomial.legendre.leggauss(4)
_GX = _GX / 2.0          # nodes on [-1/2, 1/2]
_GW = _GW / 2.0          # weights summing to 1


@dataclass
class Problem:
    """An initial state plus the grid it lives on."""
    U: np.ndarray                      # (nv, [nz,] ny, nx) float64 zone averages
    ndim: int
    n: tuple                           # (nx, ny, nz) ; nz = 1 in 2D
    h: tuple                           # (dx, dy, dz)
    origin: tuple                      # (x0, y0, z0)
    bc: tuple                          # per axis: "periodic" | "outflow"
    gamma: float = 1.4
    meta: dict = field(default_factory=dict)


def prim_to_cons(rho, vel, p, gamma):
    """Conserved variables from density, velocity components and pressure."""
    vel = [np.asarray(v, dtype=np.float64) for v in vel]
    kin = 0.5 * rho * sum(v * v for v in vel)
    out = [rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + kin]
    return np.stack([np.broadcast_to(np.asarray(o, np.float64), np.shape(rho)) for o in out])


def _centres(n, h, x0):
    return x0 + (np.arange(n) + 0.5) * h


def _cell_average(func, xs, ys, zs=None):
    """Average ``func(X, Y[, Z]) -> (nv, ...)`` over zones by tensor Gauss (4 per axis)."""
    hx = xs[1] - xs[0] if len(xs) > 1 else 1.0
    hy = ys[1] - ys[0] if len(ys) > 1 else 1.0
    acc = None
    if zs is None:
        for a, wa in zip(_GX, _GW):
            for b, wb in zip(_GX, _GW):
                Y, X = np.meshgrid(ys + b * hy, xs + a * hx, indexing="ij")
                v = wa * wb * func(X, Y)
                acc = v if acc is None else acc + v
        return acc
    hz = zs[1] - zs[0] if len(zs) > 1 else 1.0
    for a, wa in zip(_GX, _GW):
        for b, wb in zip(_GX, _GW):
            for c, wc in zip(_GX, _GW):
                Z, Y, X = np.meshgrid(zs + c * hz, ys + b * hy, xs + a * hx, indexing="ij")
                v = wa * wb * wc * func(X, Y, Z)
                acc = v if acc is None else acc + v
    return acc


def _vortex_prim(X, Y, t, L, eps, gamma, uinf):
    """Isentropic vortex (Balsara & Shu) on a periodic square of side L, centre
    translated by uinf*t; nearest periodic image of the centre is used."""
    xc = (0.5 * L + uinf[0] * t) % L
    yc = (0.5 * L + uinf[1] * t) % L
    xb = np.mod(X - xc + 0.5 * L, L) - 0.5 * L
    yb = np.mod(Y - yc + 0.5 * L, L) - 0.5 * L
    r2 = xb * xb + yb * yb
    g = np.exp(0.5 * (1.0 - r2))
    du = -(eps / (2.0 * math.pi)) * g * yb
    dv = (eps / (2.0 * math.pi)) * g * xb
    T = 1.0 - (gamma - 1.0) * eps * eps / (8.0 * gamma * math.pi ** 2) * g * g
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    return rho, uinf[0] + du, uinf[1] + dv, p


def vortex2d(n=64, L=10.0, eps=5.0, gamma=1.4, uinf=(1.0, 1.0), t=0.0):
    """2D isentropic vortex, periodic [0,L]^2, zone averages at time t (exact solution)."""
    h = L / n
    xs = _centres(n, h, 0.0)

    def f(X, Y):
        rho, u, v, p = _vortex_prim(X, Y, t, L, eps, gamma, uinf)
        return prim_to_cons(rho, (u, v), p, gamma)

    U = _cell_average(f, xs, xs)
    return Problem(U=U, ndim=2, n=(n, n, 1), h=(h, h, h), origin=(0.0, 0.0, 0.0),
                   bc=("periodic",) * 3, gamma=gamma,
                   meta=dict(name="vortex2d", L=L, eps=eps, uinf=uinf, t=t))


def vortex_exact_density(n, t, L=10.0, eps=5.0, gamma=1.4, uinf=(1.0, 1.0)):
    """Zone-averaged exact density of the translated 2D vortex at time t."""
    return vortex2d(n, L, eps, gamma, uinf, t).U[0]


def vortex3d_perturbed(n=128, seed=2, L=10.0, eps=5.0, gamma=1.4, amp=1e-2, modes=4,
                       uinf=(1.0, 1.0, 0.0)):
    """3D workload: the 2D vortex extruded along z (w = 0) with the density scaled
    by (1 + delta), delta a seeded sum of ``modes`` Fourier modes per axis of total
    amplitude ``amp``, at fixed pressure and velocity.  Periodic [0,L]^3."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, size=(3, modes))
    phi = rng.uniform(0.0, 2.0 * math.pi, size=(3, modes))
    h = L / n
    xs = _centres(n, h, 0.0)

    def f(X, Y, Z):
        rho, u, v, p = _vortex_prim(X, Y, 0.0, L, eps, gamma, uinf)
        delta = np.zeros_like(X)
        for ax, C in enumerate((X, Y, Z)):
            for m in range(modes):
                delta = delta + a[ax, m] * np.sin(2.0 * math.pi * (m + 1) * C / L + phi[ax, m])
        delta = amp * delta / a.sum()
        rho = rho * (1.0 + delta)
        return prim_to_cons(rho, (u, v, np.zeros_like(X)), p, gamma)

    U = _cell_average(f, xs, xs, xs)
    return Problem(U=U, ndim=3, n=(n, n, n), h=(h, h, h), origin=(0.0, 0.0, 0.0),
                   bc=("periodic",) * 3, gamma=gamma,
                   meta=dict(name="vortex3d_perturbed", seed=seed, L=L, amp=amp))


def multiblast(n=256, seed=3, nblast=16, gamma=1.4, rmin=0.05, rmax=0.1,
               rho0=1.0, p0=0.1, p_in=10.0):
    """Ambient gas at rest with ``nblast`` over-pressured spheres (seeded centres
    uniform in [0,1]^3, radii uniform in [rmin,rmax]); zone-centre sampling; outflow."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(nblast, 3))
    radii = rng.uniform(rmin, rmax, size=nblast)
    h = 1.0 / n
    xs = _centres(n, h, 0.0)
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    p = np.full(X.shape, p0)
    for c, r in zip(centres, radii):
        inside = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2 <= r * r
        p[inside] = p_in
    rho = np.full(X.shape, rho0)
    zero = np.zeros_like(X)
    U = prim_to_cons(rho, (zero, zero, zero), p, gamma)
    return Problem(U=U, ndim=3, n=(n, n, n), h=(h, h, h), origin=(0.0, 0.0, 0.0),
                   bc=("outflow",) * 3, gamma=gamma,
                   meta=dict(name="multiblast", seed=seed, centres=centres, radii=radii))


def four_quadrant(n=384, seed=5, gamma=1.4, ndim=3, block=None):
    """Four constant states split at x = 1/2, y = 1/2 (independent of z); per
    quadrant rho ~ U[0.5,1.5], p ~ U[0.1,1], in-plane velocity of speed ~ U[0,0.5].
    block = (lo, m): only the zones lo .. lo+m-1 of every axis (the same
    values as that slice of the whole grid; outflow boundaries)."""
    rng = np.random.default_rng(seed)
    rho_q = rng.uniform(0.5, 1.5, 4)
    p_q = rng.uniform(0.1, 1.0, 4)
    s_q = rng.uniform(0.0, 0.5, 4)
    th_q = rng.uniform(0.0, 2.0 * math.pi, 4)
    h = 1.0 / n
    xs = _centres(n, h, 0.0)
    if block is not None:
        lo, m = block
        xs = xs[lo:lo + m]
    if ndim == 3:
        Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    else:
        Y, X = np.meshgrid(xs, xs, indexing="ij")
    q = (X >= 0.5).astype(int) + 2 * (Y >= 0.5).astype(int)
    rho = rho_q[q]
    p = p_q[q]
    u = s_q[q] * np.cos(th_q[q])
    v = s_q[q] * np.sin(th_q[q])
    vel = (u, v, np.zeros_like(u)) if ndim == 3 else (u, v)
    U = prim_to_cons(rho, vel, p, gamma)
    m = len(xs)
    nn = (m, m, m if ndim == 3 else 1)
    x0 = float(xs[0] - 0.5 * h)
    return Problem(U=U, ndim=ndim, n=nn, h=(h, h, h), origin=(x0, x0, x0 if ndim == 3 else 0.0),
                   bc=("outflow",) * 3, gamma=gamma,
                   meta=dict(name="four_quadrant", seed=seed, rho=rho_q, p=p_q, block=block))


def sod(n=100, axis=0, ndim=2, ntrans=4, gamma=1.4, left=(1.0, 0.0, 1.0),
        right=(0.125, 0.0, 0.1)):
    """Sod shock tube along ``axis`` on [0,1], interface at 1/2 on a zone face;
    ``ntrans`` zones across the other axes; outflow everywhere."""
    shape = [ntrans] * ndim
    shape[ndim - 1 - axis] = n
    nn = [ntrans, ntrans, ntrans if ndim == 3 else 1]
    nn[axis] = n
    h = 1.0 / n
    coord = _centres(n, h, 0.0)
    sl = [None] * ndim
    sl[ndim - 1 - axis] = slice(None)
    c = coord[tuple(sl)] * np.ones(shape)
    L = c < 0.5
    rho = np.where(L, left[0], right[0])
    un = np.where(L, left[1], right[1])
    p = np.where(L, left[2], right[2])
    vel = [np.zeros(shape) for _ in range(ndim)]
    vel[axis] = un
    U = prim_to_cons(rho, vel, p, gamma)
    return Problem(U=U, ndim=ndim, n=tuple(nn), h=(h, h, h), origin=(0.0, 0.0, 0.0),
                   bc=("outflow",) * 3, gamma=gamma,
                   meta=dict(name="sod", axis=axis, left=left, right=right))


def entropy_wave(n=32, ndim=2, amp=0.2, vel=(1.0, 0.5, 0.25), p0=1.0, gamma=1.4, t=0.0,
                 kvec=(1, 1, 1)):
    """Density wave rho = 1 + amp*sin(2 pi k.(x - vel t)) with constant velocity and
    pressure on the periodic unit box: an exact solution of the Euler equations."""
    h = 1.0 / n
    xs = _centres(n, h, 0.0)
    vel = tuple(vel[:ndim])
    k = kvec[:ndim]

    def rho_of(*C):
        arg = sum(k[d] * (C[d] - vel[d] * t) for d in range(ndim))
        return 1.0 + amp * np.sin(2.0 * math.pi * arg)

    if ndim == 2:
        def f(X, Y):
            r = rho_of(X, Y)
            return prim_to_cons(r, [vel[d] * np.ones_like(X) for d in range(2)], p0 * np.ones_like(X), gamma)
        U = _cell_average(f, xs, xs)
        nn = (n, n, 1)
    else:
        def f(X, Y, Z):
            r = rho_of(X, Y, Z)
            return prim_to_cons(r, [vel[d] * np.ones_like(X) for d in range(3)], p0 * np.ones_like(X), gamma)
        U = _cell_average(f, xs, xs, xs)
        nn = (n, n, n)
    return Problem(U=U, ndim=ndim, n=nn, h=(h, h, h), origin=(0.0, 0.0, 0.0),
                   bc=("periodic",) * 3, gamma=gamma,
                   meta=dict(name="entropy_wave", amp=amp, vel=vel, t=t))


def uniform(n=(8, 8, 8), ndim=3, rho=1.0, vel=(0.3, -0.2, 0.1), p=0.7, gamma=1.4,
            bc="periodic", h=(0.1, 0.1, 0.1)):
    """Constant state (free stream)."""
    shape = (n[2], n[1], n[0]) if ndim == 3 else (n[1], n[0])
    r = np.full(shape, rho)
    V = [np.full(shape, vel[d]) for d in range(ndim)]
    U = prim_to_cons(r, V, np.full(shape, p), gamma)
    nn = (n[0], n[1], n[2] if ndim == 3 else 1)
    return Problem(U=U, ndim=ndim, n=nn, h=tuple(h), origin=(0.0, 0.0, 0.0),
                   bc=(bc,) * 3, gamma=gamma, meta=dict(name="uniform"))


def random_smooth(n=(8, 8, 8), ndim=3, seed=0, amp=0.05, gamma=1.4, h=(0.1, 0.1, 0.1),
                  bc="periodic"):
    """Seeded smooth random state: each primitive field is a base value times
    (1 + amp * a few random low Fourier modes).  Used for parity cases with
    non-symmetric, non-trivial data in every variable."""
    rng = np.random.default_rng(seed)
    shape = (n[2], n[1], n[0]) if ndim == 3 else (n[1], n[0])
    grids = np.meshgrid(*[(np.arange(s) + 0.5) / s for s in shape], indexing="ij")

    def field(base):
        f = np.zeros(shape)
        for _ in range(3):
            k = rng.integers(1, 3, size=ndim)
            ph = rng.uniform(0, 2 * math.pi)
            arg = sum(2 * math.pi * k[d] * grids[d] for d in range(ndim)) + ph
            f = f + rng.uniform(-1, 1) * np.sin(arg)
        return base * (1.0 + amp * f)

    rho = field(1.0)
    p = field(1.0)
    V = [field(1.0) * rng.uniform(-0.5, 0.5) for _ in range(ndim)]
    U = prim_to_cons(rho, V, p, gamma)
    nn = (n[0], n[1], n[2] if ndim == 3 else 1)
    return Problem(U=U, ndim=ndim, n=nn, h=tuple(h), origin=(0.0, 0.0, 0.0),
                   bc=(bc,) * 3, gamma=gamma, meta=dict(name="random_smooth", seed=seed))


def cold_wave(n=32, ndim=2, amp=2.0, p0=1e-3, gamma=1.4, axis=0):
    """Cold flow on the periodic unit box: rho = 1, pressure p0 (small), and a
    velocity sin wave u_axis = amp * sin(2 pi x_axis) along one axis.  Kinetic
    energy dominates, so limited slopes of the conserved variables easily give
    negative face pressures: the case for the positivity fallback."""
    shape = (n,) * ndim
    h = 1.0 / n
    coord = _centres(n, h, 0.0)
    sl = [None] * ndim
    sl[ndim - 1 - axis] = slice(None)
    u = amp * np.sin(2.0 * math.pi * coord)[tuple(sl)] * np.ones(shape)
    vel = [np.zeros(shape) for _ in range(ndim)]
    vel[axis] = u
    U = prim_to_cons(np.ones(shape), vel, p0 * np.ones(shape), gamma)
    nn = (n, n, n if ndim == 3 else 1)
    return Problem(U=U, ndim=ndim, n=nn, h=(h, h, h), origin=(0.0, 0.0, 0.0),
                   bc=("periodic",) * 3, gamma=gamma, meta=dict(name="cold_wave", amp=amp, p0=p0))

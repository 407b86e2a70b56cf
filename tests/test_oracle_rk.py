"""Pins of the oracle's Runge-Kutta steppers (Sec. I.1; Table IV's two-,
three- and five-stage schemes): the coefficient tables against the classical
order conditions, the method-of-lines operator against the exact time
derivative of linear advection, the step as the Shu-Osher combination of
operator evaluations, conservation, free stream, the design order on the
vortex, Sod, and the positivity fallback."""
import math

import numpy as np
import pytest

import icgen
import oracle
from tests.exact_riemann import zone_average_density

STAGES = {"rk2": 2, "rk3": 3, "rk4": 5}
ORDER = {"rk2": 2, "rk3": 3, "rk4": 4}


def butcher(stepper):
    """Butcher tableau (A, b, c) of a Shu-Osher table: u(i) = u(0) + sum_j A_ij dt L(u(j))."""
    s = STAGES[stepper]
    rows = np.zeros((s + 1, s))
    asum = np.zeros(s + 1)
    for i, k, alpha, beta in oracle.rk_table(stepper):
        asum[i] += alpha
        if k > 0:
            rows[i] += alpha * rows[k]
        rows[i, k] += beta
    A, b = rows[:s], rows[s]
    return A, b, A.sum(axis=1), asum[1:]


@pytest.mark.parametrize("stepper", ["rk2", "rk3", "rk4"])
def test_rk_tables_meet_the_order_conditions(stepper):
    A, b, c, asum = butcher(stepper)
    np.testing.assert_allclose(asum, 1.0, atol=1e-14)            # consistency of the convex form
    for i, k, alpha, beta in oracle.rk_table(stepper):
        assert alpha >= 0.0 and beta >= 0.0                       # strong-stability-preserving form
        assert 0 <= k < i <= STAGES[stepper]
    p = ORDER[stepper]
    conds = [(b.sum(), 1.0), (b @ c, 1 / 2)]
    if p >= 3:
        conds += [(b @ c**2, 1 / 3), (b @ A @ c, 1 / 6)]
    if p >= 4:
        conds += [(b @ c**3, 1 / 4), (b @ (c * (A @ c)), 1 / 8), (b @ A @ c**2, 1 / 12), (b @ A @ A @ c, 1 / 24)]
    for got, want in conds:
        assert abs(got - want) < 1e-14, (stepper, got, want)
    # and the order is exactly p: some condition of order p + 1 fails
    nxt = {2: [(b @ c**2, 1 / 3), (b @ A @ c, 1 / 6)],
           3: [(b @ c**3, 1 / 4), (b @ (c * (A @ c)), 1 / 8), (b @ A @ c**2, 1 / 12), (b @ A @ A @ c, 1 / 24)],
           4: [(b @ c**4, 1 / 5), (b @ A @ A @ A @ c, 1 / 120)]}[p]
    assert max(abs(g - w) for g, w in nxt) > 1e-4


def _poly_state(ndim, n, deg, vel, h, p0=0.9, gamma=1.4, seed=0):
    """Zone averages of rho = 1 + 0.02 * a seeded polynomial of degree deg,
    with constant velocity and pressure, and the exact zone-averaged time
    derivative of linear advection."""
    rng = np.random.default_rng(seed)
    coef = {}
    for a in range(deg + 1):
        for b_ in range(deg + 1 - a):
            for c_ in range(deg + 1 - a - b_ if ndim == 3 else 1):
                coef[(a, b_, c_)] = rng.uniform(-1, 1)
    gx, gw = np.polynomial.legendre.leggauss(4)
    gx, gw = 0.5 * gx, 0.5 * gw

    def rho(X, Y, Z):
        r = 0.0
        for (a, b_, c_), v in coef.items():
            r = r + v * X**a * Y**b_ * Z**c_
        return 1.0 + 0.02 * r

    shape = (n,) * ndim
    cen = [(np.arange(n) + 0.5) * h[d] - 0.5 * n * h[d] for d in range(ndim)]
    grids = np.meshgrid(*cen[::-1], indexing="ij")      # slowest axis first
    C = list(grids[::-1]) + ([np.zeros(shape)] if ndim == 2 else [])   # x, y, z centres

    def avg(fn, fixed=None):
        acc = np.zeros(shape)
        axes = [d for d in range(ndim) if d != fixed]
        for idx in np.ndindex(*([4] * len(axes))):
            P = [C[0], C[1], C[2]]
            w = 1.0
            for a_i, d in zip(idx, axes):
                P[d] = P[d] + gx[a_i] * h[d]
                w *= gw[a_i]
            if fixed is not None:
                P[fixed] = P[fixed] + fn[1] * h[fixed]
            acc = acc + w * (fn[0](*P))
        return acc

    rbar = avg((rho, 0.0))
    U = icgen.prim_to_cons(rbar, [np.full(shape, vel[d]) for d in range(ndim)], np.full(shape, p0), gamma)
    drho = np.zeros(shape)
    for d in range(ndim):
        drho -= vel[d] * (avg((rho, 0.5), fixed=d) - avg((rho, -0.5), fixed=d)) / h[d]
    dU = np.stack([drho] + [vel[d] * drho for d in range(ndim)] + [0.5 * sum(v * v for v in vel) * drho])
    return U, dU


@pytest.mark.parametrize("ndim,order", [(2, 2), (2, 3), (2, 4), (3, 2), (3, 3), (3, 4)])
def test_operator_is_exact_for_linear_advection(ndim, order):
    """Polynomial density (degree 1 at second order, 2 otherwise: every
    candidate stencil and the MC slope reproduce it), constant velocity and
    pressure: dt L(U) equals dt times the exact zone-averaged time derivative
    away from the (outflow) boundary."""
    n = 9
    h = (0.1, 0.13, 0.08)
    vel = (0.4, -0.3, 0.25)[:ndim]
    U, dU = _poly_state(ndim, n, 1 if order == 2 else 2, vel, h, seed=order + ndim)
    c = oracle.make_cfg(ndim, (n, n, n), order, h, bc=("outflow",) * 3, stepper="rk3")
    dt = 0.01
    L = oracle.rk_operator(c, U, dt)
    r = 3
    sl = (slice(None),) + (slice(r, n - r),) * ndim
    np.testing.assert_allclose(L[sl], dt * dU[sl], rtol=1e-9, atol=1e-13)


def test_step_is_the_shu_osher_combination():
    """An SSP-RK(3,3) step equals u1 = u + L(u), u2 = 3/4 u + 1/4 (u1 + L(u1)),
    u3 = 1/3 u + 2/3 (u2 + L(u2)) built here from operator evaluations (the
    published coefficients, typed here, not read from the oracle)."""
    pb = icgen.random_smooth(n=(8, 7, 6), ndim=3, seed=9, amp=0.3)
    c = oracle.cfg_from_problem(pb, 3, stepper="rk3")
    dt = 0.5 * oracle.cfl_dt(c, pb.U)[0]
    u0 = pb.U
    u1 = u0 + oracle.rk_operator(c, u0, dt)
    u2 = 0.75 * u0 + 0.25 * (u1 + oracle.rk_operator(c, u1, dt))
    u3 = u0 / 3.0 + 2.0 / 3.0 * (u2 + oracle.rk_operator(c, u2, dt))
    np.testing.assert_allclose(oracle.step(c, u0, dt), u3, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("order,stepper", [(2, "rk2"), (3, "rk3"), (4, "rk4")])
@pytest.mark.parametrize("ndim", [2, 3])
def test_rk_conservation_and_free_stream(order, stepper, ndim):
    pb = icgen.random_smooth(n=(8, 7, 6), ndim=ndim, seed=order, amp=0.3)
    c = oracle.cfg_from_problem(pb, order, stepper=stepper)
    dt, _ = oracle.cfl_dt(c, pb.U)
    U1 = oracle.step(c, pb.U, dt)
    ax = tuple(range(1, ndim + 1))
    scale = np.maximum(np.abs(pb.U).sum(axis=ax), 1.0)
    assert (np.abs(U1.sum(axis=ax) - pb.U.sum(axis=ax)) / scale).max() < 1e-14
    assert np.abs(U1 - pb.U).max() > 1e-6
    fs = icgen.uniform(n=(7, 6, 5), ndim=ndim, bc="outflow", h=(0.1, 0.13, 0.07))
    cf = oracle.cfg_from_problem(fs, order, stepper=stepper)
    np.testing.assert_allclose(oracle.step(cf, fs.U, oracle.cfl_dt(cf, fs.U)[0]), fs.U, rtol=1e-14, atol=1e-14)


@pytest.mark.slow
@pytest.mark.parametrize("order,stepper,ns", [(2, "rk2", (32, 64, 128)), (3, "rk3", (32, 64, 128)),
                                              (4, "rk4", (32, 64))])
def test_rk_vortex_design_order(order, stepper, ns):
    errs = []
    for n in ns:
        pb = icgen.vortex2d(n)
        c = oracle.cfg_from_problem(pb, order, stepper=stepper)
        U, t, _ = oracle.run(c, pb.U, t_end=1.0)
        errs.append(np.abs(U[0] - icgen.vortex_exact_density(n, t)).mean())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] >= order - 0.25, (errs, orders)
    assert orders[-1] <= order + 1.0


def test_rk3_sod_against_the_exact_riemann_solution():
    n, t_end = 100, 0.2
    pb = icgen.sod(n=n, axis=0, ndim=2, ntrans=2)
    c = oracle.cfg_from_problem(pb, 3, stepper="rk3")
    U, t, _ = oracle.run(c, pb.U, t_end=t_end)
    exact = zone_average_density((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), n, t)
    assert np.abs(U[0, 0] - exact).mean() < 6e-3
    np.testing.assert_allclose(U[:, 1], U[:, 0], rtol=0, atol=1e-15)


def test_rk_positivity_fallback_on_the_blast():
    """Multi-blast with the five-stage scheme at fourth order: without the
    zone fallback the state turns non-physical; with it the run stays
    admissible and conservative (periodic box)."""
    pb = icgen.multiblast(n=16, seed=3)
    off = oracle.make_cfg(3, pb.n, 4, pb.h, bc=("periodic",) * 3, positivity=False, stepper="rk4")
    U = pb.U
    failed = False
    for _ in range(3):
        dt, bad = oracle.cfl_dt(off, U)
        if bad >= 0:
            failed = True
            break
        U = oracle.step(off, U, dt)
    assert failed or oracle.cfl_dt(off, U)[1] >= 0
    on = oracle.make_cfg(3, pb.n, 4, pb.h, bc=("periodic",) * 3, stepper="rk4")
    U, hits = pb.U, 0
    for _ in range(3):
        dt, bad = oracle.cfl_dt(on, U)
        assert bad < 0
        U, nb = oracle.step_count(on, U, dt)
        hits += nb
    assert hits > 0
    tot0, tot1 = pb.U.sum(axis=(1, 2, 3)), U.sum(axis=(1, 2, 3))
    assert (np.abs(tot1 - tot0) / np.maximum(np.abs(pb.U).sum(axis=(1, 2, 3)), 1.0)).max() < 1e-13


def test_rk_step_depends_on_zones_within_the_stage_reach():
    """Five stages of third/fourth-order reconstruction reach 3 zones each: the
    step at a zone computed on a periodic cut-out of half-width 17 (outflow at
    the cut) equals the whole-mesh step there; with half-width 13 the cut is
    inside the reach and the result differs."""
    n = 40
    pb = icgen.vortex3d_perturbed(n=n, seed=2)
    c = oracle.cfg_from_problem(pb, 4, stepper="rk4")
    dt, _ = oracle.cfl_dt(c, pb.U)
    full = oracle.step(c, pb.U, dt)
    i, j, k = 3, 21, 38
    for r, same in ((17, True), (13, False)):
        ix = [(i + d) % n for d in range(-r, r + 1)]
        jx = [(j + d) % n for d in range(-r, r + 1)]
        kx = [(k + d) % n for d in range(-r, r + 1)]
        sub = pb.U[:, kx][:, :, jx][:, :, :, ix]
        m = 2 * r + 1
        cut = oracle.make_cfg(3, (m, m, m), 4, pb.h, gamma=pb.gamma, bc=("outflow",) * 3, stepper="rk4")
        got = oracle.step(cut, sub, dt)[:, r, r, r]
        if same:
            np.testing.assert_array_equal(got, full[:, k, j, i])
        else:
            assert np.abs(got - full[:, k, j, i]).max() > 0.0

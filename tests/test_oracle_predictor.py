"""Pins of the oracle's ADER predictor.

Closed form: for a state with constant velocity and pressure and a density
that is a polynomial of degree <= p, the Euler equations reduce to linear
advection and their flux is affine in the state, so the predictor must
return the exact translated polynomial q(x, tau) = W(x - lam*u*tau) (p Picard
steps reproduce the terminating Taylor series).  The expected values here are
computed from the translated polynomial with numpy, in all directions at once
with different lam and velocity per axis, so a swapped axis, a wrong sign or
a wrong scale of any derivative/time term fails.
"""
import numpy as np
import numpy.polynomial.legendre as npl
import numpy.polynomial.polynomial as npp
import pytest

import oracle

XG, WG = npl.leggauss(10)
XG, WG = XG / 2, WG / 2


def _basis():
    out = []
    for k in range(4):
        c = np.zeros(4)
        c[k] = 1.0
        for b in out:
            ip = np.sum(WG * npp.polyval(XG, c) * npp.polyval(XG, b))
            c = c - ip / np.sum(WG * npp.polyval(XG, b) ** 2) * b
        out.append(c)
    return out


B = _basis()


def P(k, x):
    return npp.polyval(x, B[k])


@pytest.mark.parametrize("ndim,order", [(2, 3), (2, 4), (3, 3), (3, 4)])
def test_predictor_exact_for_linear_advection(ndim, order):
    p = order - 1
    g = 1.4
    rng = np.random.default_rng(ndim * 10 + order)
    vel = np.array([0.7, -1.3, 0.45])[:ndim]
    lam = np.array([0.11, 0.07, 0.05])
    pres = 0.8
    c = oracle.make_cfg(ndim, (4, 4, 4), order, (0.1, 0.1, 0.1), gamma=g)
    m = oracle.modes(ndim, p)
    spatial = m[m[:, 3] == 0]
    al = {tuple(s[:3]): rng.normal() * 0.05 for s in spatial}
    al[(0, 0, 0)] = 1.0
    nv = ndim + 2
    W = np.zeros((len(spatial), nv))
    for i, s in enumerate(spatial):
        a = al[tuple(s[:3])]
        W[i, 0] = a
        for d in range(ndim):
            W[i, 1 + d] = vel[d] * a
        W[i, nv - 1] = 0.5 * np.dot(vel, vel) * a + (pres / (g - 1) if i == 0 else 0.0)
    q = oracle.predict(c, lam, W)

    def rho_exact(x, tau):
        xs = [x[d] - lam[d] * vel[d] * tau for d in range(ndim)]
        zz = xs[2] if ndim == 3 else 0.0
        return sum(al[(a, b, cc)] * P(a, xs[0]) * P(b, xs[1]) * P(cc, zz)
                   for (a, b, cc) in al)

    for _ in range(20):
        x = rng.uniform(-0.5, 0.5, 3)
        tau = rng.uniform(0, 1)
        got = oracle.eval_q(c, q, x[0], x[1], x[2] if ndim == 3 else 0.0, tau)
        r = rho_exact(x, tau)
        ref = np.concatenate([[r], vel * r, [0.5 * np.dot(vel, vel) * r + pres / (g - 1)]])
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("ndim,order", [(2, 3), (3, 4)])
def test_predictor_starts_from_the_reconstruction(ndim, order):
    # q(x, tau = 0) = W(x) for a general nonlinear state
    rng = np.random.default_rng(5)
    c = oracle.make_cfg(ndim, (4, 4, 4), order, (0.1, 0.1, 0.1))
    m = oracle.modes(ndim, order - 1)
    ms = int((m[:, 3] == 0).sum())
    nv = ndim + 2
    W = rng.normal(size=(ms, nv)) * 0.05
    W[0] = [1.0] + [0.3] * ndim + [2.5]
    q = oracle.predict(c, [0.2, 0.15, 0.1], W)
    np.testing.assert_array_equal(q[:ms], W)
    for _ in range(5):
        x = rng.uniform(-0.5, 0.5, 3)
        u0 = oracle.eval_q(c, q, *x, 0.0)
        phi = [P(a, x[0]) * P(b, x[1]) * P(cc, x[2] if ndim == 3 else 0.0) for a, b, cc, _ in m[:ms]]
        np.testing.assert_allclose(u0, np.array(phi) @ W, atol=1e-14)


def test_predictor_time_derivative_matches_the_pde_at_tau0():
    # For a general smooth state the tau-derivative at tau = 0 equals
    # -sum_d lam_d dF_d/dxi_d of the projected flux of W; with a linear W of
    # small slopes it is, at the zone centre, the chain-rule derivative of the
    # exact flux (written out here, differentiated by central differences).
    g = 1.4
    ndim, order = 3, 4
    c = oracle.make_cfg(ndim, (4, 4, 4), order, (0.1, 0.1, 0.1), gamma=g)
    lam = np.array([0.01, 0.02, 0.015])
    m = oracle.modes(ndim, order - 1)
    ms = int((m[:, 3] == 0).sum())
    W = np.zeros((ms, 5))
    W[0] = [1.1, 0.3, -0.2, 0.1, 2.7]
    rng = np.random.default_rng(9)

    def flux(U, d):
        rho, mom, E = U[0], U[1:4], U[4]
        u = mom / rho
        pr = (g - 1) * (E - 0.5 * rho * u @ u)
        F = np.concatenate([[mom[d]], mom * u[d], [(E + pr) * u[d]]])
        F[1 + d] += pr
        return F

    lin_index = {}
    for i, (a, b, cc, e) in enumerate(m[:ms]):
        if a + b + cc == 1:
            lin_index[(a, b, cc)] = i
    dirs = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    for dd in dirs:  # linear (P1) slopes along x, y, z only
        W[lin_index[dd]] = rng.normal(size=5) * 1e-3
    # exact d/dxi_d F_d(W(xi)) at the centre by central differences of the exact flux
    h = 1e-4
    dUdt = np.zeros(5)
    for d in range(3):
        sl = W[lin_index[dirs[d]]]
        dF = (flux(W[0] + h * sl, d) - flux(W[0] - h * sl, d)) / (2 * h)
        dUdt -= lam[d] * dF
    q = oracle.predict(c, lam, W)
    dt = 1e-6
    num = (oracle.eval_q(c, q, 0, 0, 0, dt) - oracle.eval_q(c, q, 0, 0, 0, 0.0)) / dt
    np.testing.assert_allclose(num, dUdt, rtol=1e-3, atol=1e-9)

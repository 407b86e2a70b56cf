"""Pins of the oracle's physical flux and Riemann solvers (textbook invariants)."""
import numpy as np
import pytest

import oracle

G = 1.4


def cons(rho, vel, p):
    vel = np.asarray(vel, float)
    return np.concatenate([[rho], rho * vel, [p / (G - 1) + 0.5 * rho * vel @ vel]])


def exact_flux(U, d):
    nd = len(U) - 2
    rho, mom, E = U[0], U[1:1 + nd], U[-1]
    u = mom / rho
    p = (G - 1) * (E - 0.5 * rho * u @ u)
    F = np.concatenate([[mom[d]], mom * u[d], [(E + p) * u[d]]])
    F[1 + d] += p
    return F


def cfg(ndim, solver):
    return oracle.make_cfg(ndim, (4, 4, 4), 3, (0.1, 0.1, 0.1), gamma=G, riemann=solver)


def rand_state(rng, nd, mach=1.0):
    rho = rng.uniform(0.3, 2.0)
    p = rng.uniform(0.2, 2.0)
    c = np.sqrt(G * p / rho)
    return cons(rho, rng.uniform(-mach, mach, nd) * c, p)


@pytest.mark.parametrize("nd", [2, 3])
def test_physical_flux_closed_form(nd):
    rng = np.random.default_rng(1)
    c = cfg(nd, "hllc")
    for _ in range(10):
        U = rand_state(rng, nd)
        for d in range(nd):
            np.testing.assert_allclose(oracle.phys_flux(c, d, U), exact_flux(U, d), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("solver", ["hllc", "hll", "rusanov"])
@pytest.mark.parametrize("nd", [2, 3])
def test_consistency_equal_states_give_physical_flux(solver, nd):
    rng = np.random.default_rng(2)
    c = cfg(nd, solver)
    for _ in range(20):
        U = rand_state(rng, nd, mach=2.0)
        for d in range(nd):
            np.testing.assert_allclose(oracle.riemann(c, d, U, U), exact_flux(U, d), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("solver", ["hllc", "hll"])
def test_supersonic_states_are_upwinded(solver):
    rng = np.random.default_rng(3)
    c = cfg(3, solver)
    for _ in range(10):
        rho, p = rng.uniform(0.5, 2, 2)
        cs = np.sqrt(G * p / rho)
        UL = cons(rho, [3 * cs, 0.1, 0.2], p)
        UR = cons(rho * 1.3, [3.2 * cs, -0.1, 0.0], p * 0.9)
        np.testing.assert_allclose(oracle.riemann(c, 0, UL, UR), exact_flux(UL, 0), rtol=1e-14)
        # both states moving left supersonically: the right state's flux
        VL = cons(rho * 0.8, [-3.1 * cs, 0.2, 0.0], p * 1.1)
        VR = cons(rho, [-3 * cs, -0.3, 0.1], p)
        np.testing.assert_allclose(oracle.riemann(c, 0, VL, VR), exact_flux(VR, 0), rtol=1e-14)


def test_hllc_resolves_a_stationary_contact_exactly_and_hll_does_not():
    UL = cons(1.0, [0.0, 0.3, -0.2], 0.7)
    UR = cons(0.2, [0.0, -0.5, 0.1], 0.7)
    hllc = oracle.riemann(cfg(3, "hllc"), 0, UL, UR)
    np.testing.assert_allclose(hllc, [0.0, 0.7, 0.0, 0.0, 0.0], atol=1e-15)
    hll = oracle.riemann(cfg(3, "hll"), 0, UL, UR)
    assert abs(hll[0]) > 1e-2


def test_hllc_moving_contact_is_upwinded():
    # u and p continuous, density and tangential velocity jump: the exact
    # flux is the upwind one through the contact.
    UL = cons(1.0, [0.4, 0.3, -0.2], 0.7)
    UR = cons(0.2, [0.4, -0.5, 0.1], 0.7)
    np.testing.assert_allclose(oracle.riemann(cfg(3, "hllc"), 0, UL, UR), exact_flux(UL, 0), rtol=1e-13, atol=1e-14)
    UL2 = cons(1.0, [-0.4, 0.3, -0.2], 0.7)
    UR2 = cons(0.2, [-0.4, -0.5, 0.1], 0.7)
    np.testing.assert_allclose(oracle.riemann(cfg(3, "hllc"), 0, UL2, UR2), exact_flux(UR2, 0), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("solver", ["hllc", "hll", "rusanov"])
def test_rotational_invariance(solver):
    rng = np.random.default_rng(4)
    c = cfg(3, solver)
    for _ in range(20):
        UL, UR = rand_state(rng, 3, 1.5), rand_state(rng, 3, 1.5)
        Fx = oracle.riemann(c, 0, UL, UR)
        for d, perm in ((1, [0, 2, 1, 3, 4]), (2, [0, 3, 2, 1, 4])):
            Fd = oracle.riemann(c, d, UL[perm], UR[perm])
            np.testing.assert_allclose(Fd[perm], Fx, rtol=1e-13, atol=1e-13)


def test_hllc_mirror_symmetry():
    rng = np.random.default_rng(5)
    c = cfg(2, "hllc")
    flip = np.array([1, -1, 1, 1])
    for _ in range(20):
        UL, UR = rand_state(rng, 2, 1.5), rand_state(rng, 2, 1.5)
        F = oracle.riemann(c, 0, UL, UR)
        Fm = oracle.riemann(c, 0, UR * flip, UL * flip)
        np.testing.assert_allclose(Fm, -F * flip, rtol=1e-12, atol=1e-13)

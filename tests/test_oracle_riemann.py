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


@pytest.mark.parametrize("solver", ["hllc", "hll", "rusanov", "hllem", "hlli"])
@pytest.mark.parametrize("nd", [2, 3])
def test_consistency_equal_states_give_physical_flux(solver, nd):
    rng = np.random.default_rng(2)
    c = cfg(nd, solver)
    for _ in range(20):
        U = rand_state(rng, nd, mach=2.0)
        for d in range(nd):
            np.testing.assert_allclose(oracle.riemann(c, d, U, U), exact_flux(U, d), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("solver", ["hllc", "hll", "hllem", "hlli"])
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


@pytest.mark.parametrize("solver", ["hllc", "hll", "rusanov", "hllem", "hlli"])
def test_rotational_invariance(solver):
    rng = np.random.default_rng(4)
    c = cfg(3, solver)
    for _ in range(20):
        UL, UR = rand_state(rng, 3, 1.5), rand_state(rng, 3, 1.5)
        Fx = oracle.riemann(c, 0, UL, UR)
        for d, perm in ((1, [0, 2, 1, 3, 4]), (2, [0, 3, 2, 1, 4])):
            Fd = oracle.riemann(c, d, UL[perm], UR[perm])
            np.testing.assert_allclose(Fd[perm], Fx, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("solver", ["hllc", "hll", "rusanov", "hllem", "hlli"])
def test_mirror_symmetry(solver):
    rng = np.random.default_rng(5)
    c = cfg(2, solver)
    flip = np.array([1, -1, 1, 1])
    for _ in range(20):
        UL, UR = rand_state(rng, 2, 1.5), rand_state(rng, 2, 1.5)
        F = oracle.riemann(c, 0, UL, UR)
        Fm = oracle.riemann(c, 0, UR * flip, UL * flip)
        np.testing.assert_allclose(Fm, -F * flip, rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------------------
# Isolated shocks (Rankine-Hugoniot).  A Riemann problem whose two states are
# joined by one shock has that shock as its exact solution, and the flux at
# x/t = 0 is the upwind physical flux.  HLL and HLLC with Einfeldt's speeds
# from Roe averages reproduce it exactly: Roe's matrix has the jump as an
# eigenvector with the shock speed as eigenvalue, which makes the outer
# Einfeldt speed equal to the shock speed, and HLLC's contact speed equal to
# the post-shock velocity.  Placing the shock in a slow frame makes the star
# branches carry the flux, so the contact speed, the star states and the Roe
# sound speed all enter.
# ---------------------------------------------------------------------------

def right_facing_shock(rho_pre, p_pre, mach, s, vt):
    """States (U_L, U_R) of a shock of the u+c family moving at lab speed s
    into the resting-frame pre-shock gas (rho_pre, p_pre) on the right, with
    shock Mach number mach; vt: tangential velocity, continuous across it.
    Normal-shock relations in the shock frame (e.g. Landau-Lifshitz Sec. 89)."""
    g = G
    c_pre = np.sqrt(g * p_pre / rho_pre)
    w_pre = -mach * c_pre                                   # pre-shock gas enters from the right
    rho_post = rho_pre * (g + 1) * mach ** 2 / ((g - 1) * mach ** 2 + 2)
    p_post = p_pre * (2 * g * mach ** 2 - (g - 1)) / (g + 1)
    w_post = w_pre * rho_pre / rho_post                     # mass flux continuity
    UL = cons(rho_post, [s + w_post, *vt], p_post)
    UR = cons(rho_pre, [s + w_pre, *vt], p_pre)
    return UL, UR, s + w_post


def mirror(U):
    V = U.copy()
    V[1] = -V[1]
    return V


def shock_cases():
    rng = np.random.default_rng(11)
    out = []
    for _ in range(12):
        rho, p = rng.uniform(0.4, 2.0), rng.uniform(0.2, 3.0)
        mach = rng.uniform(1.05, 6.0)
        vt = rng.uniform(-0.7, 0.7, 2)
        # post-shock speed relative to the shock: |w_post| = M c rho_pre / rho_post
        _, _, u_post0 = right_facing_shock(rho, p, mach, 0.0, vt)
        wr = abs(u_post0)
        # lab shock speeds: behind the contact branch, between contact and
        # shock (right star), left of the face, and far to the right
        for s in (0.3 * wr, 0.8 * wr, 1.5 * wr, -0.4 * wr):
            out.append((rho, p, mach, s, vt))
    return out


@pytest.mark.parametrize("solver", ["hll", "hllc", "hllem", "hlli"])
def test_isolated_shock_gives_the_exact_upwind_flux(solver):
    c = cfg(3, solver)
    n_star = 0
    for rho, p, mach, s, vt in shock_cases():
        UL, UR, u_post = right_facing_shock(rho, p, mach, s, vt)
        # Rankine-Hugoniot holds for the constructed states (pins the fixture)
        np.testing.assert_allclose(exact_flux(UR, 0) - exact_flux(UL, 0), s * (UR - UL), rtol=1e-12, atol=1e-12)
        exact = exact_flux(UL, 0) if s > 0 else exact_flux(UR, 0)
        F = oracle.riemann(c, 0, UL, UR)
        np.testing.assert_allclose(F, exact, rtol=1e-12, atol=1e-12 * np.abs(exact).max())
        # the mirror image: a shock of the u-c family moving at -s
        VL, VR = mirror(UR), mirror(UL)
        exact_m = exact_flux(VR, 0) if s > 0 else exact_flux(VL, 0)
        Fm = oracle.riemann(c, 0, VL, VR)
        np.testing.assert_allclose(Fm, exact_m, rtol=1e-12, atol=1e-12 * np.abs(exact_m).max())
        n_star += (0 < s) and (u_post < 0)
    assert n_star >= 12          # the star branch behind the contact was exercised


@pytest.mark.parametrize("solver", ["hll", "hllc", "hllem", "hlli"])
def test_isolated_shock_along_every_axis(solver):
    c = cfg(3, solver)
    for rho, p, mach, s, vt in shock_cases()[:8]:
        UL, UR, _ = right_facing_shock(rho, p, mach, s, vt)
        for d, perm in ((1, [0, 2, 1, 3, 4]), (2, [0, 3, 2, 1, 4])):
            F = oracle.riemann(c, d, UL[perm], UR[perm])
            exact = exact_flux(UL[perm] if s > 0 else UR[perm], d)
            np.testing.assert_allclose(F, exact, rtol=1e-12, atol=1e-12 * np.abs(exact).max())


def test_rusanov_smears_an_isolated_shock():
    # the single-speed solver is not exact there: the pins above can tell the solvers apart
    c = cfg(3, "rusanov")
    rho, p, mach, s, vt = shock_cases()[0]
    UL, UR, _ = right_facing_shock(rho, p, mach, s, vt)
    F = oracle.riemann(c, 0, UL, UR)
    assert np.abs(F - exact_flux(UL, 0)).max() > 1e-3


# ---------------------------------------------------------------------------
# Linearly degenerate waves.  A jump in density and tangential velocity at
# equal normal velocity and pressure is a contact (with shear): its exact
# solution moves it unchanged at the normal velocity.  HLLC, HLLEM and HLLI
# restore the dissipation HLL adds there; at rest all three are exact, and
# HLLI's anti-diffusion factor also makes a moving contact exact.
# ---------------------------------------------------------------------------

def contact_cases(u):
    rng = np.random.default_rng(12)
    out = []
    for _ in range(20):
        p = rng.uniform(0.2, 2.0)
        rl, rr = rng.uniform(0.1, 3.0, 2)
        vl, vr = rng.uniform(-0.8, 0.8, (2, 2))
        out.append((cons(rl, [u, *vl], p), cons(rr, [u, *vr], p)))
    return out


@pytest.mark.parametrize("solver", ["hllc", "hllem", "hlli"])
def test_resting_contact_and_shear_are_exact(solver):
    c = cfg(3, solver)
    for UL, UR in contact_cases(0.0):
        p = (G - 1) * (UL[-1] - 0.5 * (UL[1:4] @ UL[1:4]) / UL[0])
        np.testing.assert_allclose(oracle.riemann(c, 0, UL, UR), [0.0, p, 0.0, 0.0, 0.0], atol=1e-14)


@pytest.mark.parametrize("u", [0.45, -0.3, 0.05])
def test_hlli_resolves_a_moving_contact_exactly(u):
    c = cfg(3, "hlli")
    for UL, UR in contact_cases(u):
        exact = exact_flux(UL, 0) if u > 0 else exact_flux(UR, 0)
        np.testing.assert_allclose(oracle.riemann(c, 0, UL, UR), exact, rtol=1e-12,
                                   atol=1e-13 * np.abs(exact).max())


def test_hllem_moving_contact_error_lies_between_hlli_and_hll():
    # HLLEM keeps a fraction |u|/(c+|u|) of HLL's contact dissipation: its
    # error is positive, below HLL's, and vanishes as the contact comes to rest
    errs = {}
    for u in (0.4, 0.1, 0.01):
        for solver in ("hll", "hllem"):
            c = cfg(3, solver)
            e = 0.0
            for UL, UR in contact_cases(u):
                e = max(e, np.abs(oracle.riemann(c, 0, UL, UR) - exact_flux(UL, 0)).max())
            errs[(solver, u)] = e
    for u in (0.4, 0.1, 0.01):
        assert 0 < errs[("hllem", u)] < 0.5 * errs[("hll", u)]
    assert errs[("hllem", 0.01)] < 0.1 * errs[("hllem", 0.4)]


@pytest.mark.parametrize("solver", ["hllem", "hlli"])
def test_anti_diffusion_lies_in_the_degenerate_fields(solver):
    # F - F_HLL is a combination of the entropy and shear eigenvectors of
    # Roe's matrix, so it has no component along the two acoustic left
    # eigenvectors: l_pm . dF = 0, with l_pm the rows of the inverse of the
    # eigenvector matrix built here from the Roe state and numpy's inverse.
    rng = np.random.default_rng(13)
    for _ in range(30):
        UL, UR = rand_state(rng, 3, 0.8), rand_state(rng, 3, 0.8)
        dF = oracle.riemann(cfg(3, solver), 0, UL, UR) - oracle.riemann(cfg(3, "hll"), 0, UL, UR)
        sl, sr = np.sqrt(UL[0]), np.sqrt(UR[0])
        pl = (G - 1) * (UL[4] - 0.5 * UL[1:4] @ UL[1:4] / UL[0])
        pr = (G - 1) * (UR[4] - 0.5 * UR[1:4] @ UR[1:4] / UR[0])
        u = (sl * UL[1:4] / UL[0] + sr * UR[1:4] / UR[0]) / (sl + sr)
        H = (sl * (UL[4] + pl) / UL[0] + sr * (UR[4] + pr) / UR[0]) / (sl + sr)
        a = np.sqrt((G - 1) * (H - 0.5 * u @ u))
        R = np.array([[1, 1, 0, 0, 1],
                      [u[0] - a, u[0], 0, 0, u[0] + a],
                      [u[1], u[1], 1, 0, u[1]],
                      [u[2], u[2], 0, 1, u[2]],
                      [H - u[0] * a, 0.5 * u @ u, u[1], u[2], H + u[0] * a]])
        Linv = np.linalg.inv(R)
        assert abs(Linv[0] @ dF) <= 1e-12 * (1 + np.abs(dF).max())
        assert abs(Linv[4] @ dF) <= 1e-12 * (1 + np.abs(dF).max())
        assert np.abs(dF).max() > 1e-6      # and it does change the HLL flux


def test_hllc_with_undefined_wave_speeds_falls_through_to_the_right_flux():
    """Negative pressure on both sides (as in the face states of a cold flow
    without the positivity fallback) leaves the sound speeds and the Roe sound
    speed undefined (NaN).  Taken in the defined order S_L >= 0, S* >= 0,
    S_R > 0, every test fails and HLLC returns the physical flux of the right
    state; HLL returns NaN (its last branch is the HLL average)."""
    c2 = oracle.make_cfg(2, (4, 4, 1), 4, (0.1, 0.1, 0.1), riemann="hllc")
    UL = np.array([0.984452238, 0.378705354, 0.0, 0.0692566391])
    UR = np.array([0.984446347, 0.378744513, 0.0, 0.0694100894])
    G = 1.4
    for U in (UL, UR):
        assert (G - 1) * (U[3] - 0.5 * U[1] ** 2 / U[0]) < 0
    F = oracle.riemann(c2, 0, UL, UR)
    np.testing.assert_array_equal(F, oracle.phys_flux(c2, 0, UR))
    ch = oracle.make_cfg(2, (4, 4, 1), 4, (0.1, 0.1, 0.1), riemann="hll")
    assert np.isnan(oracle.riemann(ch, 0, UL, UR)).all()

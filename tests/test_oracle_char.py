"""Pins of the oracle's characteristic-variable reconstruction.

Each 1D WENO application projects its five-zone line on the eigenvectors of
the flux Jacobian along the sweep axis (at the mean of the zone the
application is centred at), applies the WENO operator field by field and maps
the coefficients back.  The pins: the eigenvectors diagonalise a numerically
differentiated flux Jacobian; with linear weights the projection cancels and
the result equals the component-wise reconstruction; quadratic data are
reproduced for any weights; an entropy wave (a density jump at constant
velocity and pressure) lies in one field, so every variable takes the density's
nonlinear weights; a problem along y is the one along x; and the whole scheme
keeps conservation, the Sod solution and the design order.
"""
import numpy as np
import pytest

import icgen
import oracle

G = 1.4


def cons(rho, vel, p):
    vel = np.asarray(vel, float)
    return np.concatenate([[rho], rho * vel, [p / (G - 1) + 0.5 * rho * vel @ vel]])


def flux(U, d):
    nd = len(U) - 2
    rho, mom, E = U[0], U[1:1 + nd], U[-1]
    u = mom / rho
    p = (G - 1) * (E - 0.5 * rho * u @ u)
    F = np.concatenate([[mom[d]], mom * u[d], [(E + p) * u[d]]])
    F[1 + d] += p
    return F


def cfg(ndim, order=4, linear=False, characteristic=True):
    return oracle.make_cfg(ndim, (8, 8, 8), order, (0.1, 0.1, 0.1), gamma=G, linear_weno=linear,
                           characteristic=characteristic)


@pytest.mark.parametrize("ndim", [2, 3])
def test_eigenvectors_diagonalise_the_flux_jacobian(ndim):
    rng = np.random.default_rng(1)
    c = cfg(ndim)
    for _ in range(10):
        rho, p = rng.uniform(0.3, 2.0), rng.uniform(0.2, 2.0)
        U = cons(rho, rng.uniform(-1.0, 1.0, ndim), p)
        a = np.sqrt(G * p / rho)
        for d in range(ndim):
            R, L = oracle.char_eigen(c, d, U)
            np.testing.assert_allclose(L @ R, np.eye(ndim + 2), atol=1e-13)
            h = 1e-6
            J = np.stack([(flux(U + h * e, d) - flux(U - h * e, d)) / (2 * h) for e in np.eye(ndim + 2)], axis=1)
            un = U[1 + d] / rho
            lam = np.array([un - a] + [un] * ndim + [un + a])
            np.testing.assert_allclose(J @ R, R * lam, rtol=0, atol=1e-7 * np.abs(J).max())


def rand_block(rng, ndim, jump=False):
    nzb = 5 if ndim == 3 else 1
    rho = rng.uniform(0.8, 1.2, (nzb, 5, 5))
    p = rng.uniform(0.8, 1.2, (nzb, 5, 5))
    if jump:
        rho[..., 3:] *= 4.0
        p[..., 3:] *= 6.0
    vel = rng.uniform(-0.4, 0.4, (ndim, nzb, 5, 5))
    U = np.stack([rho, *(rho * v for v in vel), p / (G - 1) + 0.5 * rho * (vel ** 2).sum(0)])
    return np.ascontiguousarray(U if ndim == 3 else U[:, 0])


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("order", [3, 4])
def test_linear_weights_give_the_component_wise_result(ndim, order):
    rng = np.random.default_rng(2 + ndim + order)
    for _ in range(5):
        blk = rand_block(rng, ndim, jump=True)
        W1 = oracle.recon_block(cfg(ndim, order, linear=True), blk)
        W0 = oracle.recon_block(cfg(ndim, order, linear=True, characteristic=False), blk)
        np.testing.assert_allclose(W1, W0, rtol=0, atol=1e-12 * np.abs(W0).max())
        # and with nonlinear weights at a jump it is a different reconstruction
        Wn = oracle.recon_block(cfg(ndim, order), blk)
        Wc = oracle.recon_block(cfg(ndim, order, characteristic=False), blk)
        assert np.abs(Wn - Wc).max() > 1e-6


def _zone_avg_poly(coef, m):
    # average over [m - 1/2, m + 1/2] of sum_k coef[k] x^k (k <= 2), exact
    lo, hi = m - 0.5, m + 0.5
    return sum(cf * (hi ** (k + 1) - lo ** (k + 1)) / (k + 1) for k, cf in enumerate(coef))


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("order", [3, 4])
def test_quadratic_data_are_reproduced_for_any_weights(ndim, order):
    # every candidate is exact on quadratics, in every field: the result is
    # the data's own modes whatever the nonlinear weights are
    rng = np.random.default_rng(20 + ndim)
    nv = ndim + 2
    mod = oracle.modes(ndim, order - 1)
    spatial = [tuple(r[:3]) for r in mod if r[3] == 0]
    for _ in range(3):
        # per variable a separable-sum quadratic: c0 + sum_d (a_d x_d + b_d x_d^2) + cross x*y
        base = np.array([1.0, 0.2, -0.1, 0.1, 2.5][:nv - 1] + [2.5])
        co = rng.normal(scale=0.05, size=(nv, ndim, 2))
        cr = rng.normal(scale=0.05, size=nv)
        nzb = 5 if ndim == 3 else 1
        blk = np.zeros((nv, nzb, 5, 5))
        for v in range(nv):
            for z in range(nzb):
                for y in range(5):
                    for x in range(5):
                        pos = [x - 2, y - 2, z - 2][:ndim]
                        val = base[v]
                        for d in range(ndim):
                            val += _zone_avg_poly([0.0, co[v, d, 0], co[v, d, 1]], pos[d])
                        val += cr[v] * pos[0] * pos[1]      # zone average of x*y is the product of centres
                        blk[v, z, y, x] = val
        blk = np.ascontiguousarray(blk if ndim == 3 else blk[:, 0])
        W = oracle.recon_block(cfg(ndim, order), blk)
        # expected undivided Legendre modes: x -> P1 coefficient a, x^2 -> P2 coefficient b
        for k, (a, b, c3) in enumerate(spatial):
            deg = (a, b, c3)[:ndim]
            for v in range(nv):
                if sum(deg) == 0:
                    exp = blk[(v, 2, 2, 2) if ndim == 3 else (v, 2, 2)]
                elif sum(deg) == 1:
                    exp = co[v, int(np.argmax(deg)), 0]
                elif sum(deg) == 2 and max(deg) == 2:
                    exp = co[v, int(np.argmax(deg)), 1]
                elif sum(deg) == 2 and deg[0] == 1 and deg[1] == 1:
                    exp = cr[v]
                else:
                    exp = 0.0
                assert abs(W[k, v] - exp) <= 1e-12, (k, v, W[k, v], exp)


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("order", [3, 4])
def test_entropy_wave_takes_the_density_weights_in_every_variable(ndim, order):
    # density jumps at constant velocity and pressure: the jump lies along the
    # entropy eigenvector (1, u, |u|^2 / 2), so the momentum and energy modes
    # are the density modes times u and |u|^2 / 2
    rng = np.random.default_rng(30 + ndim)
    vel = np.array([0.3, -0.2, 0.15][:ndim])
    nzb = 5 if ndim == 3 else 1
    for _ in range(4):
        rho = rng.uniform(0.5, 1.5, (nzb, 5, 5))
        rho[..., 3:] *= 5.0
        rho[..., 2:, :] *= 0.3
        U = np.stack([rho, *(rho * v for v in vel), 1.0 / (G - 1) + 0.5 * rho * (vel @ vel)])
        blk = np.ascontiguousarray(U if ndim == 3 else U[:, 0])
        W = oracle.recon_block(cfg(ndim, order), blk)
        for d in range(ndim):
            np.testing.assert_allclose(W[1:, 1 + d], vel[d] * W[1:, 0], rtol=0, atol=1e-12 * np.abs(W[1:, 0]).max())
        np.testing.assert_allclose(W[1:, -1], 0.5 * (vel @ vel) * W[1:, 0], rtol=0,
                                   atol=1e-12 * np.abs(W[1:, 0]).max())


@pytest.mark.parametrize("ndim", [2, 3])
def test_a_problem_along_y_is_the_problem_along_x(ndim):
    rng = np.random.default_rng(40)
    c = cfg(ndim)
    nv = ndim + 2
    line = rand_block(rng, 2, jump=True)[:, 2, :]           # (4, 5) primitive-based line along x
    rho, m1, m2, E = line
    U1 = np.zeros((nv, 5))
    U1[0], U1[1], U1[2], U1[-1] = rho, m1, m2, E
    nzb = 5 if ndim == 3 else 1
    bx = np.broadcast_to(U1[:, None, None, :], (nv, nzb, 5, 5)).copy()
    # the same data along y, with the first two momenta swapped
    Uy = U1.copy()
    Uy[[1, 2]] = U1[[2, 1]]
    by = np.broadcast_to(Uy[:, None, :, None], (nv, nzb, 5, 5)).copy()
    if ndim == 2:
        bx, by = bx[:, 0].copy(), by[:, 0].copy()
    Wx = oracle.recon_block(c, bx)
    Wy = oracle.recon_block(c, by)
    m = [tuple(r) for r in oracle.modes(ndim, 3) if r[3] == 0]
    perm = list(range(nv))
    perm[1], perm[2] = 2, 1
    for i, (a, b, cc, e) in enumerate(m):
        j = m.index((b, a, cc, e))
        np.testing.assert_allclose(Wy[j], Wx[i][perm], rtol=1e-13, atol=1e-14)


def test_scheme_with_characteristic_reconstruction_conserves():
    pb = icgen.random_smooth(n=(9, 8, 7), ndim=3, seed=4, amp=0.2)
    c = oracle.cfg_from_problem(pb, 4, characteristic=True)
    dt, _ = oracle.cfl_dt(c, pb.U)
    U = oracle.step(c, pb.U, dt)
    tot0, tot1 = pb.U.sum(axis=(1, 2, 3)), U.sum(axis=(1, 2, 3))
    assert (np.abs(tot1 - tot0) / np.abs(pb.U).sum(axis=(1, 2, 3))).max() < 1e-14
    Uc = oracle.step(oracle.cfg_from_problem(pb, 4), pb.U, dt)
    assert np.abs(U - Uc).max() > 1e-12       # the option does change the step


@pytest.mark.parametrize("order", [3, 4])
def test_sod_with_characteristic_reconstruction(order):
    from exact_riemann import zone_average_density
    n, t_end = 100, 0.2
    pb = icgen.sod(n=n, axis=0, ndim=2, ntrans=2)
    c = oracle.cfg_from_problem(pb, order, characteristic=True)
    U, t, _ = oracle.run(c, pb.U, t_end=t_end)
    exact = zone_average_density((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), n, t)
    num = U[0, 0]
    l1 = np.abs(num - exact).mean()
    assert l1 < 6e-3, l1
    assert num.max() < 1.0 + 2e-2 and num.min() > 0.125 - 2e-2
    np.testing.assert_allclose(U[:, 1], U[:, 0], rtol=0, atol=1e-15)


@pytest.mark.slow
def test_vortex_design_order_with_characteristic_reconstruction():
    errs = []
    for n in (32, 64):
        pb = icgen.vortex2d(n)
        c = oracle.cfg_from_problem(pb, 4, characteristic=True)
        U, t, _ = oracle.run(c, pb.U, t_end=1.0)
        errs.append(np.abs(U[0] - icgen.vortex_exact_density(n, t)).mean())
    order = np.log2(errs[0] / errs[1])
    assert order >= 3.75, (errs, order)

"""Pins of the oracle's 1D WENO operator and multi-D reconstruction.

Candidates are rebuilt here from their definition (reproduce the zone
averages of their stencil, solved with numpy), smoothness indicators from
their definition (integral of squared derivatives, by numpy quadrature), and
exactness is checked on polynomial data whose zone averages are integrated
numerically.
"""
import numpy as np
import numpy.polynomial.legendre as npl
import numpy.polynomial.polynomial as npp
import pytest

import oracle

XG, WG = npl.leggauss(10)
XG, WG = XG / 2, WG / 2

# Monic Legendre basis on [-1/2, 1/2] as numpy power-series coefficient arrays,
# built here by Gram-Schmidt of monomials (independent of the oracle's formulas).
def _legendre_basis(n=5):
    basis = []
    for k in range(n):
        c = np.zeros(n)
        c[k] = 1.0
        for b in basis:
            ip = np.sum(WG * npp.polyval(XG, c) * npp.polyval(XG, b))
            nb = np.sum(WG * npp.polyval(XG, b) ** 2)
            c = c - ip / nb * np.pad(b, (0, n - len(b)))
        basis.append(c)
    return basis


BASIS = _legendre_basis()


def zone_avg(coeffs, m):
    """Average over zone [m-1/2, m+1/2] of the polynomial with power coeffs."""
    return np.sum(WG * npp.polyval(XG + m, coeffs))


def candidate(v5, offsets, deg):
    """Legendre coefficients c1..deg of the polynomial reproducing the averages on offsets."""
    A = np.array([[zone_avg(BASIS[k], m) for k in range(deg + 1)] for m in offsets])
    rhs = np.array([v5[m + 2] for m in offsets])
    return np.linalg.solve(A, rhs)


def smoothness(c):
    """sum_{l>=1} int (d^l p)^2 of p = sum_k c_k P_k."""
    poly = sum(ck * np.pad(BASIS[k], (0, 5 - len(BASIS[k]))) for k, ck in enumerate(c))
    s = 0.0
    d = poly
    for _ in range(len(c) - 1):
        d = npp.polyder(d)
        s += np.sum(WG * npp.polyval(XG, d) ** 2)
    return s


def weno_definition(v5, p, g3=oracle.DEFAULT_G3, g4=oracle.DEFAULT_G4, eps=1e-12, linear=False):
    cL = candidate(v5, [-2, -1, 0], 2)
    cC = candidate(v5, [-1, 0, 1], 2)
    cR = candidate(v5, [0, 1, 2], 2)
    cands = [cL, cC, cR]
    if p == 2:
        IS = [smoothness(c) for c in cands]
        a = np.array([g / (eps + s) ** 2 for g, s in zip(g3, IS)])
        w = np.array(g3) if linear else a / a.sum()
        return sum(wk * c[1:] for wk, c in zip(w, cands))
    quart = candidate(v5, [-2, -1, 0, 1, 2], 4)
    cH = quart[:4]
    IS = [smoothness(cH)] + [smoothness(c) for c in cands]
    gam = np.array(g4)
    a = gam / (eps + np.array(IS)) ** 2
    w = gam if linear else a / a.sum()
    pad = [np.append(c, 0.0) for c in cands]
    out = w[0] / gam[0] * (cH - gam[1] * pad[0] - gam[2] * pad[1] - gam[3] * pad[2])
    out = out + w[1] * pad[0] + w[2] * pad[1] + w[3] * pad[2]
    return out[1:]


def cfg(ndim=2, order=3, linear=False):
    return oracle.make_cfg(ndim, (8, 8, 8), order, (0.1, 0.1, 0.1), linear_weno=linear)


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("linear", [False, True])
def test_weno1d_matches_its_definition(p, linear):
    rng = np.random.default_rng(10 + p)
    c = cfg(order=p + 1, linear=linear)
    for trial in range(40):
        scale = 10.0 ** rng.uniform(-3, 1)
        v5 = rng.normal(size=5) * scale + rng.normal()
        if trial % 4 == 0:  # a jump somewhere in the stencil
            v5[rng.integers(0, 5):] += rng.choice([-1, 1]) * 5 * scale
        got = oracle.weno1d(c, p, v5)[1:p + 1]
        ref = weno_definition(v5, p, linear=linear)
        np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-12 * (1 + np.abs(v5).max()))


@pytest.mark.parametrize("p", [2, 3])
def test_weno1d_exact_on_quadratic_data_for_any_weights(p):
    rng = np.random.default_rng(20 + p)
    c = cfg(order=p + 1)
    for _ in range(10):
        al = rng.normal(size=3)  # Legendre coefficients c0..c2 of a quadratic
        poly = sum(al[k] * np.pad(BASIS[k], (0, 5 - len(BASIS[k]))) for k in range(3))
        v5 = np.array([zone_avg(poly, m) for m in range(-2, 3)])
        got = oracle.weno1d(c, p, v5)
        np.testing.assert_allclose(got[1:3], al[1:3], atol=1e-13)
        if p == 3:
            assert abs(got[3]) < 1e-13


def test_weno_ao_linear_weights_give_the_high_member_exactly():
    # cubic data with omega = gamma: c = c^H, i.e. exact cubic coefficients
    rng = np.random.default_rng(3)
    c = cfg(order=4, linear=True)
    for _ in range(10):
        al = rng.normal(size=4)
        poly = sum(al[k] * np.pad(BASIS[k], (0, 5 - len(BASIS[k]))) for k in range(4))
        v5 = np.array([zone_avg(poly, m) for m in range(-2, 3)])
        np.testing.assert_allclose(oracle.weno1d(c, 3, v5)[1:4], al[1:4], atol=1e-13)


def test_constant_line_gives_linear_weights_and_zero_slopes():
    for p in (2, 3):
        c = cfg(order=p + 1)
        out = oracle.weno1d(c, p, np.full(5, 3.7))
        assert np.abs(out).max() <= 4 * 2.2e-16 * 3.7


@pytest.mark.parametrize("p", [2, 3])
def test_jump_suppresses_the_candidates_that_cross_it(p):
    # jump between v0 and v1: only the left quadratic is smooth, the result
    # tends to it (zero slope of the constant left data)
    c = cfg(order=p + 1)
    v5 = np.array([1.0, 1.0, 1.0, 2.0, 2.0])
    out = oracle.weno1d(c, p, v5)
    assert np.abs(out).max() < 1e-6
    # mirror: jump between v-1 and v0 -> right candidate
    out = oracle.weno1d(c, p, v5[::-1].copy())
    assert np.abs(out).max() < 1e-6


def _poly_block(ndim, alpha, p_deg):
    """Zone averages on the 5^d block of sum alpha[a,b,c] P_a P_b P_c (total deg <= p_deg)."""
    nb = 5
    oned = np.array([[zone_avg(np.pad(BASIS[k], (0, 5 - len(BASIS[k]))), m) for m in range(-2, 3)]
                     for k in range(4)])  # oned[k, m] = <P_k>(m)
    if ndim == 2:
        blk = np.zeros((nb, nb))
        for a in range(p_deg + 1):
            for b in range(p_deg + 1 - a):
                blk += alpha[a, b, 0] * np.outer(oned[b], oned[a])
        return blk
    blk = np.zeros((nb, nb, nb))
    for a in range(p_deg + 1):
        for b in range(p_deg + 1 - a):
            for cc in range(p_deg + 1 - a - b):
                blk += alpha[a, b, cc] * np.einsum("z,y,x->zyx", oned[cc], oned[b], oned[a])
    return blk


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("order,deg,linear", [(3, 2, False), (4, 2, False), (4, 3, True)])
def test_multid_reconstruction_reproduces_polynomials(ndim, order, deg, linear):
    rng = np.random.default_rng(100 * ndim + 10 * order + deg)
    c = cfg(ndim=ndim, order=order, linear=linear)
    m = oracle.modes(ndim, order - 1)
    spatial = m[m[:, 3] == 0]
    nv = ndim + 2
    alpha = np.zeros((nv, 4, 4, 4))
    for v in range(nv):
        for a in range(deg + 1):
            for b in range(deg + 1 - a):
                for cc in range(deg + 1 - a - b if ndim == 3 else 1):
                    alpha[v, a, b, cc] = rng.normal()
    blk = np.stack([_poly_block(ndim, alpha[v], deg) for v in range(nv)])
    W = oracle.recon_block(c, blk)
    ref = np.array([[alpha[v, a, b, cc] for v in range(nv)] for a, b, cc, _ in spatial])
    np.testing.assert_allclose(W, ref, atol=2e-12)


@pytest.mark.parametrize("linear", [False, True])
def test_reconstruction_is_symmetric_under_axis_swap(linear):
    # Pure x / y modes come from one 1D application each and must swap exactly;
    # mixed modes depend on the sweep order unless the weights are linear.
    rng = np.random.default_rng(7)
    c = cfg(ndim=2, order=4, linear=linear)
    blk = rng.normal(size=(4, 5, 5)) + 2.0
    blk2 = blk.transpose(0, 2, 1)[[0, 2, 1, 3]].copy()   # swap x, y and the momenta
    W1 = oracle.recon_block(c, blk)
    W2 = oracle.recon_block(c, blk2)
    m = [tuple(r) for r in oracle.modes(2, 3)[:10]]
    for i, (a, b, cc, e) in enumerate(m):
        if a and b and not linear:
            continue
        j = m.index((b, a, cc, e))
        np.testing.assert_allclose(W2[j], W1[i][[0, 2, 1, 3]], rtol=1e-13, atol=1e-14)

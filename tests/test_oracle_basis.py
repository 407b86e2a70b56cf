"""Pins of the oracle's bases, quadrature and mode lists against closed forms
and numpy's polynomial routines (no GPU)."""
import math

import numpy as np
import numpy.polynomial.legendre as npl
import numpy.polynomial.polynomial as npp
import pytest

import oracle

XG, WG = npl.leggauss(12)
XG, WG = XG / 2, WG / 2            # exact for degree <= 23 on [-1/2, 1/2]
TG = XG + 0.5                      # same rule on [0, 1]


@pytest.mark.parametrize("n", [2, 3, 4])
def test_gauss_rule_matches_numpy_and_is_exact(n):
    x, w = oracle.gauss(n)
    xr, wr = npl.leggauss(n)
    np.testing.assert_allclose(x, xr / 2, rtol=0, atol=2e-16)
    np.testing.assert_allclose(w, wr / 2, rtol=0, atol=2e-16)
    for k in range(2 * n):
        exact = ((0.5) ** (k + 1) - (-0.5) ** (k + 1)) / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-16


def test_legendre_basis_orthogonal_zero_mean_and_norms():
    P = np.array([[oracle.leg(a, x) for x in XG] for a in range(4)])
    G = (P * WG) @ P.T
    np.testing.assert_allclose(G, np.diag([1, 1 / 12, 1 / 180, 1 / 2800]), atol=1e-16)
    # monic of degree a: numpy fit recovers leading coefficient 1
    for a in range(4):
        c = npp.polyfit(XG, P[a], a)
        assert abs(c[a] - 1.0) < 1e-12


def test_shifted_legendre_time_basis_matches_numpy():
    for e in range(4):
        ref = npl.legval(2 * TG - 1, [0] * e + [1])
        got = np.array([oracle.sleg(e, t) for t in TG])
        np.testing.assert_allclose(got, ref, atol=1e-13)
        assert abs(np.sum(WG * got * got) - 1 / (2 * e + 1)) < 1e-14


def test_derivative_map_of_legendre_basis():
    rng = np.random.default_rng(0)
    xs = rng.uniform(-0.5, 0.5, 7)
    for a in range(1, 4):
        # derivative by numpy of the monic polynomial, vs sum dleg(a,a') P_a'
        coeffs = npp.polyfit(XG, [oracle.leg(a, x) for x in XG], a)
        der = npp.polyval(xs, npp.polyder(coeffs))
        got = np.array([sum(oracle.dleg(a, ap) * oracle.leg(ap, x) for ap in range(a)) for x in xs])
        np.testing.assert_allclose(got, der, atol=1e-13)


def test_time_integral_map():
    rng = np.random.default_rng(1)
    for e in range(4):
        for tau in rng.uniform(0, 1, 5):
            # int_0^tau of the numpy shifted Legendre polynomial, by Gauss on [0, tau]
            xs = (XG + 0.5) * tau
            ref = tau * np.sum(WG * npl.legval(2 * xs - 1, [0] * e + [1]))
            got = sum(oracle.tint(e, ep) * tau ** ep for ep in range(1, e + 2))
            assert abs(got - ref) < 1e-14


@pytest.mark.parametrize("ndim,p", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_mode_counts_and_order(ndim, p):
    m = oracle.modes(ndim, p)
    assert len(m) == math.comb(p + ndim + 1, ndim + 1)
    spatial = m[m[:, 3] == 0]
    assert len(spatial) == math.comb(p + ndim, ndim)
    # spatial block first, mean first, all total degrees <= p, no duplicates
    assert (m[: len(spatial), 3] == 0).all()
    assert tuple(m[0]) == (0, 0, 0, 0)
    assert (m.sum(axis=1) <= p).all()
    assert len({tuple(r) for r in m}) == len(m)
    if ndim == 2:
        assert (m[:, 2] == 0).all()

"""Pins of the CPU reference of the learned gate and of the oracle's gated
reconstruction (no GPU)."""
import numpy as np
import pytest

import icgen
import oracle
from oracle import gate


def test_bf16_rounding_ties_to_even():
    one = 1.0
    assert gate.bf16(one) == 1.0
    assert gate.bf16(1 + 2 ** -8) == 1.0                 # halfway, even mantissa kept
    assert gate.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6     # halfway, rounds to even (up)
    assert gate.bf16(1 + 2 ** -8 + 2 ** -12) == 1 + 2 ** -7
    assert gate.bf16(-3.0) == -3.0


def test_features_of_constant_and_linear_fields():
    pb = icgen.uniform(n=(6, 5, 4), ndim=3)
    F = gate.features(pb.U, 3, pb.bc)
    assert F.shape == (6 * 5 * 4, 65) and np.abs(F).max() == 0.0
    # density linear in x on an outflow box: x entries of the cross are
    # (-2, -1, 1, 2) / 4 away from the boundary, y/z entries 0
    U = pb.U.copy()
    U[0] = 1.0 + 0.1 * np.arange(6)[None, None, :]
    F = gate.features(U, 3, ("outflow",) * 3).reshape(4, 5, 6, 5, 13)
    np.testing.assert_allclose(F[1, 2, 2, 0, 1:5], [-0.5, -0.25, 0.25, 0.5], atol=1e-12)
    assert np.abs(F[1, 2, 2, 0, 5:]).max() == 0.0


def test_features_are_shift_and_scale_invariant():
    pb = icgen.random_smooth(n=(7, 6, 5), ndim=3, seed=4)
    F1 = gate.features(pb.U, 3, pb.bc)
    F2 = gate.features(3.0 * pb.U + 7.0, 3, pb.bc)
    np.testing.assert_allclose(F1, F2, atol=1e-9)


def test_analytic_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    nf = 36
    P = gate.init_params(nf, seed=1)
    P = {k: v.astype(np.float64) for k, v in P.items()}
    P["b1"] += 0.1
    P["b2"] += 0.05
    X = rng.normal(size=(32, nf))
    y = (rng.uniform(size=32) < 0.5).astype(float)
    cw = np.where(y > 0, 0.7, 1.3)
    L, g = gate.loss_and_grads(P, X, y, cw, rounding=False)
    for k in ("W1", "b1", "W2", "b2", "w3", "b3"):
        flat = P[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            h = 1e-6
            old = flat[idx]
            flat[idx] = old + h
            Lp, _ = gate.loss_and_grads(P, X, y, cw, rounding=False)
            flat[idx] = old - h
            Lm, _ = gate.loss_and_grads(P, X, y, cw, rounding=False)
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx)


def test_training_reference_learns_a_separable_rule():
    rng = np.random.default_rng(3)
    nf = 36
    X = rng.normal(size=(2048, nf))
    y = (X[:, 3] + 0.5 * X[:, 7] > 0).astype(float)
    P = gate.init_params(nf, seed=2)
    st = {}
    cw = np.ones_like(y)
    L0, _ = gate.loss_and_grads(P, X, y, cw)
    for _ in range(150):
        _, g = gate.loss_and_grads(P, X, y, cw)
        P = gate.adam(P, g, st, lr=3e-3)
    L1, _ = gate.loss_and_grads(P, X, y, cw)
    logit, _ = gate.forward(P, X)
    acc = np.mean((logit > 0) == (y > 0))
    assert L1 < 0.5 * L0 and acc > 0.9


def test_maxdev_zero_on_constant_and_large_at_a_jump():
    pb = icgen.uniform(n=(6, 6, 6), ndim=3)
    c = oracle.cfg_from_problem(pb, 4)
    assert oracle.zone_maxdev(c, pb.U).max() < 1e-12
    sod = icgen.sod(n=16, axis=0, ndim=3, ntrans=3)
    c = oracle.cfg_from_problem(sod, 4)
    d = oracle.zone_maxdev(c, sod.U)
    assert d[1, 1, 7] > 0.25 and d[1, 1, 8] > 0.25 and d[1, 1, 2] < 1e-12


@pytest.mark.parametrize("ndim,order", [(2, 3), (3, 4)])
def test_gated_step_limits(ndim, order):
    pb = icgen.random_smooth(n=(9, 8, 7), ndim=ndim, seed=2, amp=0.3)
    c = oracle.cfg_from_problem(pb, order)
    dt, _ = oracle.cfl_dt(c, pb.U)
    zeros = np.zeros(pb.U[0].shape, np.uint8)
    U0, _ = oracle.step_gated(c, pb.U, dt, zeros)
    np.testing.assert_array_equal(U0, oracle.step(c, pb.U, dt))
    U1, _ = oracle.step_gated(c, pb.U, dt, np.ones_like(zeros))
    lin = oracle.cfg_from_problem(pb, order, linear_weno=True)
    # applications centred outside the interior keep nonlinear weights, so only
    # zones away from the periodic seam equal the all-linear step
    Ul = oracle.step(lin, pb.U, dt)
    core = (slice(None),) + (slice(4, -4),) * ndim
    np.testing.assert_allclose(U1[core], Ul[core], rtol=0, atol=1e-15 * np.abs(Ul).max())
    # one flagged zone changes only zones within its dependence radius
    one = zeros.copy()
    idx = (3, 4, 4) if ndim == 3 else (4, 4)
    one[idx] = 1
    Ug, _ = oracle.step_gated(c, pb.U, dt, one)
    diff = np.abs(Ug - U0).max(axis=0)
    changed = np.argwhere(diff > 0)
    assert len(changed) > 0
    assert np.abs(changed - np.array(idx)).max() <= 3

"""Parity of the Runge-Kutta steppers on gfx950 (two-, three- and five-stage
SSP schemes with the same reconstruction and Riemann solver, Table IV) with
the oracle's, through the C ABI.  Same bar as the ADER step: relative L1 <=
1e-12 and element-wise 1e-12 relative; fallback counts summed over the stages
must match."""
import numpy as np
import pytest

import icgen
import oracle
from tests.test_gpu_parity import REL_L1, note, rel_l1

pytestmark = pytest.mark.gpu

PAIRS = [(2, "rk2"), (3, "rk3"), (4, "rk4")]


@pytest.fixture(scope="module")
def hog():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_13295_amd import hog as h
    h.load()
    return h


def _check_step(hog, pb, order, stepper, riemann="hllc"):
    g = hog.Grid.from_problem(pb, order, riemann=riemann, stepper=stepper)
    c = oracle.cfg_from_problem(pb, order, riemann=riemann, stepper=stepper)
    dt, bad = oracle.cfl_dt(c, pb.U)
    assert bad < 0
    dt_next = g.step(dt)
    U = g.get_state()
    Uo, nbo = oracle.step_count(c, pb.U, dt)
    assert rel_l1(U, Uo) <= REL_L1
    np.testing.assert_allclose(U, Uo, rtol=1e-12, atol=1e-13 * np.abs(Uo).max())
    dto, _ = oracle.cfl_dt(c, Uo)
    assert abs(dt_next - dto) <= 1e-13 * dto
    assert g.stats()["fallback_zones"] == nbo
    g.close()
    return nbo


@pytest.mark.parametrize("order,stepper", PAIRS)
@pytest.mark.parametrize("bc", ["periodic", "outflow"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_rk_one_step_matches_oracle(hog, ndim, bc, order, stepper):
    n = (17, 11, 9) if ndim == 3 else (37, 29, 1)
    note(f"RK one step ndim={ndim} bc={bc} order={order} {stepper}")
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=30 + order, amp=0.3, bc=bc, h=(0.1, 0.08, 0.11))
    _check_step(hog, pb, order, stepper)


@pytest.mark.parametrize("stepper", ["rk2", "rk4"])
@pytest.mark.parametrize("riemann", ["hll", "rusanov", "hllem", "hlli"])
def test_rk_other_pairings_and_solvers(hog, stepper, riemann):
    """Steppers are independent of the order: third order with two and five
    stages, HLL and Rusanov."""
    note(f"RK third order {stepper} {riemann}")
    pb = icgen.random_smooth(n=(13, 10, 7), ndim=3, seed=5, amp=0.3, bc="outflow", h=(0.1, 0.08, 0.11))
    _check_step(hog, pb, 3, stepper, riemann)


def test_rk_second_order_fused_stages_match_oracle(hog):
    """Second order: each stage is the fused kernel without the time mode; grids
    spanning several tiles and march chunks with ragged ends."""
    for n, ndim in [((37, 30, 21), 3), ((600, 45, 1), 2)]:
        note(f"RK2 second order n={n}")
        pb = icgen.random_smooth(n=n, ndim=ndim, seed=7, amp=0.4, bc="periodic", h=(0.1, 0.08, 0.11))
        _check_step(hog, pb, 2, "rk2", "hll")
        _check_step(hog, pb, 2, "rk4", "hllc")


@pytest.mark.parametrize("order,stepper", [(4, "rk4"), (2, "rk2")])
def test_rk_fallback_matches_oracle(hog, order, stepper):
    """Multi-blast (fourth order) and the cold flow (second order): equal
    fallback counts over the stages and equal states."""
    if order == 4:
        note("RK4 fourth order multiblast 20^3")
        pb = icgen.multiblast(n=20, seed=3)
    else:
        note("RK2 second order cold wave 3D 16^3")
        pb = icgen.cold_wave(n=16, ndim=3)
    assert _check_step(hog, pb, order, stepper, "hll") > 0


def test_rk_runs_match_oracle(hog):
    note("RK3 O3 vortex2d 64^2 x20")
    pb = icgen.vortex2d(64)
    g = hog.Grid.from_problem(pb, 3, stepper="rk3")
    t = g.advance(20)
    c = oracle.cfg_from_problem(pb, 3, stepper="rk3")
    Uo, to, _ = oracle.run(c, pb.U, nsteps=20)
    assert abs(t - to) <= 1e-13 * to
    assert rel_l1(g.get_state(), Uo) <= REL_L1
    g.close()
    note("RK4 O4 vortex3d_perturbed 20^3 x3")
    pb = icgen.vortex3d_perturbed(n=20, seed=2)
    g = hog.Grid.from_problem(pb, 4, stepper="rk4")
    t = g.advance(3)
    c = oracle.cfg_from_problem(pb, 4, stepper="rk4")
    Uo, to, _ = oracle.run(c, pb.U, nsteps=3)
    assert abs(t - to) <= 1e-13 * to
    assert rel_l1(g.get_state(), Uo) <= REL_L1
    g.close()
    note("RK3 O3 sod along z to t = 0.05")
    pb = icgen.sod(n=64, axis=2, ndim=3, ntrans=3)
    g = hog.Grid.from_problem(pb, 3, stepper="rk3")
    t = g.advance(100000, t_end=0.05)
    c = oracle.cfg_from_problem(pb, 3, stepper="rk3")
    Uo, to, _ = oracle.run(c, pb.U, t_end=0.05)
    assert abs(t - to) <= 1e-12
    assert rel_l1(g.get_state(), Uo) <= REL_L1
    g.close()


@pytest.mark.parametrize("ndim,n,bc", [(3, (1, 1, 1), "outflow"), (3, (3, 3, 3), "periodic"),
                                       (2, (1, 6, 1), "outflow"), (3, (2, 3, 1), "outflow")])
def test_rk_degenerate_grids_match_oracle(hog, ndim, n, bc):
    note(f"RK degenerate grid {n}")
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=sum(n) + 9, amp=0.3, bc=bc, h=(0.1, 0.08, 0.11))
    for order, stepper in PAIRS:
        _check_step(hog, pb, order, stepper)


def test_rk_larger_grid_and_conservation(hog):
    """48^3 fourth order, five stages, periodic: the whole grid against the
    oracle, and conservation to rounding."""
    note("RK4 O4 48^3 one step")
    pb = icgen.vortex3d_perturbed(n=48, seed=2)
    _check_step(hog, pb, 4, "rk4")
    g = hog.Grid.from_problem(pb, 4, stepper="rk4")
    g.advance(2)
    U = g.get_state()
    g.close()
    tot0, tot1 = pb.U.sum(axis=(1, 2, 3)), U.sum(axis=(1, 2, 3))
    assert (np.abs(tot1 - tot0) / np.maximum(np.abs(pb.U).sum(axis=(1, 2, 3)), 1.0)).max() < 1e-13


def test_rk_rejects_what_it_does_not_run(hog):
    pb = icgen.uniform(n=(6, 6, 6), ndim=3)
    for kw in ({"precision": "mixed"}, {"debug": True}):
        with pytest.raises(hog.HogError) as e:
            hog.Grid.from_problem(pb, 4, stepper="rk3", **kw)
        assert e.value.code == hog.HOG_EINVAL
    g = hog.Grid.from_problem(pb, 4, stepper="rk3")
    with pytest.raises(hog.HogError) as e:
        g.set_gate_flags(np.zeros((6, 6, 6), dtype=np.uint8))
    assert e.value.code == hog.HOG_EINVAL
    g.close()


def test_rk_full_size_first_step_sampled(hog):
    """128^3 fourth-order five-stage step of the 3D workload in the benchmark's
    launch configuration.  A Runge-Kutta zone depends on the zones within 3 per
    stage (reconstruction radius 2 plus the face neighbour), 15 for five stages:
    the oracle computes each sampled zone on the periodic cut-out of half-width
    20 around it (outflow at the cut, 5 zones beyond the reach)."""
    note("RK4 O4 vortex3d_perturbed 128^3 first step, sampled")
    n, r = 128, 20
    pb = icgen.vortex3d_perturbed(n=n, seed=2)
    g = hog.Grid.from_problem(pb, 4, stepper="rk4")
    c = oracle.cfg_from_problem(pb, 4, stepper="rk4")
    dt, _ = oracle.cfl_dt(c, pb.U)
    g.step(dt)
    U = g.get_state()
    g.close()
    rng = np.random.default_rng(3)
    pts = np.vstack([rng.integers(0, n, size=(3, 3)), [[0, 0, 0], [127, 64, 1]]])
    m = 2 * r + 1
    cut = oracle.make_cfg(3, (m, m, m), 4, pb.h, gamma=pb.gamma, bc=("outflow",) * 3, stepper="rk4")
    for i, j, k in pts:
        ix = [(i + d) % n for d in range(-r, r + 1)]
        jx = [(j + d) % n for d in range(-r, r + 1)]
        kx = [(k + d) % n for d in range(-r, r + 1)]
        sub = pb.U[:, kx][:, :, jx][:, :, :, ix]
        ref = oracle.step(cut, sub, dt)[:, r, r, r]
        np.testing.assert_allclose(U[:, k, j, i], ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())

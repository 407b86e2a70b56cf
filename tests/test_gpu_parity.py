"""Parity of the gfx950 HIP path with the FP64 CPU oracle, through the C ABI.

Bar for the FP64 path: relative L1 difference sum|gpu - oracle| / sum|oracle|
over all variables <= 1e-12 (the target of the FP64 path), element-wise
checks where stated.  Inputs are seeded synthetic states from ``icgen``; no
oracle input and no expected value comes from the GPU.
"""
import sys

import numpy as np
import pytest

import icgen
import oracle

pytestmark = pytest.mark.gpu

REL_L1 = 1e-12


@pytest.fixture(scope="module")
def hog():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_13295_amd import hog as h
    h.load()
    return h


def rel_l1(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def grid_for(hog, pb, order, **kw):
    return hog.Grid.from_problem(pb, order, **kw)


# ---------------------------------------------------------------- state I/O
def test_set_get_roundtrip_is_bitwise(hog):
    import torch
    pb = icgen.random_smooth(n=(13, 7, 5), ndim=3, seed=1)
    g = grid_for(hog, pb, 4)
    np.testing.assert_array_equal(g.get_state(), pb.U)
    aos = np.ascontiguousarray(np.moveaxis(pb.U, 0, -1))
    g.set_state(aos, layout=hog.AOS)
    np.testing.assert_array_equal(g.get_state(layout=hog.AOS), aos)
    np.testing.assert_array_equal(g.get_state(), pb.U)
    dev = torch.from_numpy(pb.U * 2.0).cuda()
    g.set_state(dev)
    out = torch.empty_like(dev)
    g.get_state_device(out)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), pb.U * 2.0)


@pytest.mark.parametrize("ndim", [2, 3])
def test_cfl_dt_matches_oracle(hog, ndim):
    pb = icgen.random_smooth(n=(11, 9, 6), ndim=ndim, seed=3, h=(0.1, 0.07, 0.13))
    g = grid_for(hog, pb, 4)
    dt_o, _ = oracle.cfl_dt(oracle.cfg_from_problem(pb, 4), pb.U)
    assert abs(g.compute_dt() - dt_o) <= 1e-14 * dt_o


# ---------------------------------------------------------------- stages
CASES = [(2, 3), (2, 4), (3, 3), (3, 4)]


@pytest.mark.parametrize("ndim,order", CASES)
def test_stage_modes_match_oracle(hog, ndim, order):
    note(f"stage taps ndim={ndim} order={order}")
    pb = icgen.random_smooth(n=(9, 8, 7), ndim=ndim, seed=10 + order, amp=0.2, bc="outflow",
                             h=(0.1, 0.12, 0.09))
    g = grid_for(hog, pb, order, debug=True)
    dt = g.compute_dt()
    g.step(dt)
    W = g.tap(hog.TAP_MODES)
    q = g.tap(hog.TAP_STMODES)
    c = oracle.cfg_from_problem(pb, order)
    Wo, qo = oracle.stage_modes(c, pb.U, dt)
    scale = np.abs(Wo).max()
    np.testing.assert_allclose(W, Wo, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(q, qo, rtol=0, atol=1e-13 * scale)


# ---------------------------------------------------------------- one step
@pytest.mark.parametrize("ndim,order", CASES)
@pytest.mark.parametrize("riemann", ["hllc", "hll", "rusanov", "hllem", "hlli"])
@pytest.mark.parametrize("bc", ["periodic", "outflow"])
def test_one_step_matches_oracle(hog, ndim, order, riemann, bc):
    note(f"one step ndim={ndim} order={order} riemann={riemann} bc={bc}")
    n = (17, 11, 9) if ndim == 3 else (37, 29, 1)
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=ndim * order, amp=0.3, bc=bc, h=(0.1, 0.08, 0.11))
    g = grid_for(hog, pb, order, riemann=riemann)
    c = oracle.cfg_from_problem(pb, order, riemann=riemann)
    dt, _ = oracle.cfl_dt(c, pb.U)
    dt_next = g.step(dt)
    U = g.get_state()
    Uo = oracle.step(c, pb.U, dt)
    assert rel_l1(U, Uo) <= REL_L1
    np.testing.assert_allclose(U, Uo, rtol=1e-12, atol=1e-13 * np.abs(Uo).max())
    dto, _ = oracle.cfl_dt(c, Uo)
    assert abs(dt_next - dto) <= 1e-13 * dto


def test_one_step_with_a_shock_matches_oracle(hog):
    """Multi-blast (100:1 pressure jumps, outflow) needs the positivity
    fallback; GPU and oracle must agree on the result and on how many zones
    fell back."""
    note("one step multiblast 24^3")
    pb = icgen.multiblast(n=24, seed=3)
    g = grid_for(hog, pb, 4)
    c = oracle.cfg_from_problem(pb, 4)
    dt, _ = oracle.cfl_dt(c, pb.U)
    g.step(dt)
    U = g.get_state()
    Uo, nbo = oracle.step_count(c, pb.U, dt)
    assert nbo > 0
    assert g.stats()["fallback_zones"] == nbo
    assert rel_l1(U, Uo) <= REL_L1


def test_shock_without_fallback_is_reported(hog):
    pb = icgen.multiblast(n=24, seed=3)
    g = grid_for(hog, pb, 4, positivity=False)
    with pytest.raises(hog.HogError) as e:
        g.step(g.compute_dt())
    assert e.value.code == hog.HOG_ENONPHYS
    np.testing.assert_array_equal(g.get_state(), pb.U)


def test_multiblast_run_matches_oracle(hog):
    note("multiblast 20^3 O4 x3")
    pb = icgen.multiblast(n=20, seed=3)
    g = grid_for(hog, pb, 4)
    t = g.advance(3)
    U = g.get_state()
    c = oracle.cfg_from_problem(pb, 4)
    Uo, to, _ = oracle.run(c, pb.U, nsteps=3)
    assert abs(t - to) <= 1e-13 * to
    assert rel_l1(U, Uo) <= REL_L1


def test_four_quadrant_reduced_matches_oracle(hog):
    note("four-quadrant 24^3 O4 x3")
    pb = icgen.four_quadrant(n=24, seed=5)
    g = grid_for(hog, pb, 4)
    g.advance(3)
    U = g.get_state()
    c = oracle.cfg_from_problem(pb, 4)
    Uo, _, _ = oracle.run(c, pb.U, nsteps=3)
    assert rel_l1(U, Uo) <= REL_L1


# ---------------------------------------------------------------- runs
def test_vortex2d_64_o3_20_steps_matches_oracle(hog):
    """2D isentropic vortex, 64^2, third order, CFL 0.4, 20 steps, HLLC."""
    note("vortex2d 64^2 O3 x20")
    pb = icgen.vortex2d(64)
    g = grid_for(hog, pb, 3)
    t = g.advance(20)
    U = g.get_state()
    c = oracle.cfg_from_problem(pb, 3)
    Uo, to, _ = oracle.run(c, pb.U, nsteps=20)
    assert abs(t - to) <= 1e-13 * to
    assert rel_l1(U, Uo) <= REL_L1
    ex = icgen.vortex_exact_density(64, to)
    e_gpu, e_or = np.abs(U[0] - ex).mean(), np.abs(Uo[0] - ex).mean()
    assert abs(e_gpu - e_or) <= 1e-10 * e_or


def test_vortex3d_perturbed_reduced_matches_oracle(hog):
    """The 3D workload (extruded vortex + seeded density modes, fourth order,
    HLLC) at 20^3 for 4 steps."""
    note("vortex3d_perturbed 20^3 O4 x4")
    pb = icgen.vortex3d_perturbed(n=20, seed=2)
    g = grid_for(hog, pb, 4)
    t = g.advance(4)
    U = g.get_state()
    c = oracle.cfg_from_problem(pb, 4)
    Uo, to, _ = oracle.run(c, pb.U, nsteps=4)
    assert abs(t - to) <= 1e-13 * to
    assert rel_l1(U, Uo) <= REL_L1


@pytest.mark.parametrize("riemann", ["hllc", "hllem", "hlli"])
def test_sod_run_matches_oracle(hog, riemann):
    note(f"sod 3D along z O4 {riemann}")
    pb = icgen.sod(n=64, axis=2, ndim=3, ntrans=3)
    g = grid_for(hog, pb, 4, riemann=riemann)
    t = g.advance(1000, t_end=0.05)
    U = g.get_state()
    c = oracle.cfg_from_problem(pb, 4, riemann=riemann)
    Uo, to, _ = oracle.run(c, pb.U, t_end=0.05)
    assert abs(t - to) <= 1e-12
    assert rel_l1(U, Uo) <= REL_L1


def test_full_size_first_step_sampled(hog):
    """128^3 fourth-order 3D workload, first step from its initial state, in the
    launch configuration of the benchmark; the oracle computes sampled zones
    (interior, faces, edges and corners of the periodic box)."""
    note("vortex3d_perturbed 128^3 first step, sampled")
    pb = icgen.vortex3d_perturbed(n=128, seed=2)
    g = grid_for(hog, pb, 4)
    dt = g.compute_dt()
    c = oracle.cfg_from_problem(pb, 4)
    dto, _ = oracle.cfl_dt(c, pb.U)
    assert abs(dt - dto) <= 1e-14 * dto
    g.step(dto)
    U = g.get_state()
    rng = np.random.default_rng(0)
    pts = rng.integers(0, 128, size=(48, 3))
    pts = np.vstack([pts, [[0, 0, 0], [127, 127, 127], [0, 127, 64], [127, 0, 1], [64, 64, 0]]])
    ref = oracle.step_zones(c, pb.U, dto, pts)
    got = np.stack([U[:, k, j, i] for i, j, k in pts])
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


def _sample_points(n, seed):
    rng = np.random.default_rng(seed)
    pts = rng.integers(0, n, size=(48, 3))
    m = n - 1
    return np.vstack([pts, [[0, 0, 0], [m, m, m], [0, m, n // 2], [m, 0, 1], [n // 2, n // 2, 0]]])


def _full_size_first_step(hog, pb, pts, precision, gate=None):
    import torch
    g = grid_for(hog, pb, 4, precision=precision)
    if gate is not None:
        g.set_gate(gate[0], theta=gate[1])
    c = oracle.cfg_from_problem(pb, 4)
    dto, _ = oracle.cfl_dt(c, pb.U)
    g.step(dto)
    U = g.get_state()
    g.close()
    del g
    torch.cuda.empty_cache()
    got = np.stack([U[:, k, j, i] for i, j, k in pts])
    return got, oracle.step_zones(c, pb.U, dto, pts)


@pytest.mark.parametrize("case", ["multiblast_256", "four_quadrant_384"])
def test_full_size_first_step_sampled_shock_configs(hog, case):
    """The two shock workloads at their full sizes (multi-blast 256^3, outflow;
    four-quadrant Riemann problem 384^3), fourth order, first step from the
    initial state in the benchmark's launch configuration: the FP64 path
    against the oracle element-wise on sampled zones, and the path these
    workloads are quoted on (mixed FP32/FP64; for the four-quadrant problem
    with the trained gate) within the mixed path's shock bound (relative L1
    over the samples against the FP64 oracle)."""
    import os
    if case == "multiblast_256":
        note("multiblast 256^3 first step, sampled")
        pb, n, gate = icgen.multiblast(n=256, seed=3), 256, None
    else:
        note("four-quadrant 384^3 first step, sampled")
        pb, n = icgen.four_quadrant(n=384, seed=5), 384
        z = np.load(os.path.join(os.path.dirname(__file__), "..", "paper_2211_13295_amd", "gate_o4_3d.npz"))
        gate = (z["params"], float(z["theta"]))
    pts = _sample_points(n, 1)
    got, ref = _full_size_first_step(hog, pb, pts, "fp64")
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())
    note(f"{case}: FP64 sampled parity ok")
    got, ref = _full_size_first_step(hog, pb, pts, "mixed", gate)
    e = rel_l1(got, ref)
    note(f"{case}: mixed{' + gate' if gate else ''} sampled relative L1 vs FP64 oracle {e:.3e}")
    assert e <= 1e-3


def test_advance_to_an_end_time_matches_oracle(hog):
    """Device-side time loop with an end time (the last step shortened to land
    on it) against the oracle's loop: same step count, end time and state."""
    note("vortex2d 32^2 O3 advance to t_end = 0.7")
    pb = icgen.vortex2d(n=32)
    c = oracle.cfg_from_problem(pb, 3)
    Uo, to, dts = oracle.run(c, pb.U, t_end=0.7)
    g = grid_for(hog, pb, 3)
    t = g.advance(100000, t_end=0.7)
    assert abs(t - to) <= 1e-14 and abs(t - 0.7) <= 1e-14
    assert rel_l1(g.get_state(), Uo) <= REL_L1


@pytest.mark.parametrize("ndim,order,n,bc", [
    (3, 4, (1, 1, 1), "outflow"), (3, 4, (1, 4, 3), "outflow"), (3, 3, (3, 3, 3), "periodic"),
    (3, 4, (2, 3, 1), "outflow"), (2, 3, (1, 6, 1), "outflow"), (2, 4, (3, 3, 1), "periodic")])
def test_degenerate_grids_match_oracle(hog, ndim, order, n, bc):
    """Grids one to three zones wide (outflow ghosts clamped to a single zone;
    periodic axes at the minimum of three zones, where every stencil wraps
    around the whole axis; partial zone groups in the predictor's
    wavefronts): one step against the oracle.  Periodic axes shorter than
    three zones are rejected by the library (checked without a device in
    test_abi)."""
    note(f"degenerate grid {n} ndim={ndim} order={order} bc={bc}")
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=sum(n) + order, amp=0.3, bc=bc, h=(0.1, 0.08, 0.11))
    g = grid_for(hog, pb, order)
    c = oracle.cfg_from_problem(pb, order)
    dt, _ = oracle.cfl_dt(c, pb.U)
    g.step(dt)
    Uo = oracle.step(c, pb.U, dt)
    np.testing.assert_allclose(g.get_state(), Uo, rtol=1e-12, atol=1e-13 * np.abs(Uo).max())


# ---------------------------------------------------------------- properties
@pytest.mark.parametrize("ndim,order", CASES)
def test_conservation_and_free_stream_on_gpu(hog, ndim, order):
    pb = icgen.random_smooth(n=(12, 10, 8), ndim=ndim, seed=5, amp=0.2)
    g = grid_for(hog, pb, order)
    g.advance(5)
    U = g.get_state()
    ax = tuple(range(1, ndim + 1))
    tot0, tot1 = pb.U.sum(axis=ax), U.sum(axis=ax)
    assert (np.abs(tot1 - tot0) / np.abs(pb.U).sum(axis=ax)).max() < 1e-13
    fs = icgen.uniform(n=(9, 8, 7), ndim=ndim, bc="outflow")
    g2 = grid_for(hog, fs, order)
    g2.advance(3)
    np.testing.assert_allclose(g2.get_state(), fs.U, rtol=1e-14, atol=1e-14)


def test_runs_are_bitwise_deterministic(hog):
    pb = icgen.multiblast(n=20, seed=4)
    outs = []
    for _ in range(2):
        g = grid_for(hog, pb, 4)
        g.advance(3)
        outs.append(g.get_state())
    np.testing.assert_array_equal(outs[0], outs[1])


# ---------------------------------------------------------------- errors
def test_error_paths(hog):
    pb = icgen.uniform(n=(6, 6, 6), ndim=3)
    g = grid_for(hog, pb, 4)
    with pytest.raises(hog.HogError) as e:
        g.step(-1.0)
    assert e.value.code == hog.HOG_EINVAL
    with pytest.raises(hog.HogError) as e:
        g.step(float("nan"))
    assert e.value.code == hog.HOG_EINVAL
    bad = pb.U.copy()
    bad[0, 1, 2, 3] = -1.0
    g.set_state(bad)
    with pytest.raises(hog.HogError) as e:
        g.compute_dt()
    assert e.value.code == hog.HOG_ENONPHYS
    assert g.last_bad_zone() == (1 * 6 + 2) * 6 + 3
    # a step that blows up keeps the pre-step state
    sm = icgen.random_smooth(n=(6, 6, 6), ndim=3, seed=2, amp=0.3)
    g.set_state(sm.U)
    with pytest.raises(hog.HogError) as e:
        g.step(50.0)
    assert e.value.code == hog.HOG_ENONPHYS
    np.testing.assert_array_equal(g.get_state(), sm.U)
    assert g.compute_dt() > 0


@pytest.mark.parametrize("t_end", [0.0, 10.0])
def test_advance_keeps_the_state_before_a_failing_step(hog, t_end):
    """A device-side run of steps that meets a non-physical state stops there:
    hog_advance returns HOG_ENONPHYS with the state before the failing step
    current and the failing step's first bad zone, like the same steps taken
    one at a time with hog_step; the handle then steps normally again.  The
    workload (a cold rarefying flow at fourth order without the positivity
    fallback) fails in its third step on the oracle too."""
    pb = icgen.cold_wave(n=32, ndim=2, amp=2.0, p0=1e-3)
    c = oracle.cfg_from_problem(pb, 4, positivity=False)
    U = pb.U
    for s in range(2):
        U = oracle.step(c, U, oracle.cfl_dt(c, U)[0])
        assert oracle.cfl_dt(c, U)[1] < 0
    assert oracle.cfl_dt(c, oracle.step(c, U, oracle.cfl_dt(c, U)[0]))[1] >= 0
    g = grid_for(hog, pb, 4, positivity=False)
    states = [pb.U]
    failed_at, bad_zone = None, None
    for s in range(10):
        try:
            g.step(g.compute_dt())
        except hog.HogError as e:
            assert e.code == hog.HOG_ENONPHYS
            failed_at, bad_zone = s, g.last_bad_zone()
            break
        states.append(g.get_state())
    assert failed_at == 2 and bad_zone >= 0
    g2 = grid_for(hog, pb, 4, positivity=False)
    with pytest.raises(hog.HogError) as e:
        g2.advance(10, t_end=t_end)
    assert e.value.code == hog.HOG_ENONPHYS
    assert g2.last_bad_zone() == bad_zone
    np.testing.assert_array_equal(g2.get_state(), states[failed_at])
    # the run is over: the handle steps and advances as usual from a new state
    g2.set_state(pb.U)
    assert g2.advance(2) > 0
    np.testing.assert_array_equal(g2.get_state(), states[2])


@pytest.mark.parametrize("riemann", ["hllc", "hll", "rusanov"])
def test_inadmissible_face_states_without_fallback_match_oracle(hog, riemann):
    """A cold rarefaction at fourth order without the positivity fallback:
    many face states have negative pressure, so the sound speeds and the
    Roe-averaged wave speeds are undefined (NaN).  The branches of the
    solvers are taken in the order the scheme defines (HLLC: S_L >= 0,
    S* >= 0, S_R > 0, else the right flux; every comparison with NaN is false),
    so the GPU takes the same branch as the oracle, state for state."""
    pb = icgen.cold_wave(n=32, ndim=2, amp=2.0, p0=1e-3)
    c = oracle.cfg_from_problem(pb, 4, positivity=False, riemann=riemann)
    dt, _ = oracle.cfl_dt(c, pb.U)
    Uo = oracle.step(c, pb.U, dt)
    g = grid_for(hog, pb, 4, positivity=False, riemann=riemann)
    g.step(dt, want_next=False)
    U = g.get_state()
    assert np.array_equal(np.isnan(U), np.isnan(Uo))
    fin = np.isfinite(Uo)
    np.testing.assert_allclose(U[fin], Uo[fin], rtol=1e-12, atol=1e-13 * np.abs(Uo[fin]).max())

"""Parity of the fused second-order kernel (Sec. II.2, Figs. 3-7) with the
oracle's second-order scheme, through the C ABI.

Same bar as the higher orders: relative L1 <= 1e-12 over all variables and
element-wise agreement to 1e-12 relative; the limited slopes, the time mode
and the face fluxes are compared through the debug taps, the positivity
fallback by its zone count.  Grid sizes span several column tiles and march
chunks with ragged ends, and include tiles that end exactly on the grid edge.
"""
import numpy as np
import pytest

import icgen
import oracle
from tests.test_gpu_parity import REL_L1, note, rel_l1

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hog():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_13295_amd import hog as h
    h.load()
    return h


def _check_step(hog, pb, riemann="hll", **kw):
    g = hog.Grid.from_problem(pb, 2, riemann=riemann, **kw)
    c = oracle.cfg_from_problem(pb, 2, riemann=riemann, **kw)
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


# 3D: x and y tiles of 14 zones, march chunks of at least 8 planes
SIZES_3D = [(37, 30, 21), (28, 14, 16), (15, 29, 9)]
SIZES_2D = [(600, 45, 1), (254, 17, 1), (255, 8, 1)]


@pytest.mark.parametrize("riemann", ["hllc", "hll", "rusanov", "hllem", "hlli"])
@pytest.mark.parametrize("bc", ["periodic", "outflow"])
@pytest.mark.parametrize("ndim", [2, 3])
def test_o2_one_step_matches_oracle(hog, ndim, bc, riemann):
    n = SIZES_3D[0] if ndim == 3 else SIZES_2D[0]
    note(f"O2 one step ndim={ndim} n={n} bc={bc} riemann={riemann}")
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=21 + ndim, amp=0.4, bc=bc, h=(0.1, 0.08, 0.11))
    _check_step(hog, pb, riemann)


@pytest.mark.parametrize("n", SIZES_3D[1:] + SIZES_2D[1:])
def test_o2_tile_edges_match_oracle(hog, n):
    """Grids whose extent is a whole number of tiles (the last tile's halo
    column is the zone one past the grid) or one zone past it."""
    ndim = 3 if n[2] > 1 else 2
    note(f"O2 tile edges n={n}")
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=sum(n), amp=0.4, bc="outflow", h=(0.1, 0.08, 0.11))
    _check_step(hog, pb, "hllc")


@pytest.mark.parametrize("ndim", [2, 3])
def test_o2_stage_taps_match_oracle(hog, ndim):
    """Mean, limited slopes and time mode of every zone (debug tap) and the
    face fluxes of every face against the oracle's modes and its Riemann
    solver at the face states of Fig. 5."""
    n = (19, 16, 11) if ndim == 3 else (40, 23, 1)
    note(f"O2 taps ndim={ndim} n={n}")
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=3, amp=0.4, bc="outflow", h=(0.1, 0.12, 0.09))
    g = hog.Grid.from_problem(pb, 2, riemann="hllc", debug=True)
    c = oracle.cfg_from_problem(pb, 2, riemann="hllc")
    dt, _ = oracle.cfl_dt(c, pb.U)
    g.step(dt)
    W, q = g.tap(hog.TAP_MODES), g.tap(hog.TAP_STMODES)
    Wo, qo = oracle.stage_modes(c, pb.U, dt)
    scale = np.abs(qo).max()
    np.testing.assert_allclose(W, Wo, rtol=0, atol=1e-14 * scale)
    np.testing.assert_allclose(q, qo, rtol=0, atol=1e-13 * scale)
    # fluxes at interior faces from the oracle's modes (both neighbours interior)
    nv = ndim + 2
    shp = (n[2], n[1], n[0]) if ndim == 3 else (n[1], n[0])
    qg = qo.reshape(shp + (2 + ndim, nv))
    for d in range(ndim):
        F = g.tap(hog.TAP_FLUX_X + d)
        F = F.reshape((nv,) + ((F.shape[1], F.shape[2], F.shape[3]) if ndim == 3 else (F.shape[2], F.shape[3])))
        ax = ndim - 1 - d
        for trial in range(40):
            rng = np.random.default_rng(trial)
            idx = [int(rng.integers(0, s)) for s in shp]
            if idx[ax] == shp[ax] - 1:
                continue
            hi = list(idx)
            hi[ax] += 1
            qa, qb = qg[tuple(idx)], qg[tuple(hi)]
            UL = qa[0] + 0.5 * qa[1 + d] + 0.5 * qa[1 + ndim]
            UR = qb[0] - 0.5 * qb[1 + d] + 0.5 * qb[1 + ndim]
            ref = oracle.riemann(c, d, UL, UR)
            fidx = list(idx)
            fidx[ax] += 1          # face box starts one face below zone 0
            got = F[(slice(None),) + tuple(fidx)]
            np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())
    g.close()


@pytest.mark.parametrize("ndim", [2, 3])
def test_o2_positivity_fallback_matches_oracle(hog, ndim):
    """Cold sinusoidal flow: GPU and oracle fall back in the same zones (same
    count) and agree on the state; without the fallback the step is refused
    and the state kept."""
    n = 40 if ndim == 2 else 20
    note(f"O2 fallback cold wave ndim={ndim} n={n}")
    pb = icgen.cold_wave(n=n, ndim=ndim)
    assert _check_step(hog, pb, "hll") > 0
    g = hog.Grid.from_problem(pb, 2, riemann="hll", positivity=False)
    U = pb.U
    raised = False
    for _ in range(3):
        try:
            g.step(g.compute_dt())
        except hog.HogError as e:
            assert e.code == hog.HOG_ENONPHYS
            raised = True
            break
    assert raised
    g.close()


def test_o2_runs_match_oracle(hog):
    """Vortex 2D, 128^2, 30 steps; Sod along z in 3D to t = 0.05; a 3D blast
    run: GPU and oracle time loops agree on step count, time and state."""
    note("O2 vortex2d 128^2 x30")
    pb = icgen.vortex2d(128)
    g = hog.Grid.from_problem(pb, 2, riemann="hll")
    t = g.advance(30)
    c = oracle.cfg_from_problem(pb, 2, riemann="hll")
    Uo, to, _ = oracle.run(c, pb.U, nsteps=30)
    assert abs(t - to) <= 1e-13 * to
    assert rel_l1(g.get_state(), Uo) <= REL_L1
    g.close()
    note("O2 sod along z to t = 0.05")
    pb = icgen.sod(n=64, axis=2, ndim=3, ntrans=3)
    g = hog.Grid.from_problem(pb, 2, riemann="hllc")
    t = g.advance(100000, t_end=0.05)
    c = oracle.cfg_from_problem(pb, 2, riemann="hllc")
    Uo, to, _ = oracle.run(c, pb.U, t_end=0.05)
    assert abs(t - to) <= 1e-12
    assert rel_l1(g.get_state(), Uo) <= REL_L1
    g.close()
    note("O2 multiblast 32^3 x5")
    pb = icgen.multiblast(n=32, seed=3)
    g = hog.Grid.from_problem(pb, 2, riemann="hll")
    g.advance(5)
    c = oracle.cfg_from_problem(pb, 2, riemann="hll")
    Uo, _, _ = oracle.run(c, pb.U, nsteps=5)
    assert rel_l1(g.get_state(), Uo) <= REL_L1
    g.close()


@pytest.mark.parametrize("ndim,n,bc", [
    (3, (1, 1, 1), "outflow"), (3, (1, 4, 3), "outflow"), (3, (3, 3, 3), "periodic"),
    (3, (2, 3, 1), "outflow"), (2, (1, 6, 1), "outflow"), (2, (3, 3, 1), "periodic")])
def test_o2_degenerate_grids_match_oracle(hog, ndim, n, bc):
    note(f"O2 degenerate grid {n} ndim={ndim} bc={bc}")
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=sum(n) + 2, amp=0.3, bc=bc, h=(0.1, 0.08, 0.11))
    _check_step(hog, pb, "hllc")


def test_o2_full_size_first_step_sampled(hog):
    """128^3 second-order step of the 3D vortex workload in the benchmark's
    launch configuration: sampled zones (interior, faces, edges, corners)
    against the oracle, plus exact conservation over the periodic box."""
    note("O2 vortex3d_perturbed 128^3 first step, sampled")
    pb = icgen.vortex3d_perturbed(n=128, seed=2)
    g = hog.Grid.from_problem(pb, 2, riemann="hll")
    c = oracle.cfg_from_problem(pb, 2, riemann="hll")
    dto, _ = oracle.cfl_dt(c, pb.U)
    g.step(dto)
    U = g.get_state()
    g.close()
    rng = np.random.default_rng(0)
    pts = np.vstack([rng.integers(0, 128, size=(64, 3)),
                     [[0, 0, 0], [127, 127, 127], [0, 127, 64], [127, 0, 1], [64, 64, 0], [13, 14, 15]]])
    ref = oracle.step_zones(c, pb.U, dto, pts)
    got = np.stack([U[:, k, j, i] for i, j, k in pts])
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())
    tot0, tot1 = pb.U.sum(axis=(1, 2, 3)), U.sum(axis=(1, 2, 3))
    assert (np.abs(tot1 - tot0) / np.maximum(np.abs(pb.U).sum(axis=(1, 2, 3)), 1.0)).max() < 1e-13


def test_o2_rejects_what_it_does_not_have(hog):
    pb = icgen.uniform(n=(6, 6, 6), ndim=3)
    with pytest.raises(hog.HogError) as e:
        hog.Grid.from_problem(pb, 2, precision="mixed")
    assert e.value.code == hog.HOG_EINVAL
    g = hog.Grid.from_problem(pb, 2)
    with pytest.raises(hog.HogError) as e:
        g.set_gate_flags(np.zeros((6, 6, 6), dtype=np.uint8))
    assert e.value.code == hog.HOG_EINVAL
    g.close()


def test_o2_runs_are_bitwise_deterministic(hog):
    pb = icgen.multiblast(n=30, seed=4)
    outs = []
    for _ in range(2):
        g = hog.Grid.from_problem(pb, 2, riemann="hllc")
        g.advance(3)
        outs.append(g.get_state())
        g.close()
    np.testing.assert_array_equal(outs[0], outs[1])

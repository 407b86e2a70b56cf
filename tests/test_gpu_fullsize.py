"""Full-size workloads over several steps, FP64 path against the FP64 oracle
(the same problem over the same steps, as the paper compares its CPU and GPU
runs in Sec. IV.1, Table XII).

* Five steps of the 128^3 vortex workload, the 256^3 multi-blast and the
  384^3 four-quadrant problem at the oracle's CFL time step of the initial
  state, in the benchmark's launch configuration; the oracle's values at 50+
  sampled zones per workload come from tests/golden/fullsize_multistep_samples.json,
  written by tests/golden/make_fullsize_samples.py (oracle runs on cut-outs
  that reproduce the whole-grid result at the sampled zones, pinned on the
  CPU in tests/test_oracle_cutout.py).  Bar: element-wise rtol 1e-12.
* The four-quadrant problem on 96^3 for 20 steps, whole grid: the state does
  not depend on z, so the oracle runs it one zone deep (bitwise the same
  columns, pinned on the CPU) and every zone of the GPU grid is compared.
  Bar: relative L1 <= 1e-12.
"""
import json
import os
import sys

import numpy as np
import pytest

import icgen
import oracle

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "fullsize_multistep_samples.json")
MAKERS = {
    "vortex3d_perturbed_128": lambda: icgen.vortex3d_perturbed(n=128, seed=2),
    "multiblast_256": lambda: icgen.multiblast(n=256, seed=3),
    "four_quadrant_384": lambda: icgen.four_quadrant(n=384, seed=5),
}


@pytest.fixture(scope="module")
def hog():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_13295_amd import hog as h
    h.load()
    return h


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name", list(MAKERS))
def test_full_size_five_steps_sampled(hog, name):
    import torch
    with open(GOLDEN) as f:
        gold = json.load(f)
    rec = gold["workloads"][name]
    steps, dt = gold["steps"], rec["dt"]
    note(f"{name}: {steps} steps at dt = {dt!r}, {len(rec['zones'])} sampled zones")
    pb = MAKERS[name]()
    assert list(pb.n) == rec["n"]
    g = hog.Grid.from_problem(pb, 4)
    dt_gpu = g.compute_dt()
    assert abs(dt_gpu - dt) <= 1e-14 * dt
    for _ in range(steps):
        g.step(dt)
    U = g.get_state()
    g.close()
    del g
    torch.cuda.empty_cache()
    zones = np.array(rec["zones"])
    ref = np.array(rec["values"])
    got = np.stack([U[:, k, j, i] for i, j, k in zones])
    note(f"{name}: max |gpu - oracle| = {np.abs(got - ref).max():.3e} (state scale {np.abs(ref).max():.3e})")
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-13 * np.abs(ref).max())


def test_four_quadrant_96_twenty_steps_whole_grid(hog):
    import torch
    n, steps = 96, 20
    pb = icgen.four_quadrant(n=n, seed=5)
    one = icgen.Problem(U=np.ascontiguousarray(pb.U[:, :1]), ndim=3, n=(n, n, 1), h=pb.h, origin=pb.origin,
                        bc=pb.bc, gamma=pb.gamma)
    c = oracle.cfg_from_problem(one, 4)
    Uo, to, dts = oracle.run(c, one.U, nsteps=steps)
    note(f"four-quadrant {n}^3 x {steps}: oracle done, t = {to!r}")
    g = hog.Grid.from_problem(pb, 4)
    for s in range(steps):
        g.step(float(dts[s]))
    U = g.get_state()
    g.close()
    del g
    torch.cuda.empty_cache()
    ref = np.broadcast_to(Uo, U.shape)
    rel = float(np.abs(U - ref).sum() / np.abs(ref).sum())
    note(f"four-quadrant {n}^3 x {steps}: whole-grid relative L1 vs oracle {rel:.3e}")
    assert rel <= 1e-12
    # and the device-side time loop takes the oracle's time steps
    g = hog.Grid.from_problem(pb, 4)
    t = g.advance(steps)
    assert abs(t - to) <= 1e-13 * to
    rel2 = float(np.abs(g.get_state() - ref).sum() / np.abs(ref).sum())
    g.close()
    assert rel2 <= 1e-12

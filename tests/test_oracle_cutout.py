"""The locality the full-size multi-step checks rest on (CPU only): after s
fourth-order ADER steps a zone depends only on the zones within 3 s of it,
so the oracle run on a cut-out with 3 s zones on every side of the sampled
zones reproduces the whole-grid result there bitwise, and a cut-out one zone
narrower does not.  Along an outflow axis the cut-out stops at the domain
boundary and keeps the real boundary condition."""
import numpy as np
import pytest

import icgen
import oracle
from cutout import cutout

S = 2


def _run(pb, dt, steps):
    c = oracle.cfg_from_problem(pb, 4)
    U = pb.U
    for _ in range(steps):
        U = oracle.step(c, U, dt)
    return U


@pytest.mark.parametrize("case", ["periodic", "outflow_corner"])
def test_cutout_reproduces_whole_grid_only_beyond_the_reach(case):
    if case == "periodic":
        pb = icgen.random_smooth(n=(20, 19, 18), ndim=3, seed=4, amp=0.2)
        lo, hi = (9, 8, 9), (10, 9, 9)
    else:
        pb = icgen.random_smooth(n=(18, 17, 16), ndim=3, seed=5, amp=0.2, bc="outflow")
        lo, hi = (0, 15, 0), (1, 16, 1)      # a box at a corner of the domain
    c = oracle.cfg_from_problem(pb, 4)
    dt, _ = oracle.cfl_dt(c, pb.U)
    full = _run(pb, dt, S)
    zones = [(i, j, k) for i in range(lo[0], hi[0] + 1) for j in range(lo[1], hi[1] + 1)
             for k in range(lo[2], hi[2] + 1)]
    want = np.stack([full[:, k, j, i] for i, j, k in zones])
    for hw, exact in ((3 * S, True), (3 * S - 1, False)):
        sub, where = cutout(pb, lo, hi, hw)
        assert all(sub.n[a] < pb.n[a] for a in range(3))
        U = _run(sub, dt, S)
        got = np.stack([U[:, where(i, j, k)[2], where(i, j, k)[1], where(i, j, k)[0]] for i, j, k in zones])
        if exact:
            np.testing.assert_array_equal(got, want)
        else:
            assert np.abs(got - want).max() > 0.0


def test_z_independent_state_gives_the_same_columns_for_any_nz():
    """A state that does not depend on z, with outflow along z, stays so, and
    each column equals the one of a grid a single zone deep, bitwise (every
    zone sees the same stencil values): the whole-grid check of the
    four-quadrant workload on a 96^3 grid rests on this."""
    a = icgen.four_quadrant(n=16, seed=5)
    one = icgen.Problem(U=np.ascontiguousarray(a.U[:, :1]), ndim=3, n=(16, 16, 1), h=a.h, origin=a.origin,
                        bc=a.bc, gamma=a.gamma)
    three = icgen.Problem(U=np.ascontiguousarray(a.U[:, :3]), ndim=3, n=(16, 16, 3), h=a.h, origin=a.origin,
                          bc=a.bc, gamma=a.gamma)
    c1 = oracle.cfg_from_problem(one, 4)
    dt, _ = oracle.cfl_dt(c1, one.U)
    U1 = _run(one, dt, S)
    U3 = _run(three, dt, S)
    for k in range(3):
        np.testing.assert_array_equal(U3[:, k], U1[:, 0])
    assert np.abs(U1 - one.U).max() > 1e-3      # the step did something

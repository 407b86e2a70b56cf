"""hog_step_static, the step that allocates nothing (its workspace is the
library's fixed device array), against hog_step on a handle with a caller
workspace: the same kernels in the same launch configuration, so the states
and the next time steps must agree bitwise.  Two calls in a row share the
array; the second runs a smaller grid, so what the first left behind must not
leak into it."""
import sys

import numpy as np
import pytest

import icgen

pytestmark = pytest.mark.gpu


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


def rel_l1(a, b):
    return float(np.abs(a - b).sum() / np.abs(b).sum())


def handle_step(hog, pb, order, **kw):
    g = hog.Grid.from_problem(pb, order, **kw)
    dt = g.compute_dt()
    dt_next = g.step(dt)
    U = g.get_state()
    cfg = g.cfg
    g.close()
    return cfg, dt, U, dt_next


def static_step(hog, cfg, U0, dt, in_place=False):
    import torch
    U_in = torch.from_numpy(np.ascontiguousarray(U0)).cuda()
    U_out = U_in if in_place else torch.empty_like(U_in)
    dt_next = hog.step_static(cfg, U_in, U_out, dt)
    torch.cuda.synchronize()
    return U_out.cpu().numpy(), dt_next


CASES = [
    # (problem, order, keyword arguments): the first call of each pair is the larger grid
    (lambda: icgen.random_smooth(n=(21, 18, 16), ndim=3, seed=11, amp=0.2), 4, {}),
    (lambda: icgen.random_smooth(n=(12, 10, 9), ndim=3, seed=12, amp=0.2, bc="outflow"), 4, {"riemann": "hll"}),
]


@pytest.mark.parametrize("first,second", [(0, 1)])
def test_static_step_equals_handle_step_two_calls(hog, first, second):
    for k in (first, second):
        make, order, kw = CASES[k]
        pb = make()
        note(f"static step case {k}: {pb.n} order {order} {kw}")
        cfg, dt, ref, ref_next = handle_step(hog, pb, order, **kw)
        got, got_next = static_step(hog, cfg, pb.U, dt)
        assert rel_l1(got, ref) <= 1e-12
        np.testing.assert_array_equal(got, ref)
        assert got_next == ref_next


@pytest.mark.parametrize("ndim,order,precision,stepper", [
    (2, 3, "fp64", "ader"), (3, 3, "mixed", "ader"), (3, 2, "fp64", "ader"), (2, 4, "fp64", "rk3")])
def test_static_step_other_paths(hog, ndim, order, precision, stepper):
    """Other orders, the mixed path, the fused second-order kernel and a
    Runge-Kutta step, each run twice (the second time in place)."""
    n = (40, 33, 1) if ndim == 2 else (17, 14, 11)
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=3 + order, amp=0.2)
    note(f"static step {ndim}D order {order} {precision} {stepper}")
    cfg, dt, ref, ref_next = handle_step(hog, pb, order, precision=precision, stepper=stepper)
    for in_place in (False, True):
        got, got_next = static_step(hog, cfg, pb.U, dt, in_place=in_place)
        np.testing.assert_array_equal(got, ref)
        assert got_next == ref_next


def test_static_step_nonphysical_leaves_output_untouched(hog):
    import torch
    pb = icgen.multiblast(n=24, seed=3)
    cfg = hog.make_config(3, pb.n, 4, pb.h, gamma=pb.gamma, bc=pb.bc, positivity=False)
    U_in = torch.from_numpy(np.ascontiguousarray(pb.U)).cuda()
    U_out = torch.full_like(U_in, 7.0)
    with pytest.raises(hog.HogError) as e:
        hog.step_static(cfg, U_in, U_out, 1e-3)
    assert e.value.code == hog.HOG_ENONPHYS
    assert bool((U_out == 7.0).all())
    # the next call on the same array starts clean
    pb2 = icgen.random_smooth(n=(9, 8, 7), ndim=3, seed=5, amp=0.2)
    cfg2, dt, ref, ref_next = handle_step(hog, pb2, 4)
    got, got_next = static_step(hog, cfg2, pb2.U, dt)
    np.testing.assert_array_equal(got, ref)
    assert got_next == ref_next


def test_static_step_rejects_grids_beyond_its_array(hog):
    import torch
    cap = hog.step_static_capacity()
    cfg = hog.make_config(3, (64, 64, 64), 4, (0.1, 0.1, 0.1))
    assert hog.workspace_size(cfg) > cap
    U = torch.zeros(5 * 64 ** 3, dtype=torch.float64, device="cuda")
    with pytest.raises(hog.HogError) as e:
        hog.step_static(cfg, U, U, 1e-3)
    assert e.value.code == hog.HOG_ENOMEM
    assert "at most" in str(e.value)

"""Slab streaming of a host-resident mesh (hog_stream_*) and the external
boundary it is built on: the streamed step must equal the in-core step of the
whole mesh zone for zone (bitwise: every zone sees the same stencil and the
same arithmetic), over several steps with the CFL dt, and match the oracle."""
import os

import numpy as np
import pytest

import icgen
import oracle
from tests.test_gpu_parity import REL_L1, note, rel_l1

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hog():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_13295_amd import hog as h
    h.load()
    return h


def _mesh(ndim, n, bc_last, seed):
    bc = ["outflow", "periodic", bc_last] if ndim == 3 else ["periodic", bc_last, "outflow"]
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=seed, amp=0.3, bc="periodic", h=(0.1, 0.08, 0.11))
    pb.bc = tuple(bc)
    return pb


@pytest.mark.parametrize("ndim,order", [(3, 4), (3, 2), (2, 3)])
def test_external_slab_matches_in_core(hog, ndim, order):
    """A slab grid whose last axis is external, given its ghost layers from the
    mesh (periodic wrap), steps its zones exactly like the whole mesh does."""
    n = (12, 9, 20) if ndim == 3 else (30, 20, 1)
    note(f"external slab ndim={ndim} order={order}")
    pb = _mesh(ndim, n, "periodic", 3)
    g = hog.Grid.from_problem(pb, order)
    c = oracle.cfg_from_problem(pb, order)
    dt, _ = oracle.cfl_dt(c, pb.U)
    g.step(dt)
    full = g.get_state()
    g.close()
    nl = n[ndim - 1]
    z0, nz = 6, 7
    idx = [(z0 + k) % nl for k in range(-3, nz + 3)]
    ext = pb.U[:, idx]
    ns = list(n)
    ns[ndim - 1] = nz
    bc = list(pb.bc)
    bc[ndim - 1] = "external"
    import torch
    for src in (ext, torch.from_numpy(np.ascontiguousarray(ext)).cuda()):     # host, then device
        s = hog.Grid(ndim, ns, order, pb.h, gamma=pb.gamma, bc=tuple(bc))
        s.set_state_ext(src)
        s.step(dt)
        got = s.get_state()
        s.close()
        np.testing.assert_array_equal(got, full[:, z0:z0 + nz])


BLOCK_CASES = [
    # ndim, order, precision, mesh boundaries, external axes
    (3, 4, "fp64", ("periodic",) * 3, (0, 1, 2)),
    (3, 4, "mixed", ("periodic",) * 3, (0, 1, 2)),
    (3, 4, "fp64", ("periodic", "outflow", "periodic"), (0, 2)),
    (3, 3, "fp64", ("outflow", "periodic", "outflow"), (1,)),
    (3, 2, "fp64", ("periodic",) * 3, (0, 1, 2)),
    (2, 4, "fp64", ("periodic", "periodic", "outflow"), (0, 1)),
    (3, 4, "mixed+gate", ("periodic",) * 3, (0, 1, 2)),
]


@pytest.mark.parametrize("ndim,order,precision,bc,axes", BLOCK_CASES)
def test_external_block_matches_in_core(hog, ndim, order, precision, bc, axes):
    """One block of a mesh, external along the given axes (with every axis
    external: one rank's share of a mesh split over devices), given its ghost
    layers from the mesh (wrapped or clamped by the mesh's boundary types:
    what the neighbouring blocks would send), steps its zones exactly like
    the whole mesh does: the same stencils, the same arithmetic."""
    n = (20, 17, 15) if ndim == 3 else (36, 30, 1)
    note(f"external block ndim={ndim} order={order} {precision} bc={bc} axes={axes}")
    # (a gentler state for the gated case, so that the network gates a good share of the zones)
    amp = 0.02 if precision == "mixed+gate" else 0.3
    pb = icgen.random_smooth(n=n, ndim=ndim, seed=7 + order, amp=amp, bc="periodic", h=(0.1, 0.08, 0.11))
    pb.bc = tuple(bc)
    riemann = "hll" if order == 2 else "hllc"
    gate = None
    if precision == "mixed+gate":
        # the trained network: a block's gate flags see the same 13-zone crosses
        # (through the supplied ghost layers) as the mesh's
        z = np.load(os.path.join(ROOT, "paper_2211_13295_amd", "gate_o4_3d.npz"))
        gate = (z["params"], float(z["theta"]))
        precision = "mixed"
    g = hog.Grid.from_problem(pb, order, precision=precision, riemann=riemann)
    if gate is not None:
        g.set_gate(gate[0], theta=gate[1])
        note(f"gated fraction {float(g.gate_eval()[1].mean()):.3f}")
    dt = g.compute_dt()
    g.step(dt)
    full = g.get_state()
    g.close()
    lo = (3, 4, 2)
    m = (11, 9, 8) if ndim == 3 else (21, 17, 1)
    idx, sl, nb, bcb = [], [], [], list(bc)
    for d in range(ndim):
        nd_ = n[d]
        if d in axes:
            ids = [lo[d] + k for k in range(-3, m[d] + 3)]
            if bc[d] == "periodic":
                ids = [x % nd_ for x in ids]
            else:
                ids = [min(max(x, 0), nd_ - 1) for x in ids]
            idx.append(ids)
            sl.append(slice(lo[d], lo[d] + m[d]))
            nb.append(m[d])
            bcb[d] = "external"
        else:
            idx.append(list(range(nd_)))
            sl.append(slice(0, nd_))
            nb.append(nd_)
    # the mesh state is [v][(z)][y][x]: the axis order is reversed
    ext = pb.U[np.ix_(range(pb.U.shape[0]), *reversed(idx))]
    want = full[(slice(None),) + tuple(reversed(sl))]
    if ndim == 2:
        nb.append(1)
    import torch
    b = hog.Grid(ndim, tuple(nb), order, pb.h, gamma=pb.gamma, bc=tuple(bcb), precision=precision, riemann=riemann)
    if gate is not None:
        b.set_gate(gate[0], theta=gate[1])
    with pytest.raises(ValueError):
        b.set_state_ext(pb.U)
    b.set_state_ext(torch.from_numpy(np.ascontiguousarray(ext)).cuda())
    b.step(dt)
    got = b.get_state()
    b.close()
    np.testing.assert_array_equal(got, want)


CASES = [(3, 4, "periodic", (14, 11, 23), 5), (3, 3, "outflow", (13, 10, 17), 8), (3, 2, "periodic", (33, 20, 19), 3),
         (3, 4, "outflow", (9, 8, 10), 10), (2, 4, "outflow", (40, 29, 1), 7), (2, 2, "periodic", (300, 26, 1), 1)]


@pytest.mark.parametrize("ndim,order,bc_last,n,slab", CASES)
def test_stream_equals_in_core(hog, ndim, order, bc_last, n, slab):
    note(f"stream ndim={ndim} order={order} {bc_last} n={n} slab={slab}")
    pb = _mesh(ndim, n, bc_last, order + slab)
    riemann = "hll" if order == 2 else "hllc"
    g = hog.Grid.from_problem(pb, order, riemann=riemann)
    st = hog.Stream.from_problem(pb, order, slab, riemann=riemann)
    dt_g, dt_s = g.compute_dt(), st.compute_dt()
    assert dt_g == dt_s
    for k in range(3):
        dt_g = g.step(dt_g)
        dt_s = st.step(0.0 if k else dt_s)
        assert dt_g == dt_s
        np.testing.assert_array_equal(st.get_state(), g.get_state())
    g.close()
    st.close()


@pytest.mark.parametrize("ndim,n,slab", [(3, (14, 11, 23), 5), (2, (40, 29, 1), 7)])
def test_stream_mixed_precision_equals_in_core(hog, ndim, n, slab):
    """The mixed FP32/FP64 path streams too: same kernels per slab, so the
    streamed steps equal the in-core mixed steps bitwise."""
    note(f"stream mixed ndim={ndim} n={n} slab={slab}")
    pb = _mesh(ndim, n, "periodic", 11)
    g = hog.Grid.from_problem(pb, 4, precision="mixed")
    st = hog.Stream.from_problem(pb, 4, slab, precision="mixed")
    dt = g.compute_dt()
    assert st.compute_dt() == dt
    for k in range(2):
        dt_g = g.step(dt)
        dt_s = st.step(dt)
        assert dt_g == dt_s
        dt = dt_g
        np.testing.assert_array_equal(st.get_state(), g.get_state())
    g.close()
    st.close()


def test_stream_matches_oracle(hog):
    note("stream 3D O4 vs oracle")
    pb = _mesh(3, (11, 10, 13), "periodic", 5)
    st = hog.Stream.from_problem(pb, 4, 4)
    c = oracle.cfg_from_problem(pb, 4)
    dt, _ = oracle.cfl_dt(c, pb.U)
    st.step(dt)
    Uo = oracle.step(c, pb.U, dt)
    assert rel_l1(st.get_state(), Uo) <= REL_L1
    st.close()


def test_stream_nonphysical_step_keeps_the_state(hog):
    note("stream non-physical")
    pb = icgen.multiblast(n=24, seed=3)
    st = hog.Stream.from_problem(pb, 4, 5, positivity=False)
    U0 = st.get_state()
    with pytest.raises(hog.HogError) as e:
        st.step(0.0)
    assert e.value.code == hog.HOG_ENONPHYS
    np.testing.assert_array_equal(st.get_state(), U0)
    st.close()


def test_stream_rejects_bad_configurations(hog):
    pb = icgen.uniform(n=(6, 6, 6), ndim=3)
    for kw, slab in (({"stepper": "rk3"}, 2), ({}, 0), ({}, 7), ({"bc": ("periodic", "periodic", "external")}, 2)):
        with pytest.raises(hog.HogError) as e:
            hog.Stream.from_problem(pb, 4, slab, **kw)
        assert e.value.code == hog.HOG_EINVAL
    # any axis may be external, but only with the one-exchange ADER step
    with pytest.raises(hog.HogError) as e:
        hog.Grid(3, (6, 6, 6), 4, (0.1, 0.1, 0.1), bc=("external", "periodic", "periodic"), stepper="rk3")
    assert e.value.code == hog.HOG_EINVAL
    with pytest.raises(hog.HogError) as e:
        hog.Stream.from_problem(pb, 4, 2, bc=("external", "periodic", "periodic"))
    assert e.value.code == hog.HOG_EINVAL
    # one host buffer for both states, or one stream for compute and copies
    import ctypes
    import torch
    L = hog.load()
    cfg = hog.make_config(3, (6, 6, 6), 4, (0.1, 0.1, 0.1))
    nb = ctypes.c_size_t(0)
    assert L.hog_stream_workspace_size(ctypes.byref(cfg), 3, ctypes.byref(nb)) == hog.HOG_OK
    ws = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
    wp = ctypes.c_void_p((ws.data_ptr() + 255) // 256 * 256)
    host = torch.empty((5, 6, 6, 6), dtype=torch.float64, pin_memory=True)
    other = torch.empty_like(host).pin_memory()
    cs, xs = torch.cuda.current_stream(), torch.cuda.Stream()
    out = ctypes.c_void_p()
    hp, op = ctypes.c_void_p(host.data_ptr()), ctypes.c_void_p(other.data_ptr())
    assert L.hog_stream_create(ctypes.byref(cfg), 3, wp, nb.value, hp, hp, ctypes.c_void_p(cs.cuda_stream),
                               ctypes.c_void_p(xs.cuda_stream), ctypes.byref(out)) == hog.HOG_EINVAL
    assert L.hog_stream_create(ctypes.byref(cfg), 3, wp, nb.value, hp, op, ctypes.c_void_p(cs.cuda_stream),
                               ctypes.c_void_p(cs.cuda_stream), ctypes.byref(out)) == hog.HOG_EINVAL


def test_stream_full_size_equals_in_core(hog):
    """The 128^3 fourth-order workload streamed in slabs of 32 planes (the
    benchmark's slab size; 4 slabs, the copies overlapping the steps) equals
    the in-core steps bitwise over two CFL steps."""
    note("stream 128^3 O4 slabs of 32 vs in core")
    import torch
    pb = icgen.vortex3d_perturbed(n=128, seed=2)
    g = hog.Grid.from_problem(pb, 4)
    st = hog.Stream.from_problem(pb, 4, 32)
    dt = g.compute_dt()
    assert st.compute_dt() == dt
    for _ in range(2):
        dt_g = g.step(dt)
        assert st.step(dt) == dt_g
        dt = dt_g
    np.testing.assert_array_equal(st.get_state(), g.get_state())
    g.close()
    st.close()
    torch.cuda.empty_cache()

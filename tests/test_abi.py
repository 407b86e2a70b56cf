"""The C-ABI library loads and exports every function include/hog.h declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2211_13295_amd", "libhog.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hog.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(hog_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hog_create", "hog_destroy", "hog_set_state", "hog_get_state", "hog_compute_dt",
                     "hog_step", "hog_advance", "hog_workspace_size", "hog_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhog.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    lib.hog_abi_version.restype = ctypes.c_int
    assert lib.hog_abi_version() == 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhog.so not built")
def test_invalid_configs_are_rejected_without_a_device():
    from paper_2211_13295_amd import hog
    c = hog.make_config(3, (8, 8, 8), 4, (0.1, 0.1, 0.1))
    assert hog.workspace_size(c) > 0
    for field, val in (("ndim", 4), ("order", 5), ("nx", 0), ("cfl", 1.5), ("gamma", 1.0), ("riemann", 7)):
        bad = hog.make_config(3, (8, 8, 8), 4, (0.1, 0.1, 0.1))
        setattr(bad, field, val)
        with pytest.raises(hog.HogError) as e:
            hog.workspace_size(bad)
        assert e.value.code == hog.HOG_EINVAL
    bad = hog.make_config(3, (2, 8, 8), 4, (0.1, 0.1, 0.1))   # periodic axis too short
    with pytest.raises(hog.HogError):
        hog.workspace_size(bad)
    # second order: FP64 only, and its plan holds no reconstruction or predictor arrays
    o2 = hog.make_config(3, (8, 8, 8), 2, (0.1, 0.1, 0.1))
    assert 0 < hog.workspace_size(o2) < hog.workspace_size(c) // 4
    for order in (1, 5):
        bad = hog.make_config(3, (8, 8, 8), 4, (0.1, 0.1, 0.1))
        bad.order = order
        with pytest.raises(hog.HogError):
            hog.workspace_size(bad)
    with pytest.raises(hog.HogError) as e:
        hog.workspace_size(hog.make_config(3, (8, 8, 8), 2, (0.1, 0.1, 0.1), precision="mixed"))
    assert e.value.code == hog.HOG_EINVAL


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2211_13295_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "liboracle" not in txt, f


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhog.so not built")
def test_stepper_external_and_stream_configs_without_a_device():
    """Host-side checks of the Runge-Kutta, external-boundary and streaming
    configurations: valid ones plan a workspace, invalid ones are refused."""
    import ctypes
    from paper_2211_13295_amd import hog
    L = hog.load()
    for st in ("rk2", "rk3", "rk4"):
        assert hog.workspace_size(hog.make_config(3, (8, 8, 8), 4, (0.1,) * 3, stepper=st)) > 0
    assert hog.workspace_size(hog.make_config(3, (8, 8, 8), 2, (0.1,) * 3, stepper="rk2")) > 0
    bad = [hog.make_config(3, (8, 8, 8), 4, (0.1,) * 3, stepper=5),
           hog.make_config(3, (8, 8, 8), 4, (0.1,) * 3, stepper="rk3", precision="mixed"),
           hog.make_config(3, (8, 8, 8), 4, (0.1,) * 3, stepper="rk3", debug=True),
           hog.make_config(3, (8, 8, 8), 4, (0.1,) * 3, bc=("external", "periodic", "periodic"), stepper="rk3"),
           hog.make_config(3, (8, 8, 8), 4, (0.1,) * 3, bc=("periodic", "periodic", "external"), stepper="rk3"),
           hog.make_config(2, (8, 8, 1), 3, (0.1,) * 3, bc=("periodic", "periodic", "external"))]
    for c in bad:
        with pytest.raises(hog.HogError) as e:
            hog.workspace_size(c)
        assert e.value.code == hog.HOG_EINVAL
    ext = hog.make_config(3, (8, 8, 8), 4, (0.1,) * 3, bc=("periodic", "periodic", "external"))
    assert hog.workspace_size(ext) > 0
    # any axis may be external (a block of a mesh split over devices: all three)
    for bc in (("external", "periodic", "periodic"), ("external", "external", "outflow"), ("external",) * 3):
        assert hog.workspace_size(hog.make_config(3, (8, 8, 8), 4, (0.1,) * 3, bc=bc)) > 0
    assert hog.workspace_size(hog.make_config(2, (8, 8, 1), 3, (0.1,) * 3, bc=("external", "external", "periodic"))) > 0
    mesh = hog.make_config(3, (8, 8, 20), 4, (0.1,) * 3)
    nb = ctypes.c_size_t(0)
    assert L.hog_stream_workspace_size(ctypes.byref(mesh), 6, ctypes.byref(nb)) == hog.HOG_OK
    # two slab grids of 6 planes and one of 2 (20 = 3 x 6 + 2) fit in less than the in-core plan
    assert 0 < nb.value < 2 * hog.workspace_size(mesh)
    for slab, cfg in ((0, mesh), (21, mesh), (6, hog.make_config(3, (8, 8, 20), 4, (0.1,) * 3, stepper="rk3")),
                      (6, ext), (6, hog.make_config(3, (8, 8, 20), 4, (0.1,) * 3, bc=("external", "periodic", "periodic")))):
        assert L.hog_stream_workspace_size(ctypes.byref(cfg), slab, ctypes.byref(nb)) == hog.HOG_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhog.so not built")
def test_static_step_rejects_grids_beyond_its_array_without_a_device():
    """hog_step_static checks the configuration and its workspace size against
    the fixed array before any device call (the state pointers are not read on
    that path)."""
    from paper_2211_13295_amd import hog
    L = hog.load()
    cap = hog.step_static_capacity()
    assert cap == 256 << 20
    big = hog.make_config(3, (41, 41, 41), 4, (0.1, 0.1, 0.1))
    fits = hog.make_config(3, (40, 40, 40), 4, (0.1, 0.1, 0.1))
    assert hog.workspace_size(fits) <= cap < hog.workspace_size(big)
    dummy = ctypes.c_void_p(256)
    assert L.hog_step_static(ctypes.byref(big), dummy, dummy, 1e-3, None, None) == hog.HOG_ENOMEM
    assert "at most" in L.hog_last_error().decode()
    ext = hog.make_config(3, (8, 8, 8), 4, (0.1, 0.1, 0.1), bc=("periodic", "periodic", "external"))
    assert L.hog_step_static(ctypes.byref(ext), dummy, dummy, 1e-3, None, None) == hog.HOG_EINVAL
    assert L.hog_step_static(ctypes.byref(fits), None, dummy, 1e-3, None, None) == hog.HOG_EINVAL
    assert L.hog_step_static(ctypes.byref(fits), dummy, dummy, -1.0, None, None) == hog.HOG_EINVAL

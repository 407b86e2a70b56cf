"""Host logic of the benchmark script, on the CPU: the one-GPU guard, the
operation counts behind the roofline figure, and the traffic record (counter
scaling by the plain copy, and its invalidation once a kernel source
changes)."""
import itertools
import json
import math
import os
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, env=e,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _modes(D, L):
    """Exponent tuples of the total-degree-L polynomials in D variables."""
    return [m for m in itertools.product(range(L + 1), repeat=D) if sum(m) <= L]


def _sum_factorised_eval(c, D, L, x):
    """Value of sum_m c[m] prod_d x_d^m_d at every node of the tensor grid
    x^D, contracting one axis at a time (first axis first), counting one FMA
    per multiply-add.  Returns (values [node tuple], FMAs)."""
    n1, fma = len(x), 0
    # T[(nodes so far), (exponents still open)]
    T = {((), m): c[m] for m in _modes(D, L)}
    for d in range(D):
        U = {}
        for (nodes, rest), v in T.items():
            for a, xa in enumerate(x):
                key = (nodes + (a,), rest[1:])
                U[key] = U.get(key, 0.0) + v * xa ** rest[0]
                fma += 1
        T = U
    assert len(T) == n1 ** D
    return {nodes: v for (nodes, _), v in T.items()}, fma


@pytest.mark.parametrize("D,L", [(2, 2), (2, 3), (3, 2), (3, 3), (3, 1)])
def test_spatial_eval_count_is_that_of_a_sum_factorised_evaluation(D, L):
    """The FMA count of the spatial evaluation equals the multiply-adds of an
    explicit axis-by-axis evaluation, which itself gives the direct values."""
    n1 = L + 1
    x, _ = np.polynomial.legendre.leggauss(n1)
    x = 0.5 * x
    rng = np.random.default_rng(D * 10 + L)
    c = {m: rng.standard_normal() for m in _modes(D, L)}
    vals, fma = _sum_factorised_eval(c, D, L, x)
    for nodes in itertools.product(range(n1), repeat=D):
        direct = sum(cm * np.prod([x[nodes[d]] ** m[d] for d in range(D)]) for m, cm in c.items())
        assert abs(vals[nodes] - direct) <= 1e-13
    assert fma == bench.spatial_eval_fma(D, L, n1)


@pytest.mark.parametrize("D,L", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_needed_projection_count(D, L):
    """Projection onto the coefficients with degree >= 1 along the derivative
    axis and total degree <= L, contracting the derivative axis first: one FMA
    per (node still open, coefficient index fixed so far) at each stage."""
    n1 = L + 1
    fma = 0
    kept = [m for m in _modes(D, L) if m[0] >= 1]
    for d in range(D):
        prefixes = {m[:d + 1] for m in kept}      # coefficient indices fixed after axis d
        fma += len(prefixes) * n1 ** (D - d)      # each summed over n1 nodes, for every open node
    assert fma == bench.needed_proj_fma(D, L, n1)


def test_predictor_flop_figures():
    """The per-zone figures the roofline uses (3D fourth order) and those
    quoted for the other orders."""
    assert bench.predictor_flops(3, 3) == 165764
    assert [bench.predictor_flops(2, 2), bench.predictor_flops(2, 3), bench.predictor_flops(3, 2)] == \
        [5556, 26000, 26892]
    with open(os.path.join(ROOT, "profiles", "bench_vortex3d_128_o4.json")) as f:
        line = json.loads(f.read().strip().splitlines()[-1])
    assert line["roofline"]["alg_flops_per_zone"] == bench.predictor_flops(3, 3)
    assert line["roofline"]["zones_per_launch"] == 130 ** 3


def test_o2_flops_scale_with_the_grid():
    """Zone, face and grown-box terms: the count per interior zone tends to a
    constant and the grid terms grow as stated."""
    f = [bench.o2_flops(3, n) / n ** 3 for n in (64, 128, 256, 512)]
    assert all(a > b for a, b in zip(f, f[1:]))
    assert abs(f[-1] - f[-2]) < 0.02 * f[-1]
    assert bench.o2_flops(2, 1) > 0


def _csv(path, rows):
    with open(path, "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for r in rows:
            f.write(",".join(str(x) for x in r) + "\n")


def test_traffic_record_scaling_and_staleness(tmp_path, monkeypatch):
    """Counter KiB per dispatch, summed over a dispatch's rows, averaged over
    dispatches and scaled so that the copy of 1 GiB reads (writes) 1 GiB; the
    record is dropped as soon as a kernel source differs from the one hashed."""
    rec_path = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(rec_path))
    gib_kib = (1 << 30) / 1024
    kname = '"k_predict<3, 3, double>(args)"'
    copy = '"elementwise<MulFunctor>"'
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    # predictor: 2 dispatches of 1000 and 1200 KiB (split over two rows);
    # copy: counter reads half of what moved -> scale 2
    _csv(fetch, [(1, kname, "FETCH_SIZE", 600), (1, kname, "FETCH_SIZE", 400), (2, kname, "FETCH_SIZE", 1200),
                 (3, copy, "FETCH_SIZE", gib_kib / 2), (4, kname, "WRITE_SIZE", 99)])
    _csv(write, [(1, kname, "WRITE_SIZE", 300), (2, copy, "WRITE_SIZE", gib_kib)])
    bench.write_traffic(str(fetch), str(write))
    rec = json.loads(rec_path.read_text())
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_bytes_per_launch"] == pytest.approx(1100 * 1024 * 2.0)
    assert rec["write_bytes_per_launch"] == pytest.approx(300 * 1024)
    assert bench.traffic_record() == pytest.approx(rec["bytes_per_launch"])
    assert rec["algorithmic_bytes_per_launch"] == 130 ** 3 * (20 + 48) * 5 * 8
    # a changed kernel source voids the record
    src = tmp_path / "kernel.h"
    src.write_text("// one\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    rec["kernel_hash"] = bench.kernel_hash([str(src)])
    rec_path.write_text(json.dumps(rec))
    assert bench.traffic_record() == pytest.approx(rec["bytes_per_launch"])
    src.write_text("// two\n")
    assert bench.traffic_record() is None
    rec_path.write_text("not json")
    assert bench.traffic_record() is None
    assert not math.isnan(rec["bytes_per_launch"])


def test_traffic_needs_both_dispatch_kinds(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "t.json"))
    f = tmp_path / "f.csv"
    _csv(f, [(1, '"elementwise<MulFunctor>"', "FETCH_SIZE", 10)])
    with pytest.raises(SystemExit):
        bench.write_traffic(str(f), str(f))
    assert not (tmp_path / "t.json").exists()


def test_zone_rate_is_zones_per_step_time():
    """The headline's value: zones / (seconds per step), e.g. the 384^3 grid at
    415 ms per step is 1.36e8 zone-updates/s (not multiplied by the step count)."""
    import bench
    assert abs(bench.zone_rate(384 ** 3, 415.0) - 384 ** 3 / 0.415) < 1e-6 * 384 ** 3
    assert 1.3e8 < bench.zone_rate(384 ** 3, 415.0) < 1.4e8

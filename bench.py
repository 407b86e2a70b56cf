#!/usr/bin/env python3
"""Throughput of the ADER-WENO Euler zone update on one MI355X.

Default line (the metric's workload): 3D Euler, ideal gas gamma = 1.4, the
four-quadrant Riemann problem (quadrant states seeded from rho in [0.5, 1.5],
p in [0.1, 1.0], in-plane speed <= 0.5, seed 5) on 384^3 zones of [0,1]^3
with outflow boundaries, fourth-order WENO + ADER, HLLC, CFL 0.4.  `value` is
the FP64 path's zone-updates/s; beside it the mixed FP32/FP64 path with the
trained smooth-zone gate (and without it) on the same time steps, each with
its relative L1 against the FP64 path after the same steps.  The 128^3 vortex
workload's figures follow as an extra key.

The timed region holds K full steps (ghost fill, reconstruction, predictor,
Riemann solver, update and CFL reduction) with the state resident in HBM,
bracketed by device synchronisation.  Per-stage times come from HIP events
recorded by the library on the stream its kernels run on.
"""
import argparse
import ctypes as C
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "zone-updates/sec, 3D Euler WENO+ADER, FP64 vs FP32+learned gate at stated L1"
UNIT = "zone-updates/s"
PEAK_FP64_VALU_TFLOPS = 78.6          # MI355X published FP64 vector peak
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_predictor_vortex3d_128.json")
TRAFFIC_FILE_C5 = os.path.join(ROOT, "profiles", "traffic_predictor_fourquad384.json")
# Algorithmic flops per zone of the fourth-order 3D predictor as estimated in
# the design's scope table (sum-factorised evaluation and projection); the
# exact count of the formulation built here is predictor_flops(3, 3).
PREDICTOR_FLOPS_ESTIMATE_3D_O4 = 2.2e5
TRAFFIC_FILE_O2 = os.path.join(ROOT, "profiles", "traffic_o2_step_vortex3d_128.json")
TRAFFIC_FILE_RK = os.path.join(ROOT, "profiles", "traffic_face_points_vortex3d_128.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2211_13295_amd", "csrc", f)
                  for f in ("hog_kernels.h", "hog_physics.h", "hog_tables.h")]
KERNEL_SOURCES_O2 = KERNEL_SOURCES + [os.path.join(ROOT, "paper_2211_13295_amd", "csrc", "hog_o2.h")]
KERNEL_SOURCES_RK = KERNEL_SOURCES + [os.path.join(ROOT, "paper_2211_13295_amd", "csrc", "hog_rk.h")]


def zone_rate(zones, ms_per_step):
    """Zone updates per second of steps over `zones` zones taking ms_per_step each."""
    return zones / (ms_per_step * 1e-3)


def _binom(n, k):
    return math.comb(n, k)


def spatial_eval_fma(D, L, N1):
    """FMAs to evaluate (or, transposed, to project onto) the total-degree-L
    spatial modes at the N1^D tensor Gauss nodes by sum factorisation."""
    if D == 3:
        return N1 * _binom(L + 3, 3) + N1 ** 2 * _binom(L + 2, 2) + N1 ** 3 * (L + 1)
    return N1 * _binom(L + 2, 2) + N1 ** 2 * (L + 1)


def needed_proj_fma(D, L, N1):
    """FMAs to project one flux row onto the coefficients its derivative needs:
    degree >= 1 along the derivative axis and total degree <= L, by sum
    factorisation with the derivative axis contracted first."""
    if D == 3:
        return N1 ** 3 * L + N1 ** 2 * (L * (L + 1) // 2) + N1 * _binom(L + 2, 3)
    return N1 ** 2 * L + N1 * (L * (L + 1) // 2)


def predictor_flops(D, P):
    """Algorithmic flops of the ADER predictor for one zone (FMA = 2).

    Formulation: P Picard iterations; the first on the spatial nodes only
    (the initial iterate does not depend on time), the others on the
    (P+1)^(D+1) space-time Gauss nodes: evaluate the space-time modes by sum
    factorisation (spatial transform of each time mode, Horner in time),
    physical fluxes of all D axes, contraction against the P time modes that
    feed a derivative, and for each (axis d, flux time mode e, variable) the
    L2 projection onto the only coefficients the update uses (degree >= 1
    along d, total space-time degree <= P), the derivative along d and the
    time-integral assembly of the new modes; then the face-point states
    (normal-axis contraction, tangential x time transform at 2^D points) for
    the Riemann solver.  Division counted as one flop.
    """
    N1, NV = P + 1, D + 2
    ns, nst = _binom(P + D, D), _binom(P + D + 1, D + 1)
    flux_node = D * D + 5 * D + 5                 # 1/rho, velocities, pressure, D flux vectors
    total = 0
    for it in range(P):
        if it == 0:
            ev = spatial_eval_fma(D, P, N1) * NV
            nodes = N1 ** D
            ne = 1
            tcon = 0
        else:
            ev = (sum(spatial_eval_fma(D, P - e, N1) for e in range(P + 1)) + N1 ** (D + 1) * P) * NV
            nodes = N1 ** (D + 1)
            ne = P
            tcon = nodes * D * ne * NV                # FMAs
        proj = D * NV * sum(needed_proj_fma(D, P - e, N1) for e in range(ne))
        # derivative along d of the kept coefficients: one FMA per (hi > lo) pair
        deriv = 0
        for e in range(ne):
            L = P - e
            for s in range(L):                     # s = degree along the other axes
                nother = s + 1 if D == 3 else 1
                deriv += nother * sum(L - s - lo for lo in range(L - s))
        deriv *= D * NV
        # time-integral assembly: one FMA per (axis, flux time mode, target) term
        asm = D * (nst - ns) * NV * P
        total += 2 * (ev + tcon + proj + deriv + asm) + nodes * flux_node
    # face-point states: per face side contract the normal axis, then the
    # (D-1 spatial + time) polynomial of degree P at 2^D points
    face_side = nst + sum(2 ** (k + 1) * _binom(P + D - k, D - k) for k in range(D))
    total += 2 * D * 2 * face_side * NV
    return total


def o2_flops(D, n, solver="hll"):
    """Algorithmic FP64 operations of one second-order step of an n^D periodic
    grid (each add, mul, div, sqrt, min, max, abs-scale counts 1, an FMA 2):

    modes, on the interior grown by one zone per axis (their faces bound the
    interior): per axis and variable the MC slope (two differences, the sum,
    its half, two compression products, two mins: 8), the face-centre values
    U -+ S/2 (2 x 2), two physical fluxes (3D + 8 each: 1/rho, kinetic
    energy, pressure, normal velocity, momentum and energy fluxes) and the
    time-mode sum lam (Fp - Fm) (3 per variable); face states U -+ S/2 + U5/2
    (3 per variable and face, plus U5/2) and their pressures for the
    admissibility check (2D + 3 each);
    Riemann problems, one per face ((n + 1) n^(D-1) per axis): HLL with
    Einfeldt-Roe bounds = two fluxes, two sound speeds, the Roe averages and
    bounds, and the HLL combination (7 per variable);
    update and CFL, per interior zone: three operations per axis and variable
    and the signal speed (3D + 8)."""
    NV = D + 2
    flux = 3 * D + 8
    per_axis = 15 * NV + 2 * flux
    modes = D * per_axis + 2 * D * NV * 3 + NV + 2 * D * (2 * D + 3)
    riem = {"hll": 2 * flux + 6 + 2 + 2 + 4 + 4 * D + (2 * D - 1) + 4 + 4 + 6 + 2 + 7 * NV + 1}[solver]
    upd = 3 * D * NV + 3 * D + 8
    zones_m = (n + 2) ** D
    faces = D * (n + 1) * n ** (D - 1)
    return modes * zones_m + riem * faces + upd * n ** D


def kernel_hash(sources=KERNEL_SOURCES):
    h = hashlib.sha256()
    for f in sources:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(second_order=False, kind=None):
    """HBM bytes per launch of the dominant kernel (the predictor, the fused
    second-order kernel, or with kind="rk" the Runge-Kutta face-point kernel)
    measured with rocprofv3 counters, if the kernel sources have not changed
    since they were taken."""
    path, src = (TRAFFIC_FILE_O2, KERNEL_SOURCES_O2) if second_order else (TRAFFIC_FILE, KERNEL_SOURCES)
    if kind == "rk":
        path, src = TRAFFIC_FILE_RK, KERNEL_SOURCES_RK
    if kind == "c5":
        path = TRAFFIC_FILE_C5
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash(src):
        return None
    return rec.get("bytes_per_launch")


PMC_COMMAND = ("export TMPDIR=/tmp; timeout -s KILL 240 rocprofv3 --pmc {ctr} --kernel-include-regex "
               "\"k_predict|elementwise\" -f csv -d gpurun_out/prof_{tag} -o {tag} -- python3 bench.py --vortex128 "
               "--steps 2 --warmup 0 --no-cpu-baseline --no-mixed --copy-calibration")
PMC_COMMAND_C5 = ("export TMPDIR=/tmp; timeout -s KILL 300 rocprofv3 --pmc {ctr} --kernel-include-regex "
                  "\"k_predict|elementwise\" -f csv -d gpurun_out/prof_{tag} -o {tag} -- python3 bench.py --steps 1 "
                  "--warmup 0 --no-cpu-baseline --no-mixed --no-vortex128 --copy-calibration")
PMC_COMMAND_RK = ("export TMPDIR=/tmp; timeout -s KILL 300 rocprofv3 --pmc {ctr} --kernel-include-regex "
                  "\"k_face_points|elementwise\" -f csv -d gpurun_out/prof_{tag} -o {tag} -- python3 bench.py "
                  "--ader-vs-rk --steps 1 --copy-calibration")
PMC_COMMAND_O2 = ("export TMPDIR=/tmp; timeout -s KILL 240 rocprofv3 --pmc {ctr} --kernel-include-regex "
                  "\"k_o2_step|elementwise\" -f csv -d gpurun_out/prof_{tag} -o {tag} -- python3 bench.py "
                  "--second-order --steps 3 --warmup 0 --no-cpu-baseline --copy-calibration")


def write_traffic(fetch_csv, write_csv, n=128, second_order=False, kind=None):
    """Traffic record of the FP64 predictor (or of the fused second-order
    kernel) from two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE, KiB
    per dispatch) of this script with --copy-calibration: each counter is
    scaled by what it reads for the plain copy of 2^27 doubles (1 GiB read,
    1 GiB written) in the same run."""
    kname = "k_o2_step<3" if second_order else "k_predict<3, 3, double>"
    if kind == "rk":
        kname = "k_face_points<3, 3>"
    import csv
    from collections import defaultdict

    def per_dispatch(path, counter):
        acc = defaultdict(float)
        names = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                acc[r["Dispatch_Id"]] += float(r["Counter_Value"])
                names[r["Dispatch_Id"]] = r["Kernel_Name"]
        pred = [v * 1024 for d, v in acc.items() if kname in names[d]]
        copy = [v * 1024 for d, v in acc.items() if "MulFunctor" in names[d]]   # the x * 1.0 copies
        if not pred or not copy:
            raise SystemExit(f"{path}: no {kname} or copy dispatch with {counter}")
        return sum(pred) / len(pred), sum(copy) / len(copy)

    gib = float(1 << 30)
    fetch, fcopy = per_dispatch(fetch_csv, "FETCH_SIZE")
    write, wcopy = per_dispatch(write_csv, "WRITE_SIZE")
    fs, ws = gib / fcopy, gib / wcopy
    if kind == "rk":
        rec = {
            "kernel": "k_face_points<3, 3> (Runge-Kutta face points, fourth order, FP64)",
            "workload": f"3D vortex + density modes, {n}^3, order 4, SSP-RK(5,4)",
            "kernel_hash": kernel_hash(KERNEL_SOURCES_RK),
            "bytes_per_launch": fetch * fs + write * ws,
            "fetch_bytes_per_launch": fetch * fs,
            "write_bytes_per_launch": write * ws,
            "fetch_scale": fs,
            "write_scale": ws,
            "algorithmic_bytes_per_launch": (n + 2) ** 3 * (20 + 24) * 5 * 8,
            "commands": [PMC_COMMAND_RK.format(ctr="FETCH_SIZE", tag="rkfetch"),
                         PMC_COMMAND_RK.format(ctr="WRITE_SIZE", tag="rkwrite")],
            "calibration": "plain elementwise copy of 2^27 doubles (1 GiB read + 1 GiB written) in the same runs",
        }
        with open(TRAFFIC_FILE_RK, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec, indent=1))
        return
    if second_order:
        rec = {
            "kernel": "k_o2_step<3, HLL> (fused second-order step, FP64)",
            "workload": f"3D vortex + density modes, {n}^3, order 2, HLL",
            "kernel_hash": kernel_hash(KERNEL_SOURCES_O2),
            "bytes_per_launch": fetch * fs + write * ws,
            "fetch_bytes_per_launch": fetch * fs,
            "write_bytes_per_launch": write * ws,
            "fetch_scale": fs,
            "write_scale": ws,
            "algorithmic_bytes_per_launch": n ** 3 * 5 * 8 * 2,
            "commands": [PMC_COMMAND_O2.format(ctr="FETCH_SIZE", tag="fetch"),
                         PMC_COMMAND_O2.format(ctr="WRITE_SIZE", tag="write")],
            "calibration": "plain elementwise copy of 2^27 doubles (1 GiB read + 1 GiB written) in the same runs",
        }
        with open(TRAFFIC_FILE_O2, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec, indent=1))
        return
    zones = (n + 2) ** 3
    if kind == "c5":
        rec = {
            "kernel": "k_predict<3,3> (FP64)",
            "workload": f"four-quadrant Riemann problem, {n}^3 outflow, order 4",
            "kernel_hash": kernel_hash(),
            "bytes_per_launch": fetch * fs + write * ws,
            "fetch_bytes_per_launch": fetch * fs,
            "write_bytes_per_launch": write * ws,
            "fetch_scale": fs,
            "write_scale": ws,
            "algorithmic_bytes_per_launch": zones * (20 + 48) * 5 * 8,
            "commands": [PMC_COMMAND_C5.format(ctr="FETCH_SIZE", tag="c5fetch"),
                         PMC_COMMAND_C5.format(ctr="WRITE_SIZE", tag="c5write")],
            "calibration": "plain elementwise copy of 2^27 doubles (1 GiB read + 1 GiB written) in the same runs",
        }
        with open(TRAFFIC_FILE_C5, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec, indent=1))
        return
    rec = {
        "kernel": "k_predict<3,3> (FP64)",
        "workload": f"3D vortex + density modes, {n}^3, order 4",
        "kernel_hash": kernel_hash(),
        "bytes_per_launch": fetch * fs + write * ws,
        "fetch_bytes_per_launch": fetch * fs,
        "write_bytes_per_launch": write * ws,
        "fetch_scale": fs,
        "write_scale": ws,
        "algorithmic_bytes_per_launch": zones * (20 + 48) * 5 * 8,
        "commands": [PMC_COMMAND.format(ctr="FETCH_SIZE", tag="fetch"),
                     PMC_COMMAND.format(ctr="WRITE_SIZE", tag="write")],
        "calibration": "plain elementwise copy of 2^27 doubles (1 GiB read + 1 GiB written) in the same runs",
    }
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


def cpu_baseline_o2(seconds, n=64):
    """The CPU oracle's second-order scheme timed on this host on a bounded
    sample: whole steps of the same 3D workload at 64^3."""
    import icgen
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    os.environ["OMP_NUM_THREADS"] = str(threads)
    pb = icgen.vortex3d_perturbed(n=n, seed=2)
    c = oracle.cfg_from_problem(pb, 2, riemann="hll")
    U = pb.U
    dt, _ = oracle.cfl_dt(c, U)
    steps = 0
    t0 = time.perf_counter()
    while True:
        U = oracle.step(c, U, dt)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 200:
            break
    return {"value": n ** 3 * steps / el, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"{steps} full second-order steps of the same 3D workload at {n}^3 "
                      f"({el:.1f} s, OpenMP threads={threads})"}


def second_order_line(hog, torch, args):
    """Benchmark line of the second-order scheme (Figs. 3-7, HLL) on the same
    128^3 workload: one fused kernel per step; roofline of that kernel against
    its operation count (o2_flops) and its compulsory HBM bytes (state read
    once, new state written once: 80 B per zone)."""
    import icgen
    n = args.n
    pb = icgen.vortex3d_perturbed(n=n, seed=2)
    g = hog.Grid.from_problem(pb, 2, riemann="hll")
    if args.warmup > 0:
        g.advance(args.warmup)
    g.set_state(pb.U)
    torch.cuda.synchronize()
    g.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.advance(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.profile_read()
    g.profile(False)
    g.close()
    elapsed = t1 - t0
    zones = n ** 3
    k_ms, k_calls = prof["predictor"]
    avg_s = k_ms / 1e3 / max(k_calls, 1)
    flops = o2_flops(3, n)
    achieved = flops / avg_s / 1e12
    hbm_bytes = zones * 5 * 8 * 2
    out = {
        "metric": METRIC, "value": zones * args.steps / elapsed, "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"3D Euler isentropic vortex extruded along z + seeded density modes "
                               f"(amp 1e-2, 4 per axis), {n}^3 periodic [0,10]^3, second-order scheme of "
                               f"Figs. 3-7 (MC limiter 2/1.5, Hancock time mode, midpoint HLL), CFL 0.4, FP64",
                   "zones": zones, "order": 2, "riemann": "hll", "precision": "fp64"},
        "roofline": {"bound": "alu", "kernel": "k_o2_step (fused second-order step)", "achieved": achieved,
                     "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU_TFLOPS,
                     "traffic": traffic_record(second_order=True), "alg_flops_per_launch": flops, "alg_flops_per_zone": flops / zones,
                     "avg_launch_ms": avg_s * 1e3,
                     "hbm": {"alg_bytes_per_launch": hbm_bytes, "achieved_GBps": hbm_bytes / avg_s / 1e9,
                             "peak_GBps": 8000.0, "frac": hbm_bytes / avg_s / 8e12}},
        "stages_ms_per_launch": {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items()},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_o2(args.cpu_seconds)
    return out


def ader_vs_rk(hog, torch, args):
    """Table IV on one MI355X: zone-updates/s of the ADER step and of the
    Runge-Kutta scheme of the same order (2, 3, 5 stages; same reconstruction
    and HLLC solver, face points in space only) on the 128^3 workload, FP64,
    with per-stage times of each (ms per step, HIP events)."""
    import icgen
    n = args.n
    pb = icgen.vortex3d_perturbed(n=n, seed=2)
    rows = []
    for order, stepper in ((2, "rk2"), (3, "rk3"), (4, "rk4")):
        row = {"order": order}
        # second-order steps take a fraction of a millisecond: time 10x as many so
        # that the timed region is long against the GPU's clock ramp
        steps = args.steps * (10 if order == 2 else 1)
        for st in ("ader", stepper):
            g = hog.Grid.from_problem(pb, order, stepper=st)
            g.advance(steps // 2)
            g.set_state(pb.U)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.advance(steps)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            # stage breakdown from a separate run with the library's HIP events
            g.set_state(pb.U)
            g.profile(True)
            g.advance(steps)
            prof = g.profile_read()
            g.profile(False)
            g.close()
            key = "ader" if st == "ader" else "rk"
            row[key] = {"stepper": st, "steps": steps, "zone_updates_per_s": n ** 3 * steps / el,
                        "ms_per_step": el * 1e3 / steps,
                        "stage_ms_per_step": {k: round(v[0] / steps, 4) for k, v in prof.items() if v[1]}}
        row["ader_over_rk"] = row["ader"]["zone_updates_per_s"] / row["rk"]["zone_updates_per_s"]
        if order >= 3:
            # dominant Runge-Kutta kernels at third/fourth order: the face-point
            # evaluation (the "predictor" stage slot) and the reconstruction, both
            # HBM-bound; roofline of the face-point kernel: per zone of the grown
            # box it reads the spatial modes once and writes the face states once
            from math import comb
            ns, npt = comb(order - 1 + 3, 3), 2 * 3 * 4
            zones_r = (n + 2) ** 3
            alg = zones_r * (ns + npt) * 5 * 8
            nst = {"rk2": 2, "rk3": 3, "rk4": 5}[stepper]
            t = row["rk"]["stage_ms_per_step"]["predictor"] / nst / 1e3
            row["rk"]["roofline"] = {"bound": "hbm", "kernel": f"k_face_points<3, {order - 1}>",
                                     "achieved": alg / t / 1e9, "peak": 8000.0, "unit": "GB/s",
                                     "frac": alg / t / 8e12,
                                     "traffic": traffic_record(kind="rk") if order == 4 else None,
                                     "alg_bytes_per_launch": alg, "avg_launch_ms": t * 1e3}
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    return {"metric": "zone-updates/s, ADER vs SSP Runge-Kutta of the same order (Table IV)", "unit": UNIT,
            "n_gpus": 1, "steps": args.steps, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"3D vortex + density modes, {n}^3 periodic, HLLC, CFL 0.4, FP64; "
                                   "second order: MC slopes (Hancock step for ADER), third/fourth: WENO"},
            "rows": rows}


def host_round_trip(hog, torch, args):
    """The paper's per-step host round trip of the zone means (its U_skinny
    array, Figs. 1-2, Table II) on one MI355X: each step copies the zone means
    host -> device (pinned host buffer, zone-major [z][y][x][v] as U_skinny),
    takes the step with the dt of the previous one, reads dt_next and copies the
    new zone means back.  Against the resident loop (state stays in HBM)."""
    import icgen
    n = args.n
    pb = icgen.vortex3d_perturbed(n=n, seed=2)
    out = {"metric": "zone-updates/s with and without the per-step host round trip of the zone means",
           "unit": UNIT, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"3D vortex + density modes, {n}^3 periodic, FP64, CFL 0.4"}, "rows": []}
    for order, riemann in ((4, "hllc"), (2, "hll")):
        steps = args.steps * (10 if order == 2 else 1)
        g = hog.Grid.from_problem(pb, order, riemann=riemann)
        host = torch.from_numpy(np.ascontiguousarray(np.moveaxis(pb.U, 0, -1))).pin_memory()
        hp = C.c_void_p(host.data_ptr())
        lib = hog.load()
        dt = g.compute_dt()
        for _ in range(3):                       # warm-up of the same loop
            dt = g.step(dt)
        g.set_state(pb.U)
        dt = g.compute_dt()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            hog._check(lib.hog_set_state(g._h, hp, hog.AOS, hog.HOST))
            dt = g.step(dt)
            hog._check(lib.hog_get_state(g._h, hp, hog.AOS, hog.HOST))
        torch.cuda.synchronize()
        rt = time.perf_counter() - t0
        g.set_state(pb.U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.advance(steps)
        torch.cuda.synchronize()
        res = time.perf_counter() - t0
        g.close()
        nbytes = n ** 3 * 5 * 8
        out["rows"].append({"order": order, "riemann": riemann, "steps": steps,
                            "resident_zone_updates_per_s": n ** 3 * steps / res, "resident_ms_per_step": res * 1e3 / steps,
                            "round_trip_zone_updates_per_s": n ** 3 * steps / rt, "round_trip_ms_per_step": rt * 1e3 / steps,
                            "bytes_each_way_per_step": nbytes,
                            "transfer_ms_per_step": (rt - res) * 1e3 / steps})
        print(json.dumps(out["rows"][-1]), file=sys.stderr, flush=True)
    return out


def stream_vs_in_core(hog, torch, args):
    """A host-resident mesh stepped through the GPU in slabs (hog_stream_*)
    against the same mesh in core: 256^3 3D workload, fourth order (HLLC) and
    second order (HLL), FP64, slabs of 32 planes; the copies of one slab
    overlap the step of the other, so the streamed rate is bounded by the
    larger of compute and PCIe time."""
    import icgen
    n = 256
    pb = icgen.vortex3d_perturbed(n=n, seed=2)
    out = {"metric": "zone-updates/s, host-resident mesh streamed in slabs vs in core", "unit": UNIT, "n_gpus": 1,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"3D vortex + density modes, {n}^3 periodic, FP64, CFL 0.4, slabs of 32 planes"},
           "rows": []}
    for order, riemann, steps in ((4, "hllc", 5), (2, "hll", 20)):
        g = hog.Grid.from_problem(pb, order, riemann=riemann)
        dt = g.compute_dt()
        g.advance(2)
        g.set_state(pb.U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.advance(steps)
        torch.cuda.synchronize()
        t_in = (time.perf_counter() - t0) / steps
        g.close()
        del g
        torch.cuda.empty_cache()
        st = hog.Stream.from_problem(pb, order, 32, riemann=riemann)
        st.step(dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st.step(0.0)
        t_st = (time.perf_counter() - t0) / steps
        st.close()
        del st
        torch.cuda.empty_cache()
        nbytes = n ** 3 * 5 * 8
        moved = nbytes * (1 + 6 / 32) + nbytes           # slabs with ghost layers in, interiors out
        row = {"order": order, "riemann": riemann, "steps": steps, "slab_planes": 32,
               "in_core_zone_updates_per_s": n ** 3 / t_in, "in_core_ms_per_step": t_in * 1e3,
               "streamed_zone_updates_per_s": n ** 3 / t_st, "streamed_ms_per_step": t_st * 1e3,
               "bytes_moved_per_step": moved, "pcie_GBps_if_transfer_bound": moved / t_st / 1e9}
        out["rows"].append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    return out


def rank_block(hog, torch, args):
    """One rank's share of the 384^3 four-quadrant problem split 2 x 2 x 2 over
    eight devices: the 192^3 centre block with every axis external, its three
    ghost layers on all sides cut from the whole state (what the neighbouring
    blocks would send: 27.4 MB per step). Timed: the FP64 step of the block
    (ghosts as given; a real rank refreshes them between steps) and the device
    copy that packs a block with its ghost layers (hog_set_state_ext from
    device memory), against the same block stepped as a standalone outflow grid."""
    import icgen
    N, m, g3 = C5_N, C5_N // 2, 3
    lo = (N - m) // 2
    pb = icgen.four_quadrant(n=N, seed=5, block=(lo - g3, m + 2 * g3))
    pin = icgen.four_quadrant(n=N, seed=5, block=(lo, m))
    steps = max(3, min(args.steps, 10))
    ext = torch.from_numpy(np.ascontiguousarray(pb.U)).cuda()
    out = {"metric": "zone-updates/s, one rank's block with every axis external", "unit": UNIT, "n_gpus": 1,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"centre {m}^3 block of the {N}^3 four-quadrant Riemann problem (2 x 2 x 2 split), "
                                  "order 4 WENO+ADER, HLLC, FP64, ghost layers from the whole state"}}
    g = hog.Grid(3, (m, m, m), 4, pin.h, gamma=pin.gamma, bc=("external",) * 3)
    g.set_state_ext(ext)
    dt = g.compute_dt()
    g.step(dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.set_state_ext(ext)
    torch.cuda.synchronize()
    t_pack = (time.perf_counter() - t0) / steps
    g.set_state_ext(ext)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.step(dt, want_next=False)
    torch.cuda.synchronize()
    t_ext = (time.perf_counter() - t0) / steps
    g.close()
    del g
    torch.cuda.empty_cache()
    h = hog.Grid.from_problem(pin, 4)
    h.step(dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        h.step(dt, want_next=False)
    torch.cuda.synchronize()
    t_out = (time.perf_counter() - t0) / steps
    h.close()
    ghost_bytes = ((m + 2 * g3) ** 3 - m ** 3) * 5 * 8
    out.update({"value": m ** 3 / t_ext, "ms_per_step": t_ext * 1e3, "steps": steps,
                "standalone_outflow_ms_per_step": t_out * 1e3,
                "pack_with_ghosts_ms": t_pack * 1e3, "ghost_bytes_per_step": ghost_bytes,
                "zones": m ** 3})
    return out


def cpu_baseline(order, seconds):
    """The CPU oracle (plain FP64 C, OpenMP over zones) timed on this host on a
    bounded sample: whole steps of the same 3D workload at 32^3 (per-zone work
    of the scheme does not depend on the grid size)."""
    import icgen
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    os.environ["OMP_NUM_THREADS"] = str(threads)
    n = 32
    pb = icgen.vortex3d_perturbed(n=n, seed=2)
    c = oracle.cfg_from_problem(pb, order)
    U = pb.U
    dt, _ = oracle.cfl_dt(c, U)
    steps = 0
    t0 = time.perf_counter()
    while True:
        U = oracle.step(c, U, dt)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 50:
            break
    return {"value": n ** 3 * steps / el, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"{steps} full fourth-order steps of the same 3D workload at {n}^3 "
                      f"({el:.1f} s, OpenMP threads={threads})"}


GATE_FILE = os.path.join(ROOT, "paper_2211_13295_amd", "gate_o4_3d.npz")


def mixed_run(hog, torch, pb, order, steps, ref, gate=None):
    """Same workload on the mixed path (FP32 reconstruction / predictor / face
    states / Riemann solver, FP64 weights, face sum, update and CFL), timed the
    same way; L1 against the FP64 path's state after the same steps (that path
    matches the FP64 CPU oracle to 1e-12 relative L1 in the parity tests)."""
    import numpy as np
    g = hog.Grid.from_problem(pb, order, precision="mixed")
    if gate is not None:
        g.set_gate(gate[0], theta=gate[1])
    g.advance(2)
    g.set_state(pb.U)
    torch.cuda.synchronize()
    g.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.advance(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = g.profile_read()
    g.profile(False)
    U = g.get_state()
    rel = float(np.abs(U - ref).sum() / np.abs(ref).sum())
    rho_l1 = float(np.abs(U[0] - ref[0]).mean())
    out = {"value": pb.U[0].size * steps / el, "unit": UNIT, "ms_per_step": el * 1e3 / steps,
           "dtype": "f32+f64", "rel_l1_vs_fp64": rel, "density_l1_vs_fp64": rho_l1,
           "stages_ms_per_step": {k: round(v[0] / steps, 4) for k, v in prof.items()}}
    if gate is not None:
        _, flags = g.gate_eval()
        out["gate_theta"] = gate[1]
        out["gated_fraction_final_state"] = float(flags.mean())
    g.close()
    return out


def shock_workload(hog, torch, name, steps, timed_steps):
    """Accuracy and throughput of the mixed FP32/FP64 path on a shock workload
    at full size, against the FP64 path (which matches the FP64 CPU oracle on
    sampled zones of the same first step in the parity tests).  Both paths take
    the FP64 run's time steps, so their states compare at the same times; the
    throughput runs use the device-side time step."""
    import icgen
    import numpy as np
    if name == "multiblast256":
        pb, label, gate = icgen.multiblast(n=256, seed=3), "multi-blast 256^3 outflow", None
    else:
        pb, label = icgen.four_quadrant(n=384, seed=5), "four-quadrant Riemann problem 384^3 outflow"
        z = np.load(GATE_FILE)
        gate = (z["params"], float(z["theta"]))
    order = 4
    zones = pb.U[0].size

    def timed(precision, with_gate):
        g = hog.Grid.from_problem(pb, order, precision=precision)
        if with_gate:
            g.set_gate(gate[0], theta=gate[1])
        g.advance(1)
        g.set_state(pb.U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.advance(timed_steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        g.close()
        torch.cuda.empty_cache()
        return zones * timed_steps / el, el * 1e3 / timed_steps

    def stepped(precision, with_gate, dts=None):
        g = hog.Grid.from_problem(pb, order, precision=precision)
        if with_gate:
            g.set_gate(gate[0], theta=gate[1])
        out = []
        dt = g.compute_dt() if dts is None else dts[0]
        for s in range(steps):
            if dts is not None:
                dt = dts[s]
            out.append(dt)
            nxt = g.step(dt)
            dt = nxt
            if (s + 1) % 25 == 0:
                print(f"{name} {precision}: step {s + 1}/{steps}", file=sys.stderr, flush=True)
        U = g.get_state()
        g.close()
        torch.cuda.empty_cache()
        return U, out

    v64, ms64 = timed("fp64", False)
    vmx, msmx = timed("mixed", gate is not None)
    ref, dts = stepped("fp64", False)
    U, _ = stepped("mixed", gate is not None, dts)
    rel = float(np.abs(U - ref).sum() / np.abs(ref).sum())
    rho = float(np.abs(U[0] - ref[0]).mean())
    return {"workload": label, "order": order, "zones": zones, "steps_compared": steps,
            "fp64": {"value": v64, "unit": UNIT, "ms_per_step": ms64},
            "mixed" + ("_gated" if gate is not None else ""): {
                "value": vmx, "unit": UNIT, "ms_per_step": msmx,
                "rel_l1_vs_fp64": rel, "density_l1_vs_fp64": rho, "t_end": float(sum(dts))},
            "timed_steps": timed_steps}


def gate_ablation(hog, torch, name, steps, timed_steps, label_samples=1_000_000):
    """The gate's speed-up at equal accuracy on a full-size shock workload,
    mixed FP32/FP64 path, four variants on the same time steps (those of the
    FP64 run): (A) full WENO, (B) the trained gate, (C) linear weights in
    every zone, (D) a fresh random selection each step with B's smooth
    fraction.  Per variant: ms per step (device-side time step), relative L1
    against the FP64 path, smooth fraction, and for B and D the false-smooth
    rate against full-WENO labels (weight deviation > 0.25) on sampled zones of
    the final state.  Also the Amdahl ceiling from the stage times of A."""
    import icgen
    import numpy as np
    pb = icgen.multiblast(n=256, seed=3) if name == "multiblast256" else icgen.four_quadrant(n=384, seed=5)
    label = "multi-blast 256^3 outflow" if name == "multiblast256" else "four-quadrant Riemann problem 384^3 outflow"
    z = np.load(GATE_FILE)
    params, theta = z["params"], float(z["theta"])
    order, zones = 4, pb.U[0].size
    rng = np.random.default_rng(7)

    def free(g):
        g.close()
        torch.cuda.empty_cache()

    # FP64 reference and its time steps
    g = hog.Grid.from_problem(pb, order)
    dts, dt = [], g.compute_dt()
    for s in range(steps):
        dts.append(dt)
        dt = g.step(dt)
        if (s + 1) % 50 == 0:
            print(f"ablation {name} fp64: step {s + 1}/{steps}", file=sys.stderr, flush=True)
    ref = g.get_state()
    free(g)

    def setup(g, variant, frac):
        if variant == "B":
            g.set_gate(params, theta=theta)
        elif variant == "C":
            g.set_gate_flags(np.ones(pb.U[0].shape, np.uint8))
        elif variant == "D":
            g.set_gate_flags((rng.uniform(size=pb.U[0].shape) < frac).astype(np.uint8))

    out, frac_b, state_b, state_d = {}, 0.0, None, None
    for variant in ("A", "B", "C", "D"):
        g = hog.Grid.from_problem(pb, order, precision="mixed")
        setup(g, variant, frac_b)
        g.profile(True)
        t0 = time.perf_counter()
        try:
            g.advance(timed_steps)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / timed_steps
        except hog.HogError as e:
            ms = None
            print(f"ablation {name} {variant}: timed run stopped: {e}", file=sys.stderr, flush=True)
        prof = g.profile_read()
        g.profile(False)
        g.set_state(pb.U)
        fracs, failed = [], None
        for s in range(steps):
            if variant == "B" and s % 25 == 0:
                fracs.append(float(g.gate_eval()[1].mean()))
            if variant == "D":
                g.set_gate_flags((rng.uniform(size=pb.U[0].shape) < frac_b).astype(np.uint8))
            try:
                g.step(dts[s])
            except hog.HogError as e:
                failed = f"step {s + 1}: {e}"
                break
            if (s + 1) % 50 == 0:
                print(f"ablation {name} {variant}: step {s + 1}/{steps}", file=sys.stderr, flush=True)
        rec = {"ms_per_step": ms, "zone_updates_per_s": zones / ms * 1e3 if ms else None}
        if failed:
            rec["failed"] = failed
        else:
            U = g.get_state()
            rec["rel_l1_vs_fp64"] = float(np.abs(U - ref).sum() / np.abs(ref).sum())
            rec["density_l1_vs_fp64"] = float(np.abs(U[0] - ref[0]).mean())
            if variant == "B":
                state_b = U
            if variant == "D":
                state_d = U
        if variant == "A":
            rec["stages_ms_per_step"] = {k: round(v[0] / timed_steps, 4) for k, v in prof.items()}
        if variant == "B":
            frac_b = float(np.mean(fracs))
            rec["gate_ms_per_step"] = round(prof["gate"][0] / timed_steps, 4)
        rec["smooth_fraction"] = {"A": 0.0, "B": frac_b, "C": 1.0, "D": frac_b}[variant]
        out[variant] = rec
        free(g)

    # false-smooth rates on sampled zones of the final states, labels from full WENO (FP64 weights)
    sample = np.sort(rng.choice(zones, min(label_samples, zones), replace=False))
    for variant, U in (("B", state_b), ("D", state_d)):
        if U is None:
            continue
        g = hog.Grid.from_problem(pb, order)
        g.set_state(U)
        _, dev = g.harvest(sample)
        nonsmooth = dev.cpu().numpy() > 0.25
        if variant == "B":
            g.set_gate(params, theta=theta)
            flags = g.gate_eval()[1].reshape(-1)[sample] > 0
        else:
            flags = rng.uniform(size=sample.size) < frac_b
        out[variant]["false_smooth_rate"] = float((flags & nonsmooth).sum() / max(1, nonsmooth.sum()))
        out[variant]["nonsmooth_fraction_final"] = float(nonsmooth.mean())
        free(g)
    a = out["A"]["stages_ms_per_step"]
    step_ms = sum(a.values())
    out["amdahl_ceiling"] = {"reconstruction_share": a["reconstruction"] / step_ms,
                             "speedup_if_reconstruction_were_free": step_ms / (step_ms - a["reconstruction"])}
    return {"workload": label, "order": order, "zones": zones, "steps_compared": steps, "timed_steps": timed_steps,
            "path": "mixed FP32/FP64", "gate_theta": theta, "variants": out}


def vortex128_line(hog, torch, args, n=128):
    """The 128^3 vortex workload (3D isentropic vortex extruded along z with
    seeded density modes, periodic [0,10]^3, fourth order, HLLC, FP64), with
    the mixed path and the gated mixed path on the same steps."""
    import icgen
    order = args.order
    pb = icgen.vortex3d_perturbed(n=n, seed=2)
    g = hog.Grid.from_problem(pb, order)
    if args.warmup > 0:
        g.advance(args.warmup)
    g.set_state(pb.U)
    torch.cuda.synchronize()
    g.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.advance(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = g.profile_read()
    g.profile(False)
    elapsed = t1 - t0
    zones = n ** 3
    value = zones * args.steps / elapsed
    ms_step = elapsed * 1e3 / args.steps
    # run-to-run spread: four more timed runs of the same K steps from the same state
    reps = [ms_step]
    for _ in range(4):
        g.set_state(pb.U)
        torch.cuda.synchronize()
        r0 = time.perf_counter()
        g.advance(args.steps)
        torch.cuda.synchronize()
        reps.append((time.perf_counter() - r0) * 1e3 / args.steps)
    reps_sorted = sorted(reps)

    D, P = 3, order - 1
    zones_per_launch = (n + 2) ** 3                       # predictor runs on the interior grown by one zone
    pflops = predictor_flops(D, P) * zones_per_launch
    pred_ms, pred_calls = prof["predictor"]
    avg_s = pred_ms / 1e3 / max(pred_calls, 1)
    achieved = pflops / avg_s / 1e12
    traffic = traffic_record()
    stage_ms = {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items()}
    step_sum = sum(v[0] for v in prof.values()) / args.steps

    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"3D Euler isentropic vortex extruded along z + seeded density modes "
                               f"(amp 1e-2, 4 per axis), {n}^3 periodic [0,10]^3, order {order} "
                               f"WENO+ADER, HLLC, CFL 0.4, FP64",
                   "zones": zones, "order": order, "riemann": "hllc", "precision": "fp64"},
        "roofline": {"bound": "alu", "kernel": "k_predict (ADER predictor)", "achieved": achieved,
                     "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VALU_TFLOPS, "traffic": traffic,
                     "alg_flops_per_zone": predictor_flops(D, P), "zones_per_launch": zones_per_launch,
                     "avg_launch_ms": avg_s * 1e3},
        "stages_ms_per_launch": stage_ms,
        "repeats_ms_per_step": {"n": len(reps), "median": reps_sorted[len(reps) // 2], "min": reps_sorted[0],
                                "max": reps_sorted[-1]},
        "predictor_fraction_of_step": prof["predictor"][0] / args.steps / step_sum if step_sum > 0 else None,
    }
    ref = g.get_state()
    g.close()
    torch.cuda.empty_cache()
    if not args.no_mixed:
        out["mixed"] = mixed_run(hog, torch, pb, order, args.steps, ref)
        if os.path.exists(GATE_FILE):
            import numpy as np
            z = np.load(GATE_FILE)
            out["mixed_gated"] = mixed_run(hog, torch, pb, order, args.steps, ref,
                                           gate=(z["params"], float(z["theta"])))
    return out


def gate_train_throughput(hog, torch, args):
    """Training throughput of the gate network on the GPU's own kernels (BF16
    MFMA forward, backward and weight gradients, FP32 Adam): Adam steps on
    batches of 4096 samples drawn from stencils harvested from the 128^3
    vortex workload and the 128^3 multi-blast (FP64 runs, fourth order); one
    JSON line with samples/s."""
    import icgen
    feats, labels = [], []
    for pb in (icgen.vortex3d_perturbed(n=128, seed=2), icgen.multiblast(n=128, seed=3)):
        g = hog.Grid.from_problem(pb, 4)
        F, dev = g.harvest(np.arange(0, pb.U[0].size, 4))
        feats.append(F)
        labels.append((dev <= 0.25).float())
        g.close()
        torch.cuda.empty_cache()
    X = torch.cat(feats)
    y = torch.cat(labels)
    batch, steps = 4096, args.steps * 50
    m = hog.Mlp(X.shape[1], batch_max=batch)
    z = np.load(GATE_FILE)
    m.set_params(z["params"])
    gen = torch.Generator(device="cpu").manual_seed(0)
    idx = torch.randint(0, X.shape[0], (steps + 10, batch), generator=gen).cuda()
    batches = [(X[i].contiguous(), y[i].contiguous()) for i in idx[:16]]
    for k in range(10):
        m.step(*batches[k % 16], None, lr=1e-4, want_loss=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        m.step(*batches[k % 16], None, lr=1e-4, want_loss=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"metric": "gate training samples/s (Adam steps, batch 4096)", "value": steps * batch / el,
            "unit": "samples/s", "steps": steps, "ms_per_step": el * 1e3 / steps, "batch": batch,
            "features": int(X.shape[1]), "params": m.np,
            "data": "stencils harvested from the 128^3 vortex and multi-blast workloads (FP64, order 4)"}


def c5_cutout(m):
    """A bounded sample of the four-quadrant workload for the CPU oracle: the
    m^3 block of the 384^3 initial state around the domain centre, where the
    four quadrants meet, with outflow boundaries."""
    import icgen
    return icgen.four_quadrant(n=C5_N, seed=5, block=(C5_N // 2 - m // 2, m))


def cpu_sample(threads, seconds, m=32):
    """Child-process leg of the CPU baseline: the oracle (plain FP64 C,
    OpenMP over zones) on the m^3 cut-out of the four-quadrant workload,
    whole fourth-order steps until `seconds` have passed; prints one JSON line."""
    import oracle
    pb = c5_cutout(m)
    c = oracle.cfg_from_problem(pb, 4)
    U = pb.U
    dt, _ = oracle.cfl_dt(c, U)
    steps = 0
    t0 = time.perf_counter()
    while True:
        U = oracle.step(c, U, dt)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 200:
            break
    print(json.dumps({"value": m ** 3 * steps / el, "unit": UNIT, "cores": threads, "kind": "oracle",
                      "sample": f"{steps} fourth-order steps of the {m}^3 centre block of the 384^3 four-quadrant "
                                f"initial state (outflow), {el:.1f} s, OpenMP threads={threads}"}), flush=True)


def cpu_baseline_c5(seconds):
    """The CPU oracle timed on this host's cores on a bounded sample of the
    headline workload, with all host threads and with one; each in a child
    process started before this process touches the GPU (OMP_NUM_THREADS is
    read when the OpenMP runtime starts)."""
    import subprocess
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    out = {}
    for t in (threads, 1):
        env = dict(os.environ, OMP_NUM_THREADS=str(t))
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-sample", str(t),
                            "--cpu-seconds", str(seconds)], env=env, capture_output=True, text=True, check=True)
        out[t] = json.loads(r.stdout.strip().splitlines()[-1])
    res = dict(out[threads])
    res["single_thread"] = {"value": out[1]["value"], "cores": 1, "sample": out[1]["sample"]}
    return res


C5_N = 384


def headline(hog, torch, args, cpu):
    """The metric's workload: FP64 vs mixed FP32/FP64 with the trained gate on
    the 384^3 four-quadrant problem, fourth order, HLLC.

    FP64: a stepped run of K steps (host-read CFL time steps, recorded), then
    the timed runs of K steps with the device-side time step (the same steps:
    the CFL reduction is the same arithmetic on the same states).  Mixed with
    the gate, and mixed without it: timed the same way, then stepped with the
    FP64 run's time steps; relative L1 of each against the FP64 state after the
    same K steps (the FP64 path matches the FP64 CPU oracle on this workload
    to 1e-12: whole grid on a 96^3 version over 20 steps, sampled zones at
    384^3 over 5 steps, in the GPU parity tests)."""
    import icgen
    n, order, K = args.headline_n, 4, args.steps
    pb = icgen.four_quadrant(n=n, seed=5)
    zones = pb.U[0].size
    z = np.load(GATE_FILE)
    gate = (z["params"], float(z["theta"]))

    def free(g):
        g.close()
        torch.cuda.empty_cache()

    def timed(g, reps):
        g.set_state(pb.U)
        torch.cuda.synchronize()
        g.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.advance(K)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = g.profile_read()
        g.profile(False)
        ms = [el * 1e3 / K]
        for _ in range(reps - 1):
            g.set_state(pb.U)
            torch.cuda.synchronize()
            r0 = time.perf_counter()
            g.advance(K)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - r0) * 1e3 / K)
        return ms, prof

    def stepped(g, dts=None):
        g.set_state(pb.U)
        rec = []
        dt = g.compute_dt() if dts is None else dts[0]
        for s_ in range(K):
            if dts is not None:
                dt = dts[s_]
            rec.append(dt)
            dt = g.step(dt)
        return g.get_state(), rec

    # FP64
    print(f"headline: FP64 {n}^3, {K} steps", file=sys.stderr, flush=True)
    g = hog.Grid.from_problem(pb, order)
    if args.warmup > 0:
        g.advance(args.warmup)
    ref, dts = stepped(g)
    ms64, prof = timed(g, args.repeats)
    free(g)
    ms_step = ms64[0]
    value = zone_rate(zones, ms_step)
    srt = sorted(ms64)

    D, P = 3, order - 1
    zones_per_launch = (n + 2) ** 3
    pred_ms, pred_calls = prof["predictor"]
    avg_s = pred_ms / 1e3 / max(pred_calls, 1)
    achieved = PREDICTOR_FLOPS_ESTIMATE_3D_O4 * zones_per_launch / avg_s / 1e12
    achieved_exact = predictor_flops(D, P) * zones_per_launch / avg_s / 1e12
    stage_ms = {k: round(v[0] / max(v[1], 1), 4) for k, v in prof.items()}
    step_sum = sum(v[0] for v in prof.values()) / K

    def mixed(with_gate):
        tag = "mixed + gate" if with_gate else "mixed"
        print(f"headline: {tag} {n}^3, {K} steps", file=sys.stderr, flush=True)
        g = hog.Grid.from_problem(pb, order, precision="mixed")
        if with_gate:
            g.set_gate(gate[0], theta=gate[1])
        if args.warmup > 0:
            g.advance(args.warmup)
        ms, prof_m = timed(g, args.repeats)
        U, _ = stepped(g, dts)
        rec = {"value": zone_rate(zones, ms[0]), "unit": UNIT, "ms_per_step": ms[0],
               "repeats_ms_per_step": {"n": len(ms), "median": sorted(ms)[len(ms) // 2], "min": min(ms),
                                       "max": max(ms)},
               "dtype": "f32+f64",
               "rel_l1_vs_fp64": float(np.abs(U - ref).sum() / np.abs(ref).sum()),
               "density_l1_vs_fp64": float(np.abs(U[0] - ref[0]).mean()),
               "stages_ms_per_step": {k: round(v[0] / K, 4) for k, v in prof_m.items()}}
        if with_gate:
            _, flags = g.gate_eval()
            rec["gate_theta"] = gate[1]
            rec["gated_fraction_final_state"] = float(flags.mean())
        free(g)
        return rec

    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"3D Euler four-quadrant Riemann problem (quadrant states seeded: rho U[0.5,1.5], "
                               f"p U[0.1,1.0], in-plane speed U[0,0.5], seed 5), {n}^3 outflow [0,1]^3, order 4 "
                               f"WENO+ADER, HLLC, CFL 0.4, FP64 vs FP32+learned gate",
                   "zones": zones, "order": order, "riemann": "hllc", "precision": "fp64"},
        "roofline": {"bound": "alu", "kernel": "k_predict (ADER predictor, FP64)", "achieved": achieved,
                     "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VALU_TFLOPS, "traffic": traffic_record(kind="c5"),
                     "alg_flops_per_zone": PREDICTOR_FLOPS_ESTIMATE_3D_O4, "zones_per_launch": zones_per_launch,
                     "avg_launch_ms": avg_s * 1e3,
                     "exact_count": {"alg_flops_per_zone": predictor_flops(D, P), "achieved": achieved_exact,
                                     "frac": achieved_exact / PEAK_FP64_VALU_TFLOPS}},
        "stages_ms_per_launch": stage_ms,
        "repeats_ms_per_step": {"n": len(ms64), "median": srt[len(srt) // 2], "min": srt[0], "max": srt[-1]},
        "predictor_fraction_of_step": prof["predictor"][0] / K / step_sum if step_sum > 0 else None,
    }
    if not args.no_mixed:
        out["mixed_gated"] = mixed(True)
        out["mixed"] = mixed(False)
        out["gate_speedup_vs_mixed"] = out["mixed"]["ms_per_step"] / out["mixed_gated"]["ms_per_step"]
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if not args.no_vortex128:
        print("headline: 128^3 vortex workload", file=sys.stderr, flush=True)
        v = vortex128_line(hog, torch, args, n=128)
        out["vortex128"] = {k: v[k] for k in ("value", "ms_per_step", "config", "roofline", "stages_ms_per_launch",
                                              "repeats_ms_per_step") if k in v}
        for k in ("mixed", "mixed_gated"):
            if k in v:
                out["vortex128"][k] = v[k]
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--repeats", type=int, default=3, help="timed repetitions of the K steps (median/min/max)")
    ap.add_argument("--n", type=int, default=128, help="grid of the 128^3-workload legs")
    ap.add_argument("--headline-n", type=int, default=C5_N, help="grid of the four-quadrant headline workload")
    ap.add_argument("--vortex128", action="store_true",
                    help="instead of the headline: the 128^3 vortex workload line (FP64, mixed, mixed + gate)")
    ap.add_argument("--no-vortex128", action="store_true", help="leave the 128^3 vortex figures out of the line")
    ap.add_argument("--cpu-sample", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--order", type=int, default=4)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed FP32/FP64 comparison run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain elementwise copy of 2 x 1 GiB (known bytes) to "
                         "calibrate the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--shock-workload", choices=["multiblast256", "fourquad384"],
                    help="instead of the benchmark line: mixed (with the trained gate on the four-quadrant "
                         "problem) vs FP64 on a full-size shock workload; prints one JSON line")
    ap.add_argument("--gate-ablation", choices=["multiblast256", "fourquad384"],
                    help="instead of the benchmark line: full WENO / trained gate / all linear / random gate "
                         "on the mixed path of a full-size shock workload; prints one JSON line")
    ap.add_argument("--second-order", action="store_true",
                    help="instead of the benchmark line: the second-order scheme of Figs. 3-7 (HLL) on the "
                         "same workload; prints one JSON line")
    ap.add_argument("--host-round-trip", action="store_true",
                    help="instead of the benchmark line: steps with the paper's per-step host round trip of the "
                         "zone means vs the resident loop; prints one JSON line")
    ap.add_argument("--rank-block", action="store_true",
                    help="one rank's 192^3 block of the 384^3 headline problem with every axis external")
    ap.add_argument("--stream", action="store_true",
                    help="instead of the benchmark line: a host-resident 256^3 mesh streamed through the GPU in "
                         "slabs vs in core; prints one JSON line")
    ap.add_argument("--ader-vs-rk", action="store_true",
                    help="instead of the benchmark line: ADER vs Runge-Kutta throughput at orders 2-4 (Table IV); "
                         "prints one JSON line")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the predictor traffic record from two rocprofv3 counter files and exit")
    ap.add_argument("--traffic-kind", choices=["c5"], help="with --traffic-from: the headline's 384^3 record")
    ap.add_argument("--gate-train", action="store_true",
                    help="instead of the headline: training throughput of the gate network (samples/s)")
    args = ap.parse_args()
    if args.cpu_sample:
        cpu_sample(args.cpu_sample, args.cpu_seconds)
        return
    if args.traffic_from:
        kind = "rk" if args.ader_vs_rk else args.traffic_kind
        write_traffic(*args.traffic_from, n=C5_N if kind == "c5" else 128, second_order=args.second_order,
                      kind=kind)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the multi-GPU path (halo exchange and a min "
              "all-reduce of dt) is designed but not implemented.", file=sys.stderr)
        sys.exit(2)

    special = (args.gate_ablation or args.second_order or args.ader_vs_rk or args.host_round_trip or args.stream
               or args.shock_workload or args.vortex128 or args.gate_train or args.rank_block)
    # the CPU baseline runs before this process touches the GPU
    cpu = None if (special or args.no_cpu_baseline) else cpu_baseline_c5(args.cpu_seconds)

    import torch
    from paper_2211_13295_amd import hog

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    hog.load()
    if args.gate_ablation:
        steps = 100 if args.gate_ablation == "multiblast256" else 200
        print(json.dumps(gate_ablation(hog, torch, args.gate_ablation, steps, 20)), flush=True)
        return
    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)            # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        print(f"copy calibration: 3 launches of {x.numel() * 8} bytes read + written", flush=True)
        del x, y
    if args.second_order:
        print(json.dumps(second_order_line(hog, torch, args)), flush=True)
        return
    if args.ader_vs_rk:
        print(json.dumps(ader_vs_rk(hog, torch, args)), flush=True)
        return
    if args.host_round_trip:
        print(json.dumps(host_round_trip(hog, torch, args)), flush=True)
        return
    if args.stream:
        print(json.dumps(stream_vs_in_core(hog, torch, args)), flush=True)
        return
    if args.rank_block:
        print(json.dumps(rank_block(hog, torch, args)), flush=True)
        return
    if args.shock_workload:
        steps = 100 if args.shock_workload == "multiblast256" else 200
        print(json.dumps(shock_workload(hog, torch, args.shock_workload, steps, 20)), flush=True)
        return
    if args.gate_train:
        print(json.dumps(gate_train_throughput(hog, torch, args)), flush=True)
        return
    if args.vortex128:
        out = vortex128_line(hog, torch, args, n=args.n or 128)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(args.order, args.cpu_seconds)
        print(json.dumps(out), flush=True)
        return
    out = headline(hog, torch, args, cpu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

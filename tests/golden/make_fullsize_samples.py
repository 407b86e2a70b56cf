"""Writes fullsize_multistep_samples.json: the FP64 oracle's state after five
steps of each full-size 3D workload, at sampled zones.

Workloads (fourth order, HLLC, CFL 0.4, positivity fallback on): the vortex
extruded along z with seeded density modes on 128^3 (periodic), the
multi-blast on 256^3 (outflow) and the four-quadrant Riemann problem on
384^3 (outflow).  The time step is fixed for all five steps: the oracle's
CFL time step of the initial state.  Zones are sampled in clusters of ten
inside 5^3 boxes (box centres at boundaries, corners, discontinuities and
at random); each cluster's values come from the oracle run on the cut-out
holding the box plus 3 * 5 + 2 zones on every side (tests/cutout.py), which
reproduces the whole-grid result there.

Run from the repository root:  python tests/golden/make_fullsize_samples.py
(calls only the oracle and the input generators)."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import icgen      # noqa: E402
import oracle     # noqa: E402
from cutout import cutout  # noqa: E402

STEPS = 5
HALF = 3 * STEPS + 2
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_multistep_samples.json")

WORKLOADS = {
    "vortex3d_perturbed_128": (lambda: icgen.vortex3d_perturbed(n=128, seed=2),
                               [(0, 0, 0), (64, 64, 64), (127, 5, 70), (40, 90, 127)]),
    "multiblast_256": (lambda: icgen.multiblast(n=256, seed=3),
                       [(0, 0, 0), (255, 128, 255), (128, 128, 128), (30, 200, 100)]),
    "four_quadrant_384": (lambda: icgen.four_quadrant(n=384, seed=5),
                          [(192, 192, 0), (191, 100, 200), (2, 383, 383), (300, 191, 50)]),
}
RANDOM_CLUSTERS = 1
PER_CLUSTER = 10


def main():
    rng = np.random.default_rng(2024)
    out = {"steps": STEPS, "half_width": HALF, "order": 4, "riemann": "hllc", "cfl": 0.4, "workloads": {}}
    for name, (make, centres) in WORKLOADS.items():
        pb = make()
        n = pb.n
        c = oracle.cfg_from_problem(pb, 4)
        dt, bad = oracle.cfl_dt(c, pb.U)
        assert bad < 0
        if name == "multiblast_256":
            # one cluster on the rim of a blast sphere: the densest zone of high pressure next to ambient
            p = (pb.U[4] > 1.0)
            k, j, i = np.argwhere(p)[0]
            centres = centres + [(int(i), int(j), int(k))]
        cs = list(centres) + [tuple(int(rng.integers(0, n[a])) for a in range(3)) for _ in range(RANDOM_CLUSTERS)]
        zones, values = [], []
        for ci, cen in enumerate(cs):
            lo = [max(0, cen[a] - 2) for a in range(3)]
            hi = [min(n[a] - 1, cen[a] + 2) for a in range(3)]
            box = np.array(np.meshgrid(*[np.arange(lo[a], hi[a] + 1) for a in range(3)], indexing="ij")).reshape(3, -1).T
            pick = box[rng.choice(len(box), size=min(PER_CLUSTER, len(box)), replace=False)]
            if ci == 0:
                pick[0] = cen
            sub, where = cutout(pb, lo, hi, HALF)
            cs_ = oracle.cfg_from_problem(sub, 4)
            t0 = time.perf_counter()
            U = sub.U
            for _ in range(STEPS):
                U = oracle.step(cs_, U, dt)
            print(f"{name} cluster {cen}: cut-out {sub.n}, {time.perf_counter() - t0:.1f} s", flush=True)
            for (i, j, k) in pick:
                a, b, cc = where(int(i), int(j), int(k))
                zones.append([int(i), int(j), int(k)])
                values.append([float(x) for x in U[:, cc, b, a]])
        out["workloads"][name] = {"n": list(n), "dt": dt, "zones": zones, "values": values}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()

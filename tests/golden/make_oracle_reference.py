"""Writes oracle reference states for sampled cells of the large workloads.

The GPU parity tests of the full-size workloads and the benchmark's accuracy figures compare
against oracle states this script stores (the oracle, a CPU FP64 BDF with full Newton and
dense LU, needs seconds to minutes per cell at rtol 1e-10). It calls only `oracle/` and the
seeded workload generator; nothing here comes from the GPU path.

Usage: python tests/golden/make_oracle_reference.py [c1|c2|c3|c5 ...]
Writes tests/golden/oracle_<workload>.json: workload, n_cells, sampled cells, tolerances,
the oracle's final states (user species order) and statuses.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.solve import oracle_solve_parallel  # noqa: E402
from paper_2111_07436_amd import workloads as W  # noqa: E402

RTOL, ATOL = 1e-10, 1e-20
# (n_cells the workload is generated with, sampled cells), both at full size: the first and
# last cells, cells spread evenly over the rest, and zero-aerosol cells (C3 cells 1 and 5, C5 cells
# 2 and 3 have no aerosol mass in the seeded draws).
SAMPLES = {
    "c1": (100, [0, 9, 18, 27, 36, 45, 54, 63, 72, 81, 90, 99]),
    "c2": (10_000, [int(c) for c in np.linspace(0, 9_999, 16)]),
    "c3": (100_000, [0, 1, 2, 5, 25_000, 50_000, 75_000, 99_999]),
    "c5": (500_000, [0, 2, 3] + [int(c) for c in np.linspace(38_461, 461_538, 12)] + [499_999]),
}


def make(name, processes):
    n, cells = SAMPLES[name]
    wl = W.make_workload(name, n_cells=n)
    t = time.time()
    y, st = oracle_solve_parallel(wl.mech, wl.env, wl.y0, wl.dt, wl.n_calls, RTOL, ATOL, cells, processes)
    zero = [int(c) for c in cells if np.all(wl.env.mass[c] == 0.0)] if wl.env.mass.size else []
    out = {"workload": name, "n_cells": n, "cells": cells, "zero_aerosol_cells": zero, "rtol": RTOL, "atol": ATOL,
           "n_calls": wl.n_calls, "dt": wl.dt, "status": [int(s) for s in st],
           "y": [[float(v) for v in row] for row in y], "oracle_seconds": time.time() - t}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"{path}: {len(cells)} cells, statuses {out['status']}, {out['oracle_seconds']:.0f} s", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(SAMPLES)
    for nm in names:
        make(nm, processes=min(8, os.cpu_count() or 1))

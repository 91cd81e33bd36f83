"""Time-convergence study with the manufactured solution on the GPU.

    python -m paper_2103_06998_amd.mms_study [--N 16] [--p 2]
        [--steps 10 20 40 80 160 320 640 1280]

For each number of steps K over [0, 1] (tau = 1/K): the state starts as the
L2 projection of u_A(0), takes K ADI steps, and after every step the L2 and
H(curl) errors of E and H against u_A are computed on the GPU; the maximum
over the steps is reported (the quantities behind the paper's Figs. 2-4),
with the observed order between successive tau.  Prints one JSON line per
tau and a summary.
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np


def run_tau(N: int, p: int, K: int, precision: str = "fp64") -> dict:
    from .solver import Solver

    s = Solver(N, p, precision)
    s.set_material_dof(1.0, 1.0, 0.0)
    s.factor(1.0 / K)
    s.mms_project(t=0.0)
    worst = {k: 0.0 for k in ("E_L2", "E_Hcurl", "H_L2", "H_Hcurl")}
    t0 = time.perf_counter()
    for _ in range(K):
        s.step(1)
        e = s.mms_errors()
        for k in worst:
            worst[k] = max(worst[k], e[k])
    wall = time.perf_counter() - t0
    s.close()
    return dict(steps=K, tau=1.0 / K, wall_s=round(wall, 3), **worst)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--N", type=int, default=16)
    ap.add_argument("--p", type=int, default=2)
    ap.add_argument("--steps", type=int, nargs="*",
                    default=[10, 20, 40, 80, 160, 320, 640, 1280])
    ap.add_argument("--precision", default="fp64")
    args = ap.parse_args(argv)
    rows = []
    for K in args.steps:
        r = run_tau(args.N, args.p, K, args.precision)
        if rows:
            prev = rows[-1]
            for k in ("E_L2", "H_L2"):
                r["order_" + k] = round(math.log(prev[k] / r[k]) / math.log(r["steps"] / prev["steps"]), 3)
        rows.append(r)
        print(json.dumps(r), flush=True)
    return rows


if __name__ == "__main__":
    main()

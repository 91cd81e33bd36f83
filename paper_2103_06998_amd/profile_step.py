"""Run a few eager ADI steps and one device copy of known size, for
hardware-counter profiles (rocprofv3 --pmc) of the step's kernels.

    python -m paper_2103_06998_amd.profile_step [--workload shell128]
        [--precision fp64|fp32_refine] [--steps 3] [--copy-mib 1024]

The steps are enqueued eagerly (one dispatch per kernel, no graph), after
one warm-up step; the copy (device to device, copy-mib MiB) calibrates the
memory counters: its fetched and written bytes are known exactly.
"""
from __future__ import annotations

import argparse
import sys

import numpy as np


def main(argv=None):
    import torch

    import workloads
    from .solver import Solver

    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="shell128")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--copy-mib", type=int, default=1024)
    args = ap.parse_args(argv)

    w = workloads.make(args.workload)
    n = w.N + w.p
    s = Solver(w.N, w.p, args.precision)
    m = w.material
    s.set_material(m.eps_r, m.mu_r, m.sigma_nd)
    if w.source is not None:
        src = w.source
        s.set_source(src.xs, src.comp, src.amp, src.f0, src.t0, src.width)
    s.factor(w.dt)
    s.set_fields(np.zeros((6, n, n, n)), 0.0)
    s.profile(1)
    s.profile(args.steps)
    s.sync()
    nbytes = args.copy_mib << 20
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(f"profiled {args.steps} eager steps of {args.workload} ({args.precision}) and a "
          f"{args.copy_mib} MiB device copy", flush=True)
    s.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())

#!/usr/bin/env python
"""Benchmark of the ADI Maxwell step on one MI355X.

Metric: field DOF-updates per second = 6 n^3 * steps / wall time of the
timed steps (both substeps of a step update every E and H coefficient once),
on the 128^3-element p=3 workload: a 256^3 voxel map of nested ellipsoidal
shells (air / skull-like / tissue-like, seed 3), a dipole source in air at
(0.5, 0.5, 0.04), dt = 1/256.  The headline run is the float32 bulk path with
float64 factors and one float64 residual correction per E solve; the float64
path is measured beside it.  All inputs are resident in device memory
before the timed region starts.

Per-kernel durations come from HIP events recorded around every kernel
launch on the library's stream, in a second timed pass that enqueues the
same kernels without the graph (graph replays cannot be split by events).
The roofline object reports the kernel class with the largest share of the
step time: algorithmic bytes per launch / average launch duration against
the 8 TB/s HBM peak.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import resource
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(launch, D, wbytes, refine=False):
    """Bytes a launch must move at minimum (each array read or written once).

    rhs_E:  6 fields + alpha, beta, gamma read, 3 right-hand sides written
            (refine mode: float32 fields, float64 coefficients, the float64
            right-hand sides and their float32 copies written);
    rhs_H:  9 fields (H, E old, E new) + delta read, 3 written;
    residual64 (refine mode): float32 solution x, float64 right-hand sides b
            and alpha read, float32 residuals b - P x written;
    sweeps: per component the right-hand side read and the solution written,
            plus the per-row coefficient on a material-modified axis.
    """
    k = launch["kind"]
    if k == "rhs_E":
        return D * (6 * 4 + 3 * 8 + 3 * 8 + 3 * 4) if refine else 12 * D * wbytes
    if k == "rhs_H":
        return 13 * D * wbytes
    if k == "residual64":
        return D * (3 * 4 + 3 * 8 + 8 + 3 * 4)
    return D * wbytes * (2 * launch["ncomp"] + launch["nmod"])


def summarize(launches, D, wbytes, refine):
    by = {}
    for L in launches:
        b = by.setdefault(L["kind"], dict(total_ms=0.0, launches=0, bytes=0.0))
        b["total_ms"] += L["ms"]
        b["launches"] += 1
        b["bytes"] += algorithmic_bytes(L, D, wbytes, refine)
    for k, b in by.items():
        b["avg_ms"] = b["total_ms"] / b["launches"]
        b["achieved_GBs"] = b["bytes"] / (b["total_ms"] * 1e-3) / 1e9
    return by


def traffic_from_profiles(kind, precision):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_2103_06998_amd", "csrc", "kernels.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("kernels_sha256") != digest:
        return None
    return rec.get("per_launch_bytes", {}).get(f"{precision}:{kind}")


def run_gpu(precision, w, steps, warmup):
    import torch
    from paper_2103_06998_amd.solver import Solver

    n = w.N + w.p
    D = n ** 3
    s = Solver(w.N, w.p, precision)
    m = w.material
    s.set_material(m.eps_r, m.mu_r, m.sigma_nd)
    src = w.source
    s.set_source(src.xs, src.comp, src.amp, src.f0, src.t0, src.width)
    s.factor(w.dt)
    s.set_fields(np.zeros((6, n, n, n)), 0.0)
    s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # kernel durations: the same kernels enqueued eagerly on the same stream
    # with HIP events around every launch, averaged over the profiled steps
    s.profile(max(5, min(steps, 50)))
    launches = s.profile_read()
    wbytes = 8 if precision == "fp64" else 4
    refine = precision != "fp64"
    kinds = summarize(launches, D, wbytes, refine)
    EH, t = s.get_fields()
    finite = bool(np.isfinite(EH).all())
    s.close()
    ms_step = elapsed * 1e3 / steps
    value = 6.0 * D * steps / elapsed
    dom = max(kinds, key=lambda k: kinds[k]["total_ms"])
    b = kinds[dom]
    per_launch_bytes = b["bytes"] / b["launches"]
    achieved = per_launch_bytes / (b["avg_ms"] * 1e-3) / 1e9
    # per-line factors streamed by the class's material-modified launches
    # ((2p+1) words per row: L, D*U, D): in the counter traffic, not in the
    # algorithmic bytes
    dom_launches = [L for L in launches if L["kind"] == dom]
    factor_bytes = sum(L["nmod"] * (2 * w.p + 1) * D * wbytes for L in dom_launches)
    roofline = {
        "bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic_from_profiles(dom, precision),
        "bytes_per_launch": int(per_launch_bytes), "avg_launch_ms": round(b["avg_ms"], 5),
        "factor_bytes_per_launch": int(factor_bytes / max(1, len(dom_launches))),
    }
    step_bytes = sum(algorithmic_bytes(L, D, wbytes, refine) for L in launches)
    kernel_ms = sum(L["ms"] for L in launches)
    return dict(value=value, ms_per_step=ms_step, roofline=roofline, finite=finite,
                kernels={k: {kk: (round(vv, 5) if isinstance(vv, float) else vv)
                             for kk, vv in v.items()} for k, v in kinds.items()},
                step_algorithmic_bytes=int(step_bytes),
                step_kernel_ms=round(kernel_ms, 4),
                step_frac_hbm=round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))


def cpu_baseline(w):
    """The float64 oracle on the host: one full step of the same workload."""
    from oracle import maxwell

    n = w.N + w.p
    prob = maxwell.problem_from_voxels(w.N, w.p, w.material, w.dt, w.source)
    rng = np.random.default_rng(0)
    E = [1e-3 * rng.standard_normal((n, n, n)) for _ in range(3)]
    H = [1e-3 * rng.standard_normal((n, n, n)) for _ in range(3)]
    E, H = prob.constrain(E, H)
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    steps, t = 0, 0.45
    # whole steps until about 10 s of work (at most 8 steps)
    while steps < 8 and (steps == 0 or time.perf_counter() - t0 < 10.0):
        E, H, t = prob.step(E, H, t)
        steps += 1
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    return {"value": 6.0 * n ** 3 * steps / wall, "unit": "field DOF-updates/s",
            "cores": max(1, int(round(cpu / wall))), "kind": "oracle",
            "sample": f"{steps} full step(s) (both substeps) of the {w.N}^3 p={w.p} workload, "
                      f"float64 NumPy oracle, {wall:.1f} s wall, {cpu:.1f} s CPU"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-256", action="store_true",
                    help="skip the 256^3 p=2 throughput lines (reported beside the headline)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path has no "
              "multi-GPU implementation (the step runs on one GPU)", file=sys.stderr)
        sys.exit(2)

    import workloads

    w = workloads.make("shell128")
    n = w.N + w.p
    log(f"workload shell128: N={w.N} p={w.p} n={n} dt={w.dt}")
    res32 = run_gpu("fp32_refine", w, args.steps, args.warmup)
    log(f"fp32_refine: {res32['ms_per_step']:.3f} ms/step {res32['value']:.3e} DOF/s")
    res64 = run_gpu("fp64", w, args.steps, args.warmup)
    log(f"fp64: {res64['ms_per_step']:.3f} ms/step {res64['value']:.3e} DOF/s")
    big = None
    if not args.no_256:
        w4 = workloads.make("shell256")
        n4 = w4.N + w4.p
        big = {"workload": "shell256: 256^3 elements, p=2, n=258, 256^3 shell map (seed 4), "
                           "dipole in air, dt=1/512, 50 steps", "dofs": 6 * n4 ** 3}
        for prec in ("fp32_refine", "fp64"):
            r = run_gpu(prec, w4, w4.steps, args.warmup)
            log(f"shell256 {prec}: {r['ms_per_step']:.3f} ms/step {r['value']:.3e} DOF/s")
            big[prec] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                         "roofline": r["roofline"], "step_frac_hbm": r["step_frac_hbm"],
                         "finite": r["finite"]}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w)
        log(f"cpu oracle: {cpu['value']:.3e} DOF/s on {cpu['cores']} core(s)")

    out = {
        "metric": "field DOF-updates/s per ADI step at 128^3 p=3 (FP64/FP32); % HBM roofline",
        "value": res32["value"],
        "unit": "field DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "shell128: 128^3 elements, p=3, n=131 coefficients per axis, "
                               "256^3 ellipsoidal-shell voxel map (seed 3), dipole in air at "
                               "(0.5,0.5,0.04), dt=1/256, float32 bulk + float64 factors + one "
                               "float64 residual correction per E solve",
                   "N": w.N, "p": w.p, "dofs": 6 * n ** 3},
        "roofline": res32["roofline"],
        "cpu_baseline": cpu,
        "fp64": {"value": res64["value"], "ms_per_step": res64["ms_per_step"], "dtype": "f64",
                 "roofline": res64["roofline"], "step_frac_hbm": res64["step_frac_hbm"],
                 "kernels": res64["kernels"], "finite": res64["finite"]},
        "fp32_refine_detail": {"kernels": res32["kernels"],
                               "step_frac_hbm": res32["step_frac_hbm"],
                               "step_algorithmic_bytes": res32["step_algorithmic_bytes"],
                               "finite": res32["finite"]},
        "shell256": big,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

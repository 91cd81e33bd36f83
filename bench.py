#!/usr/bin/env python
"""Benchmark of the ADI Maxwell step on one MI355X.

Metric: field DOF-updates per second = 6 n^3 * steps / wall time of the
timed steps (both substeps of a step update every E and H coefficient once),
on the 128^3-element p=3 workload: a 256^3 voxel map of nested ellipsoidal
shells (air / skull-like / tissue-like, seed 3), a dipole source in air at
(0.5, 0.5, 0.04), dt = 1/256.  The headline run is the float32 mode (float32
state and sweeps, factors computed in float64, every stage solved in
increment form from a float64 residual of the old state); the float64 path
is measured beside it.  All inputs are resident in device memory
before the timed region starts.

Per-kernel durations come from HIP events recorded around every kernel
launch on the library's stream, in a second timed pass that enqueues the
same kernels without the graph (graph replays cannot be split by events).
The roofline object reports the single kernel with the largest share of the
step time: its algorithmic bytes per launch / its average launch duration
against the 8 TB/s HBM peak.  step_frac_hbm is the step's algorithmic
traffic (130 words per coefficient and step) over the step time, against
the same peak; step_bytes also gives the bytes the launches as built move.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(launch, D, wbytes):
    """Bytes a launch must move at minimum (each array read or written once).

    rhs_E:  float64 path: 6 fields + gamma, beta, alpha read, 3 right-hand
            sides written; float32 mode: the same arrays in float32 (the
            increments b - P E_old: 6 fields, gamma - 1, beta, alpha read,
            3 increments written);
    rhs_H:  float64 path: 9 fields (H, E old, E new) + delta read, 3 written;
            float32 mode: the increments b - M H_old read E old, E new and
            delta only (6 + 1 read, 3 written);
    sweeps: per component the right-hand side read and the solution written,
            plus the per-row coefficient on a material-modified axis, plus the
            old state read where the float32 mode adds it (nacc).
    """
    k = launch["kind"]
    refine = wbytes == 4
    if k == "rhs_E":
        return 12 * D * wbytes
    if k == "rhs_H":
        return (10 if refine else 13) * D * wbytes
    return D * wbytes * (2 * launch["ncomp"] + launch["nmod"] + launch.get("nacc", 0))


RES64_DEFAULT = 4  # float32 mode: the E stage of substep 2 forms its increment in float64


def kernel_key(launch, nth, n, p, precision, res64=RES64_DEFAULT):
    """Name of the HIP kernel a profiled launch ran (as rocprofv3 reports it,
    without namespace and arguments); nth = index among launches of its kind
    in the step (right-hand sides: 0 = substep 1, 1 = substep 2); res64 =
    the float32 mode's mask of stages whose increment uses float64
    arithmetic (bit 2 (sub - 1) + (0 for E, 1 for H))."""
    k = launch["kind"]
    T = "double" if precision == "fp64" else "float"
    if k in ("rhs_E", "rhs_H"):
        sub = nth
        if precision == "fp64":
            stage = (0, 1)[sub] if k == "rhs_E" else (2, 3)[sub]
            return f"rhs_kernel<double, double, double, double, {p}, {stage}>"
        stage = (8, 9)[sub] if k == "rhs_E" else (10, 11)[sub]
        bit = 1 << (2 * sub + (0 if k == "rhs_E" else 1))
        TC = "double" if res64 & bit else "float"
        return f"rhs_kernel<float, {TC}, float, float, {p}, {stage}>"
    spike = 48 <= n <= 288 and launch["nmod"] == 0
    S = 8 if n >= 193 else 4  # segments per line of the partitioned solve
    m = (n + S - 1) // S      # rows per segment
    MR = next(r for r in (24, 36, 48) if m <= r)
    mod = "true" if launch["nmod"] else "false"
    if k == "apply_xyz":  # H stage: apply-and-solve lines (partitioned solves only)
        if launch["ncomp"] == 3:
            return f"spike_mixed_kernel<{T}, {p}, {MR}, {S}, true>"
        xax = "true" if launch["ncomp"] == 1 else "false"
        return f"spike_kernel<{T}, {p}, {xax}, {MR}, {S}, true>"
    if k == "sweep_xyz":
        return f"spike_mixed_kernel<{T}, {p}, {MR}, {S}, false>" if spike else \
            f"sweep_mixed_kernel<{T}, {p}, {mod}>"
    xax = "true" if k == "sweep_x" else "false"
    return f"spike_kernel<{T}, {p}, {xax}, {MR}, {S}, false>" if spike else \
        f"sweep_kernel<{T}, {p}, {xax}, {mod}>"


def summarize(launches, D, n, p, precision, res64=RES64_DEFAULT):
    """Per kernel: launches per step, total and mean duration, algorithmic bytes."""
    wbytes = 8 if precision == "fp64" else 4
    by, seen = {}, {}
    for L in launches:
        nth = seen.get(L["kind"], 0)
        seen[L["kind"]] = nth + 1
        key = kernel_key(L, nth, n, p, precision, res64)
        b = by.setdefault(key, dict(total_ms=0.0, launches=0, bytes=0.0, factor_bytes=0.0))
        b["total_ms"] += L["ms"]
        b["launches"] += 1
        b["bytes"] += algorithmic_bytes(L, D, wbytes)
        # cached per-line factors ((2p+1) words per row: L, D*U, D) that the
        # material-modified launches stream; in the counter traffic, not in
        # the algorithmic bytes
        b["factor_bytes"] += L["nmod"] * (2 * p + 1) * D * wbytes
    for b in by.values():
        b["avg_ms"] = b["total_ms"] / b["launches"]
        b["achieved_GBs"] = b["bytes"] / (b["total_ms"] * 1e-3) / 1e9
    return by


def traffic_from_profiles(key, precision):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_2103_06998_amd", "csrc", "kernels.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("kernels_sha256") != digest:
        return None
    return rec.get("per_launch_bytes", {}).get(f"{precision}:{key}")


# Algorithmic words per step in units of D = n^3 (both substeps; each 1D
# pass reads and writes its array once, the x sweep fused into the
# right-hand side): E stage 38 and H stage 27 per substep.
MODEL_WORDS_PER_STEP = 130


def run_gpu(precision, w, steps, warmup, res64=RES64_DEFAULT):
    import torch
    from paper_2103_06998_amd.solver import Solver

    n = w.N + w.p
    D = n ** 3
    s = Solver(w.N, w.p, precision)
    m = w.material
    s.set_material(m.eps_r, m.mu_r, m.sigma_nd)
    src = w.source
    s.set_source(src.xs, src.comp, src.amp, src.f0, src.t0, src.width)
    s.set_residual64(res64)
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
    # kernel durations: the same kernels enqueued eagerly on the library's
    # stream with HIP events around every launch, averaged over the steps
    s.profile(max(5, min(steps, 50)))
    launches = s.profile_read()
    wbytes = 8 if precision == "fp64" else 4
    kernels = summarize(launches, D, n, w.p, precision, res64)
    EH, t = s.get_fields()
    finite = bool(np.isfinite(EH).all())
    s.close()
    ms_step = elapsed * 1e3 / steps
    value = 6.0 * D * steps / elapsed
    # the single kernel with the largest share of the step time
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    b = kernels[dom]
    per_launch = b["bytes"] / b["launches"]
    achieved = per_launch / (b["avg_ms"] * 1e-3) / 1e9
    roofline = {
        "bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic_from_profiles(dom, precision),
        "bytes_per_launch": int(per_launch), "avg_launch_ms": round(b["avg_ms"], 5),
        "launches_per_step": b["launches"],
        "share_of_step": round(b["total_ms"] / sum(k["total_ms"] for k in kernels.values()), 4),
        "factor_bytes_per_launch": int(b["factor_bytes"] / b["launches"]),
    }
    model_bytes = MODEL_WORDS_PER_STEP * D * wbytes
    executed_bytes = sum(k["bytes"] for k in kernels.values())
    return dict(value=value, ms_per_step=ms_step, roofline=roofline, finite=finite,
                kernels={k: {kk: (round(vv, 5) if isinstance(vv, float) else vv)
                             for kk, vv in v.items()} for k, v in kernels.items()},
                step_kernel_ms=round(sum(L["ms"] for L in launches), 4),
                step_bytes={"model_130_words": int(model_bytes), "executed": int(executed_bytes),
                            "overhead": int(executed_bytes - model_bytes)},
                step_frac_hbm=round(model_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))


def _oracle_steps(args):
    """Worker: whole oracle steps of a workload until about `budget` seconds."""
    name, budget, seed = args
    import workloads
    from oracle import maxwell

    w = workloads.make(name)
    n = w.N + w.p
    prob = maxwell.problem_from_voxels(w.N, w.p, w.material, w.dt, w.source)
    rng = np.random.default_rng(seed)
    E = [1e-3 * rng.standard_normal((n, n, n)) for _ in range(3)]
    H = [1e-3 * rng.standard_normal((n, n, n)) for _ in range(3)]
    E, H = prob.constrain(E, H)
    t0 = time.perf_counter()
    steps, t = 0, 0.45
    while steps < 8 and (steps == 0 or time.perf_counter() - t0 < budget):
        E, H, t = prob.step(E, H, t)
        steps += 1
    return steps, time.perf_counter() - t0, t0


def cpu_baseline(name, n):
    """The float64 oracle on the host, on one core and on all usable cores.

    The oracle is NumPy with one thread per process; the all-cores figure
    runs one independent oracle per core (each stepping its own state of the
    same workload) and counts the DOF-updates of all of them over the wall
    time from the first start to the last end."""
    import concurrent.futures
    import multiprocessing as mp

    one_steps, one_wall, _ = _oracle_steps((name, 10.0, 0))
    single = 6.0 * n ** 3 * one_steps / one_wall
    ncpu = os.cpu_count() or 1
    cores = max(1, min(ncpu, 16))
    ctx = mp.get_context("spawn")
    with concurrent.futures.ProcessPoolExecutor(cores, mp_context=ctx) as ex:
        res = list(ex.map(_oracle_steps, [(name, 10.0, k + 1) for k in range(cores)]))
    start = min(r[2] for r in res)
    end = max(r[2] + r[1] for r in res)
    total_steps = sum(r[0] for r in res)
    value = 6.0 * n ** 3 * total_steps / (end - start)
    return {"value": value, "unit": "field DOF-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} concurrent float64 NumPy oracles (one per core, one thread "
                      f"each, host has {ncpu} logical CPUs), {total_steps} full steps of the "
                      f"{name} workload in {end - start:.1f} s wall",
            "single_core": {"value": single, "cores": 1,
                            "sample": f"{one_steps} full step(s), {one_wall:.1f} s wall"}}


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
    cpu = None
    if not args.no_cpu_baseline:
        # before the GPU is touched: the worker processes start clean
        cpu = cpu_baseline("shell128", n)
        log(f"cpu oracle: {cpu['value']:.3e} DOF/s on {cpu['cores']} core(s), "
            f"{cpu['single_core']['value']:.3e} on one")
    log(f"workload shell128: N={w.N} p={w.p} n={n} dt={w.dt}")
    res32 = run_gpu("fp32_refine", w, args.steps, args.warmup)
    log(f"fp32_refine: {res32['ms_per_step']:.3f} ms/step {res32['value']:.3e} DOF/s")
    r64 = run_gpu("fp64", w, args.steps, args.warmup)
    log(f"fp64: {r64['ms_per_step']:.3f} ms/step {r64['value']:.3e} DOF/s")
    # the float32 mode with its increments in float32 arithmetic everywhere
    # (mask 0) and in float64 for every stage (mask 15), beside the default
    residual = {}
    for mask in (0, 15):
        r = run_gpu("fp32_refine", w, args.steps, args.warmup, mask)
        log(f"fp32_refine, float64 increments mask {mask}: {r['ms_per_step']:.3f} ms/step")
        residual[str(mask)] = {"ms_per_step": r["ms_per_step"], "value": r["value"],
                               "finite": r["finite"]}
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
                         "step_bytes": r["step_bytes"], "finite": r["finite"]}

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
                               "(0.5,0.5,0.04), dt=1/256, float32 state, right-hand sides and "
                               "sweeps with float32 accumulation, factors computed in float64, "
                               "every stage solved in increment form (residual correction of "
                               "the old state), the residual of the E stage that closes each "
                               "step formed in float64 arithmetic",
                   "res64_mask": RES64_DEFAULT,
                   "N": w.N, "p": w.p, "dofs": 6 * n ** 3},
        "roofline": res32["roofline"],
        "cpu_baseline": cpu,
        "step_frac_hbm": res32["step_frac_hbm"],
        "step_bytes": res32["step_bytes"],
        "kernels": res32["kernels"],
        "fp64": {"value": r64["value"], "ms_per_step": r64["ms_per_step"], "dtype": "f64",
                 "roofline": r64["roofline"], "step_frac_hbm": r64["step_frac_hbm"],
                 "step_bytes": r64["step_bytes"], "kernels": r64["kernels"],
                 "finite": r64["finite"]},
        "finite": res32["finite"],
        "fp32_residual_masks": residual,
        "shell256": big,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

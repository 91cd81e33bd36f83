"""Per-launch HBM traffic of the step's kernel classes from rocprofv3 counter
runs, calibrated on a device copy of known size.

    python -m paper_2103_06998_amd.pmc_traffic FETCH_DIR WRITE_DIR PRECISION \\
        [--copy-mib 1024] [--out profiles/pmc_traffic.json]

FETCH_DIR / WRITE_DIR hold the run_counter_collection.csv of a
`rocprofv3 --pmc FETCH_SIZE` and a `rocprofv3 --pmc WRITE_SIZE` run of
`python -m paper_2103_06998_amd.profile_step --precision PRECISION`.  Both
counters are in KiB per dispatch; each is scaled by (copy bytes) / (what the
counter reads for the copy dispatch of that run), then averaged per launch
over the dispatches of each kernel.  The result is merged into the output
JSON under "<precision>:<kernel>" (the kernel's name without namespace and
arguments) together with the sha256 of the kernel source it was measured on.
"""
from __future__ import annotations

import argparse
import csv
import collections
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def kernel_class(name: str):
    """Kernel name without namespace and arguments (e.g.
    "sweep_mixed_kernel<float, 3, true>"), "copy" for the runtime's copy
    kernel, None for anything else."""
    if "copyBuffer" in name:
        return "copy"
    m = re.search(r"(\w+_kernel<[^()]*>)\(", name)
    return m.group(1) if m else None


def per_dispatch(path, counter):
    rows = list(csv.DictReader(open(os.path.join(path, "run_counter_collection.csv"))))
    vals, names = collections.defaultdict(float), {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        d = int(r["Dispatch_Id"])
        vals[d] += float(r["Counter_Value"])
        names[d] = r["Kernel_Name"]
    return vals, names


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("precision")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "pmc_traffic.json"))
    args = ap.parse_args(argv)
    copy_bytes = float(args.copy_mib << 20)
    result = {}
    factors = {}
    for which, path, counter in (("fetch", args.fetch_dir, "FETCH_SIZE"),
                                 ("write", args.write_dir, "WRITE_SIZE")):
        vals, names = per_dispatch(path, counter)
        copies = [v for d, v in vals.items() if kernel_class(names[d]) == "copy"]
        big = max(copies) * 1024.0  # the calibration copy is the largest copy dispatch
        factor = copy_bytes / big
        factors[which] = factor
        acc = collections.defaultdict(list)
        for d, v in vals.items():
            k = kernel_class(names[d])
            if k and k != "copy":
                acc[k].append(v * 1024.0 * factor)
        for k, lst in acc.items():
            result.setdefault(k, {})[which] = sum(lst) / len(lst)
    rec = {}
    if os.path.exists(args.out):
        rec = json.load(open(args.out))
    src = os.path.join(HERE, "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("kernels_sha256") != sha:
        rec = {"kernels_sha256": sha, "per_launch_bytes": {}, "calibration": {}}
    for k, v in result.items():
        rec["per_launch_bytes"][f"{args.precision}:{k}"] = int(v.get("fetch", 0) + v.get("write", 0))
        rec.setdefault("detail", {})[f"{args.precision}:{k}"] = {
            "fetch_bytes": int(v.get("fetch", 0)), "write_bytes": int(v.get("write", 0))}
    rec["calibration"][args.precision] = {"copy_bytes": int(copy_bytes),
                                          "fetch_factor": factors["fetch"],
                                          "write_factor": factors["write"]}
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(json.dumps(rec, indent=1, sort_keys=True))


if __name__ == "__main__":
    main()

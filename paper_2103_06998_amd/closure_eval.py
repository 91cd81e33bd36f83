"""Train the closure network on solver-generated pairs and evaluate it.

    python -m paper_2103_06998_amd.closure_eval [--train-p 2] [--maps 64]
        [--pairs-per-map 32] [--iters 8000] [--eval-seeds 9001 9002 9003]

Training: 64^3 elements of degree train-p on three-class blob maps (seeds
100, 101, ...), a dipole at a random position per map; pairs are one ADI
step of 4 h_t against four steps of h_t = 1/(2N) from states along a fine
trajectory.  Evaluation (--eval shell128): 128^3 elements, p = 3, unseen
nested-shell maps, the dipole of the shell workload, 200 steps of
h_t = 1/256 for plain ADI against 50 closure steps of 4 h_t, every run
against float64 ADI at h_t / 4; --eval blob: in distribution, on unseen blob
maps and dipoles at the training grid, degree and h_t.  The gate judges each
correction against the coarse step's change (adi_step_closure).
Prints one JSON object per evaluation map and a summary line.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def main(argv=None):
    import torch

    import workloads
    from . import closure

    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train-p", type=int, default=2)
    ap.add_argument("--train-N", type=int, default=64)
    ap.add_argument("--maps", type=int, default=64)
    ap.add_argument("--pairs-per-map", type=int, default=32)
    ap.add_argument("--iters", type=int, default=8000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--gate", type=float, default=0.5)
    ap.add_argument("--eval", choices=("shell128", "blob"), default="shell128")
    ap.add_argument("--dagger", type=int, default=0,
                    help="rounds of extra pairs sampled along the closure's own "
                         "trajectories, each followed by more training")
    ap.add_argument("--eval-seeds", type=int, nargs="*", default=[9001, 9002, 9003])
    ap.add_argument("--save", default="")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    N, p = args.train_N, args.train_p
    h_t = 1.0 / (2 * N)
    dtc = 4 * h_t

    def train_source(seed):
        r = np.random.default_rng(seed)
        return workloads.DipoleSource(xs=tuple(r.uniform(0.1, 0.9, 3)),
                                      f0=float(r.uniform(1.5, 3.0)))

    t0 = time.time()
    seeds = list(range(100, 100 + args.maps))
    pairs = None
    for k in range(0, len(seeds), 8):
        chunk = seeds[k:k + 8]
        pairs = closure.generate_pairs(N, p, [workloads.blob_map(N, s) for s in chunk],
                                       [train_source(s) for s in chunk], dtc, 4,
                                       pairs_per_map=args.pairs_per_map, every=3, warmup=16,
                                       pairs=pairs)
    held = closure.generate_pairs(N, p, [workloads.blob_map(N, 99)], [train_source(99)], dtc, 4,
                                  pairs_per_map=16, every=3, warmup=20)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    log(f"pairs: {len(pairs.x)} training, {len(held.x)} held out, {gen_s:.1f} s")

    net = closure.Network()
    net.set_params(closure.init_params(0))
    t0 = time.time()
    closure.train(net, pairs, iters=args.iters, lr=args.lr, lr_final=1e-5,
                  log_every=max(1, args.iters // 8), log=log)
    for r in range(args.dagger):
        # states the closure itself visits (its own trajectory, gated), on
        # the first 16 training maps, then more training on all pairs
        chunk = seeds[:16]
        pairs = closure.generate_pairs(N, p, [workloads.blob_map(N, s) for s in chunk],
                                       [train_source(s) for s in chunk], dtc, 4,
                                       pairs_per_map=args.pairs_per_map // 2, every=2,
                                       warmup=4, pairs=pairs, rollout_net=net, gate=args.gate)
        closure.train(net, pairs, iters=args.iters // 2, lr=args.lr / 4, lr_final=1e-5,
                      seed=r + 1, log_every=max(1, args.iters // 4), log=log)
        log(f"dagger round {r + 1}: {len(pairs.x)} pairs")
    torch.cuda.synchronize()
    train_s = time.time() - t0
    held_ratio = closure.evaluate_loss(net, held) / closure.target_energy(held)
    log(f"training: {args.iters} iterations in {train_s:.1f} s; held-out one-step loss / "
        f"zero-correction loss = {held_ratio:.3f}")
    if args.save:
        np.save(args.save, net.get_params())

    wl = workloads.make("shell128")
    rows = []
    for seed in args.eval_seeds:
        if args.eval == "shell128":
            res = closure.run_comparison(128, 3, workloads.shell_map(256, seed), wl.source,
                                         1.0 / 256, 200, net, gate=args.gate, time_reps=2)
        else:
            res = closure.run_comparison(N, p, workloads.blob_map(N, seed), train_source(seed),
                                         h_t, 200, net, gate=args.gate, time_reps=2)
        row = dict(seed=seed, fine_err=res["fine"]["rel_l2"], coarse_err=res["coarse"]["rel_l2"],
                   closure_err=res["closure"]["rel_l2"], fine_ms=res["fine"]["ms"],
                   coarse_ms=res["coarse"]["ms"], closure_ms=res["closure"]["ms"],
                   rejected=res.get("rejected", 0), speedup_vs_fine=res["speedup_vs_fine"])
        rows.append(row)
        log(json.dumps(row))
    summary = dict(eval=args.eval, dagger=args.dagger, train_p=p, train_N=N, pairs=len(pairs.x), iters=args.iters,
                   train_s=round(train_s, 2), pair_gen_s=round(gen_s, 2),
                   held_one_step_ratio=round(held_ratio, 4), gate=args.gate,
                   mean_fine_err=float(np.mean([r["fine_err"] for r in rows])),
                   mean_coarse_err=float(np.mean([r["coarse_err"] for r in rows])),
                   mean_closure_err=float(np.mean([r["closure_err"] for r in rows])),
                   mean_speedup_vs_fine=float(np.mean([r["speedup_vs_fine"] for r in rows])))
    log(json.dumps(summary))
    net.close()
    return summary


if __name__ == "__main__":
    main()

"""Saturation study of the learned warm start on one mesh: the network trained on
n cold solves (random roots, onsets and smooth velocity scales) for growing n,
each evaluated on the same held-out cases.  Reports, per n, the guess error and
the work and time of the warm-started solve against the cold one, so that the
training-set size can be chosen where the error stops improving.

    python -m paper_2308_08410_amd.learned_study --nodes 500000 --sizes 32,128,512,2048,10000
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import binding as B
from . import warmstart as WS


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--nodes", type=int, default=500_000)
    ap.add_argument("--sizes", default="32,128,512,2048,10000")
    ap.add_argument("--steps-per-solve", type=float, default=2.0)
    ap.add_argument("--min-steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--test", type=int, default=6)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--scale-bank", type=int, default=128,
                    help="distinct smooth velocity-scale fields shared by the training cases")
    args = ap.parse_args(argv)
    import gbp_inputs as gi
    dev = torch.device("cuda", 0)
    p = gi.shell_problem(args.nodes, seed=args.seed, n_roots=5, n_leads=12)
    plan = B.Plan(p.xyz, p.tets)
    D = torch.as_tensor(p.D, device=dev)
    sizes = [int(x) for x in args.sizes.split(",")]
    t0 = time.perf_counter()
    data = WS.make_dataset(plan, p.xyz, D, p.extra["endo"], max(sizes), seed=4_000_000,
                           scale_bank=args.scale_bank, log_every=250)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    test = WS.make_dataset(plan, p.xyz, D, p.extra["endo"], args.test, seed=9_000_000)
    print(json.dumps(dict(nodes=p.n_v, solves=max(sizes), data_seconds=t_data)), flush=True)
    for n in sizes:
        ws = WS.WarmStart(p.xyz, p.extra["node_fibre"], max_rows=args.batch, seed=args.seed)
        steps = max(args.min_steps, int(args.steps_per_solve * n))
        t0 = time.perf_counter()
        print(f"[train] {n} solves, {steps} steps", flush=True)
        hist = WS.train(ws, data[:n], steps, batch=args.batch, lr=1e-3, log_every=max(1, steps // 10),
                        verbose=True)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        rows = WS.evaluate(ws, plan, D, test, repeats=2)
        mean = lambda f: float(np.mean([f(r) for r in rows]))
        print(json.dumps(dict(
            solves=n, steps=steps, train_seconds=t_train, loss_last=hist[-1][1],
            guess_rel_l2=dict(mlp=mean(lambda r: r["guess_rel_l2"]["mlp"]),
                              geo=mean(lambda r: r["guess_rel_l2"]["geo"])),
            face_solves=dict(cold=mean(lambda r: r["cold"]["face_solves"]),
                             warm_mlp=mean(lambda r: r["warm_mlp"]["face_solves"])),
            rounds=dict(cold=mean(lambda r: r["cold"]["rounds"]), warm_mlp=mean(lambda r: r["warm_mlp"]["rounds"])),
            ms=dict(cold=mean(lambda r: r["cold_ms"]), warm_mlp=mean(lambda r: r["warm_ms"]),
                    predict=mean(lambda r: r["predict_ms"])),
            fallbacks=sum(r["warm_mlp"]["fallback"] for r in rows),
            max_warm_vs_cold_rel=max(r["warm_vs_cold_rel_max"]["mlp"] for r in rows))), flush=True)


if __name__ == "__main__":
    sys.exit(main())

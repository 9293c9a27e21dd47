"""Writes shell500k_reference.npz: the FP64 oracle's activation times for the
benchmark workload (500k-vertex shell, perturbed root onsets, smooth velocity
scale), stored as float32, with a hash of the inputs.  Calls only gbp_inputs and
oracle.  Takes a few minutes of CPU time.

    python tests/golden/make_shell500k_reference.py
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gbp_inputs as gi  # noqa: E402
import oracle as O  # noqa: E402

OUT = os.path.join(HERE, "shell500k_reference.npz")


def bench_like(n):
    p = gi.shell_problem(n, seed=2, n_roots=5, n_leads=12)
    rng = np.random.Generator(np.random.PCG64(21))
    rt = (p.root_t + rng.uniform(-5, 5, size=len(p.root_t))).astype(np.float32)
    vs = gi.smooth_field(p.xyz, 0.7, 1.3, seed=20)
    return p, rt, vs


def input_hash(p, rt, vs):
    h = hashlib.sha256()
    for a in (p.xyz, p.tets, p.D, p.root_node, rt, vs):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    t = time.time()
    p, rt, vs = bench_like(500_000)
    T, st = O.solve(p.xyz, p.tets, p.D, vs, p.root_node, rt)
    print(f"oracle solve: {time.time() - t:.1f}s {st}", flush=True)
    np.savez_compressed(OUT, T=T.astype(np.float32), input_sha256=input_hash(p, rt, vs),
                        sweeps=st["sweeps"], solves=st["solves"])
    print(OUT)


if __name__ == "__main__":
    main()

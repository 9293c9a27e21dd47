"""Learned warm start for the eikonal forward (an extension beyond the paper,
which starts every solve from +inf).

A small network (libgbp's gbp_mlp: 16 -> 4 x 256 ReLU -> 1, bf16 matrix-core
kernels) predicts the activation time of every vertex from its position, fibre
direction, the sorted per-root values |x - x_r| / L + t_r / T_s and the velocity
scale.  The prediction seeds the two-sided solve (gbp_eikonal_forward with
T_init), or, with the plan's warm order on, orders a cold solve's hold-back;
either way the fixed point is the cold solution whatever the guess, so the
prediction can only change the work, never the answer; a solve that does not
converge from the guess is redone cold.

The network is trained per mesh on solves of that mesh with random roots, onsets
and smooth velocity scales (the situation of a patient-specific inverse problem,
where the mesh is fixed and the parameters move).

    python -m paper_2308_08410_amd.warmstart --nodes 100000 --solves 64 --steps 2000
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

from . import binding as B
from . import runlog


class WarmStart:
    """Feature extraction, the network and the warm-started forward for one mesh."""

    def __init__(self, xyz, node_fibre, max_rows=1 << 16, seed=0, v_ref=0.6, device="cuda"):
        xyz = np.ascontiguousarray(np.asarray(xyz, np.float32))
        dev = torch.device(device)
        c = 0.5 * (xyz.min(0) + xyz.max(0))
        L = float(np.linalg.norm(xyz - c, axis=1).max())
        # features measure lengths in L and times in the time to cross L at v_ref
        self.norm = (float(c[0]), float(c[1]), float(c[2]), L, L / v_ref)
        self.time_scale = L / v_ref
        self.v_ref = v_ref
        self.n_v = len(xyz)
        self.xyz_h = xyz
        self.xyz = torch.as_tensor(xyz, device=dev)
        self.fibre = torch.as_tensor(np.ascontiguousarray(node_fibre, np.float32), device=dev)
        self.mlp = B.MLP(max_rows, seed)
        self.device = dev

    def root_xyz(self, root_node):
        rn = np.asarray(root_node.cpu() if isinstance(root_node, torch.Tensor) else root_node, np.int64)
        if not 1 <= len(rn) <= 8:
            raise ValueError("the learned warm start takes 1 to 8 roots")
        return torch.as_tensor(np.ascontiguousarray(self.xyz_h[rn]), device=self.device)

    def features(self, root_node, root_t, vscale=None, rows=None, T=None):
        return B.mlp_features(self.xyz, self.fibre, self.root_xyz(root_node), root_t, self.norm,
                              vscale=vscale, rows=rows, T=T)

    def predict(self, root_node, root_t, vscale=None, out=None):
        """Predicted activation times [n_v] (device): the features of every vertex,
        then one inference pass over all of them."""
        if out is None:
            out = torch.empty(self.n_v, dtype=torch.float32, device=self.device)
        rx = self.root_xyz(root_node)
        X = B.mlp_features(self.xyz, self.fibre, rx, root_t, self.norm, vscale=vscale)
        self.mlp.forward(X, out_scale=self.time_scale, out=out)
        return out

    def forward(self, plan, D, vscale, root_node, root_t, out=None, fallback=True):
        """Warm-started eikonal forward from the network's guess; (T, stats)
        with stats['fallback'] telling whether the cold solve had to be run."""
        guess = self.predict(root_node, root_t, vscale)
        try:
            T, st = B.eikonal_forward(plan, D, vscale, root_node, root_t, T_init=guess, out=out)
            st["fallback"] = False
        except B.GbpError as e:
            if not fallback or e.name != "GBP_ERR_NOT_CONVERGED":
                raise
            T, st = B.eikonal_forward(plan, D, vscale, root_node, root_t, out=out)
            st["fallback"] = True
        return T, st


# ---------------------------------------------------------------- data, training, evaluation
def random_case(xyz, candidates, seed, roots=(1, 8), t_range=(0.0, 20.0), vscale_range=(0.5, 1.5),
                with_scale=True):
    """Random roots (count, nodes, onsets) and a smooth velocity scale (None
    unless with_scale)."""
    import gbp_inputs as gi
    r = np.random.Generator(np.random.PCG64(seed))
    R = int(r.integers(roots[0], roots[1] + 1))
    rn, rt = gi.random_roots(candidates, R, t_range[0], t_range[1], seed=seed + 1)
    lo = float(r.uniform(vscale_range[0], 1.0))
    hi = float(r.uniform(1.0, vscale_range[1]))
    vs = gi.smooth_field(xyz, lo, hi, seed=seed + 2) if with_scale else None
    return rn, rt, vs


def make_dataset(plan, xyz, D, candidates, n_solves, seed=0, scale_bank=0, log_every=0, **kw):
    """Cold solves of the mesh for random cases (the training targets).  With
    scale_bank > 0 the velocity scales come from that many seeded smooth fields,
    reused across cases (each paired with its own random roots and onsets), since
    a smooth field over a large mesh takes longer to make than a solve."""
    dev = D.device
    data = []
    bank = []
    for k in range(n_solves):
        rn, rt, vs = random_case(xyz, candidates, seed + 7919 * k,
                                 with_scale=(k < scale_bank) if scale_bank else True, **kw)
        if scale_bank:
            if k < scale_bank:
                bank.append(torch.as_tensor(vs, device=dev))
            vsd = bank[k % scale_bank]
        else:
            vsd = torch.as_tensor(vs, device=dev)
        d = dict(root_node=torch.as_tensor(rn, device=dev), root_t=torch.as_tensor(rt, device=dev), vscale=vsd)
        d["T"], _ = B.eikonal_forward(plan, D, d["vscale"], d["root_node"], d["root_t"])
        data.append(d)
        if log_every and (k + 1) % log_every == 0:
            print(f"[data] {k + 1} of {n_solves} solves", flush=True)
    return data


def train(ws: WarmStart, data, steps, batch=8192, lr=1e-3, lr_min=1e-5, log_every=100, seed=0, verbose=False,
          checkpoint=None, checkpoint_every=0, resume=False, log: runlog.RunLog | None = None, stop=None):
    """Adam on random row batches of the solves, cosine learning-rate decay over
    `steps` steps.  Returns [(step, mse in normalised time units)].  With
    `checkpoint` the network, its Adam state, the step and the row generator's
    state are saved every checkpoint_every steps and where the call stops; `stop`
    ends the call before step `stop` of the schedule (a time-bounded job);
    resume=True continues from the checkpoint (the same steps follow as in an
    uninterrupted run)."""
    if batch > ws.mlp.max_rows:
        raise ValueError("batch exceeds the network's max_rows")
    g = torch.Generator(device=ws.device)
    g.manual_seed(seed)
    loss = torch.empty(1, dtype=torch.float32, device=ws.device)
    hist = []
    first = 0
    if resume:
        c = runlog.load_checkpoint(checkpoint)
        ws.mlp.set_params(c["params"])
        ws.mlp.set_state(dict(m=c["m"], v=c["v"], step=int(c["adam_step"])))
        g.set_state(torch.as_tensor(c["rng"]))
        first = int(c["step"])
        hist = [(int(a), float(b)) for a, b in c["hist"]]

    def save(done):
        st = ws.mlp.get_state()
        runlog.save_checkpoint(checkpoint, params=ws.mlp.get_params(), m=st["m"], v=st["v"],
                               adam_step=np.int64(st["step"]), step=np.int64(done),
                               rng=g.get_state().numpy(), hist=np.asarray(hist, np.float64).reshape(-1, 2))

    last = steps if stop is None else min(int(stop), steps)
    for s in range(first, last):
        d = data[s % len(data)]
        rows = torch.randint(0, ws.n_v, (batch,), dtype=torch.int32, device=ws.device, generator=g)
        X, tgt = ws.features(d["root_node"], d["root_t"], d["vscale"], rows=rows, T=d["T"])
        lr_s = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * s / max(steps, 1)))
        ws.mlp.train_step(X, tgt, lr_s, loss=loss)
        if log_every and (s % log_every == 0 or s == steps - 1):
            hist.append((s, float(loss)))
            if verbose:
                print(f"[train] step {s} of {steps}: mse {hist[-1][1]:.4g}", flush=True)
            if log is not None:
                log.write(event="train", step=s, mse=hist[-1][1], lr=lr_s)
        if checkpoint and ((checkpoint_every and (s + 1) % checkpoint_every == 0) or s == last - 1):
            save(s + 1)
    return hist


def geometric_guess(ws: WarmStart, root_node, root_t):
    """Baseline guess without a network: min over roots of |x - x_r| / v_ref + t_r."""
    rx = ws.root_xyz(root_node)
    return (torch.cdist(ws.xyz, rx) / ws.v_ref + root_t[None, :]).min(dim=1).values.contiguous()


def _timed(fn):
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    out = fn()
    b.record()
    torch.cuda.synchronize()
    return out, a.elapsed_time(b)


def evaluate(ws: WarmStart, plan, D, cases, repeats=3):
    """Per held-out case: cold solve, warm solve from the network's guess (time
    includes the prediction; two-sided, and ordered: a cold solve whose hold-back
    is keyed by the guess, in the plan's hold-back setting) and from the geometric
    guess; work counters, times, guess errors and the warm-vs-cold difference."""
    rows = []
    order0 = B.get_warm_order(plan)
    for d in cases:
        args = (plan, D, d["vscale"], d["root_node"], d["root_t"])
        best = {}
        for _ in range(repeats):
            (Tc, sc), tc = _timed(lambda: B.eikonal_forward(*args))
            B.set_warm_order(plan, False)
            (Tw, sw), tw = _timed(lambda: ws.forward(*args))
            B.set_warm_order(plan, True)
            (To, so), to = _timed(lambda: ws.forward(*args))
            B.set_warm_order(plan, order0)
            guess_m, tp = _timed(lambda: ws.predict(d["root_node"], d["root_t"], d["vscale"]))
            guess_g = geometric_guess(ws, d["root_node"], d["root_t"])
            (Tg, sg), tg = _timed(lambda: B.eikonal_forward(*args, T_init=guess_g))
            for k, v in (("cold_ms", tc), ("warm_ms", tw), ("ordered_ms", to), ("predict_ms", tp), ("geo_ms", tg)):
                best[k] = min(best.get(k, v), v)
        fin = torch.isfinite(Tc)
        scale = float(Tc[fin].abs().max())
        rel = lambda a: float((a[fin] - Tc[fin]).norm() / Tc[fin].norm())
        rows.append(dict(
            n_roots=int(d["root_node"].numel()),
            cold=dict(rounds=sc["rounds"], face_solves=sc["face_solves"], node_updates=sc["node_updates"]),
            warm_mlp=dict(rounds=sw["rounds"], face_solves=sw["face_solves"],
                          node_updates=sw["node_updates"], fallback=sw["fallback"]),
            warm_mlp_ordered=dict(rounds=so["rounds"], face_solves=so["face_solves"],
                                  node_updates=so["node_updates"]),
            warm_geo=dict(rounds=sg["rounds"], face_solves=sg["face_solves"], node_updates=sg["node_updates"]),
            guess_rel_l2=dict(mlp=rel(guess_m), geo=rel(guess_g)),
            guess_max_abs_ms=dict(mlp=float((guess_m[fin] - Tc[fin]).abs().max()),
                                  geo=float((guess_g[fin] - Tc[fin]).abs().max())),
            warm_vs_cold_rel_max=dict(mlp=float((Tw[fin] - Tc[fin]).abs().max()) / scale,
                                      mlp_ordered=float((To[fin] - Tc[fin]).abs().max()) / scale,
                                      geo=float((Tg[fin] - Tc[fin]).abs().max()) / scale),
            **best))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--nodes", type=int, default=100_000)
    ap.add_argument("--solves", type=int, default=64)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--test", type=int, default=6)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--log", default="", help="JSON-lines run log (appended)")
    ap.add_argument("--checkpoint", default="", help="training checkpoint file (.npz)")
    ap.add_argument("--checkpoint-every", type=int, default=0)
    ap.add_argument("--resume", action="store_true", help="continue training from --checkpoint")
    args = ap.parse_args(argv)
    import gbp_inputs as gi
    dev = torch.device("cuda", 0)
    p = gi.shell_problem(args.nodes, seed=args.seed)
    plan = B.Plan(p.xyz, p.tets)
    D = torch.as_tensor(p.D, device=dev)
    t0 = time.perf_counter()
    data = make_dataset(plan, p.xyz, D, p.extra["endo"], args.solves, seed=1000 + args.seed)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    ws = WarmStart(p.xyz, p.extra["node_fibre"], max_rows=args.batch, seed=args.seed)
    t0 = time.perf_counter()
    log = runlog.RunLog(args.log, "warmstart", dict(vars(args), n_v=p.n_v, n_e=p.n_e)) if args.log else None
    hist = train(ws, data, args.steps, batch=args.batch, lr=args.lr, log_every=max(1, args.steps // 20),
                 checkpoint=args.checkpoint or None, checkpoint_every=args.checkpoint_every,
                 resume=args.resume, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    test = make_dataset(plan, p.xyz, D, p.extra["endo"], args.test, seed=900_000 + args.seed)
    rows = evaluate(ws, plan, D, test)
    mean = lambda f: float(np.mean([f(r) for r in rows]))
    summary = dict(
        nodes=p.n_v, solves=args.solves, steps=args.steps, batch=args.batch,
        data_seconds=t_data, train_seconds=t_train, loss_first=hist[0][1], loss_last=hist[-1][1],
        mean_face_solves=dict(cold=mean(lambda r: r["cold"]["face_solves"]),
                              warm_mlp=mean(lambda r: r["warm_mlp"]["face_solves"]),
                              warm_geo=mean(lambda r: r["warm_geo"]["face_solves"])),
        mean_rounds=dict(cold=mean(lambda r: r["cold"]["rounds"]), warm_mlp=mean(lambda r: r["warm_mlp"]["rounds"]),
                         warm_geo=mean(lambda r: r["warm_geo"]["rounds"])),
        mean_ms=dict(cold=mean(lambda r: r["cold_ms"]), warm_mlp=mean(lambda r: r["warm_ms"]),
                     predict=mean(lambda r: r["predict_ms"]), warm_geo=mean(lambda r: r["geo_ms"])),
        mean_guess_rel_l2=dict(mlp=mean(lambda r: r["guess_rel_l2"]["mlp"]),
                               geo=mean(lambda r: r["guess_rel_l2"]["geo"])),
        max_warm_vs_cold_rel=max(max(r["warm_vs_cold_rel_max"].values()) for r in rows),
        cases=rows)
    if log is not None:
        log.close(**{k: v for k, v in summary.items() if k != "cases"})
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    sys.exit(main())

"""Launch-configuration autotuner.

For a plan and a representative problem it times the eikonal forward (and
optionally the adjoint) under each candidate configuration -- lanes per vertex
in a relaxation round, grid of a round, launches between convergence checks,
queue split over the XCDs or not, then the cold forward's hold-back (bucket
width in units of the front's mean advance per round, and when the next bucket
opens) -- keeps the fastest, and records the rounds/levels that carried work so
that graph-captured iterations can be given launch budgets.  tune_hold searches
the hold-back alone, also for the ordered warm start (gbp_plan_set_warm_order:
the forward solves cold, its evaluation order keyed by a guess of the solution).  Results are cached in a JSON file
keyed by the mesh size class (override the path with GBP_TUNE_CACHE).
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import binding as B

SPACE = [dict(lanes=lanes, sweep_blocks=sb, level_blocks=2048, sync_batch=bt, split=sp)
         for sp in (1, 0) for lanes in (8, 16, 32) for sb in (256, 512, 768, 1024, 1536, 2048)
         for bt in (16, 32, 64)]
LEVEL_SPACE = (256, 512, 1024, 2048)   # searched second, with the best of SPACE
# a short list for plans of millions of vertices, where every trial costs a
# forward and backward of the whole union (16 lanes, convergence read every 16
# launches, 2048 blocks per level: the full search's picks on such plans)
SPACE_LARGE = [dict(lanes=16, sweep_blocks=sb, level_blocks=2048, sync_batch=16, split=sp)
               for sp in (1, 0) for sb in (768, 1024, 2048)]
# hold-back candidates, searched last: (bucket width / mean front advance per round,
# buckets past the current one that propagate, opening threshold / vertices one
# round's grid takes at once, None: open a bucket every round); (0, 0, 0) is off
HOLD_SPACE = ((0, 0, 0.0), (1, 2, None), (2, 0, 1.0), (2, 0, 2.0), (3, 0, 1.0), (4, 0, 1.0), (4, 0, 2.0),
              (4, 0, 4.0))


def cache_path() -> str:
    return os.environ.get("GBP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gbp", "launch.json"))


def size_key(plan: B.Plan) -> str:
    b = lambda x: 2 ** int(round(math.log2(max(x, 1))))
    return f"gfx950/v{b(plan.n_v)}/e{b(plan.n_e)}"


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(db):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(fn, repeats):
    ts = []
    for _ in range(repeats):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune(plan: B.Plan, D, vscale, root_node, root_t, backward=True, space=None, repeats=3,
         use_cache=True, save=True, hold=None):
    """Pick and apply the fastest launch configuration; returns its record
    (configuration, ms per forward[+backward], rounds, levels).  Turns the plan's
    warm order off (see tune_hold for the ordered warm start).  The adjoint's grid
    and the hold-back are searched after the launch space when `space` is the
    full one (hold: None) or when hold is True."""
    B.set_warm_order(plan, False)
    key = size_key(plan)
    db = _load() if use_cache else {}
    if use_cache and key in db:
        rec = db[key]
        B.set_launch(plan, rec["lanes"], rec["sweep_blocks"], rec["level_blocks"], rec.get("sync_batch", 16))
        B.set_queue_split(plan, rec.get("split", 1))
        B.set_hold(plan, rec.get("hold_delta", 0.0), rec.get("hold_window", 0), rec.get("hold_open", 0))
        return dict(rec, cached=True)
    gT = torch.ones(plan.n_v, dtype=torch.float32, device=D.device)
    T = torch.empty(plan.n_v, dtype=torch.float32, device=D.device)

    def run():
        B.eikonal_forward(plan, D, vscale, root_node, root_t, out=T)
        if backward:
            B.eikonal_backward(plan, D, vscale, root_node, root_t, T, gT, want_D=False)

    best = None
    for cfg in (space or SPACE):
        B.set_launch(plan, cfg["lanes"], cfg["sweep_blocks"], cfg["level_blocks"], cfg["sync_batch"])
        B.set_queue_split(plan, cfg["split"])
        run()                                    # warm-up
        ms = _time(run, repeats)
        if best is None or ms < best["ms"]:
            best = dict(cfg, ms=ms)
    if backward and space is None:
        for lb in LEVEL_SPACE:
            cfg = dict(best, level_blocks=lb)
            B.set_launch(plan, cfg["lanes"], cfg["sweep_blocks"], lb, cfg["sync_batch"])
            B.set_queue_split(plan, cfg["split"])
            run()
            ms = _time(run, repeats)
            if ms < best["ms"]:
                best = dict(cfg, ms=ms)
    B.set_launch(plan, best["lanes"], best["sweep_blocks"], best["level_blocks"], best["sync_batch"])
    B.set_queue_split(plan, best["split"])
    best.update(hold_delta=0.0, hold_window=0, hold_open=0)
    if (space is None) if hold is None else hold:
        best.update(tune_hold(plan, D, vscale, root_node, root_t, backward=backward, repeats=repeats))
    run()
    best.update(B.last_counts(plan))
    if save:
        db = _load()
        db[key] = best
        _save(db)
    return dict(best, cached=False)


def tune_hold(plan: B.Plan, D, vscale, root_node, root_t, guess=None, backward=True, repeats=3):
    """Search the hold-back (HOLD_SPACE) in the plan's current launch
    configuration and apply the fastest; returns (hold_delta, hold_window,
    hold_open, ms).  guess: time ordered warm forwards from it instead of cold
    ones (the plan's warm order is left on; guess must not be the output)."""
    ordered = guess is not None
    gT = torch.ones(plan.n_v, dtype=torch.float32, device=D.device)
    T = torch.empty(plan.n_v, dtype=torch.float32, device=D.device)
    lanes, sweep_blocks = B.get_launch(plan)["lanes"], B.get_launch(plan)["sweep_blocks"]

    def run():
        B.eikonal_forward(plan, D, vscale, root_node, root_t, T_init=guess, out=T)
        if backward:
            B.eikonal_backward(plan, D, vscale, root_node, root_t, T, gT, want_D=False)

    B.set_warm_order(plan, False)
    B.set_hold(plan, 0.0)
    B.eikonal_forward(plan, D, vscale, root_node, root_t, out=T)
    fin = torch.isfinite(T)
    rounds = max(B.last_counts(plan)["rounds"], 1)
    span = float(T[fin].max() - T[fin].min()) if bool(fin.any()) else 0.0
    unit = span / rounds                        # mean advance of the front per round
    cap = sweep_blocks * (256 // lanes)
    B.set_warm_order(plan, ordered)
    best = None
    for mult, window, frac in HOLD_SPACE:
        if mult and not unit > 0:
            continue
        cfg = dict(hold_delta=mult * unit, hold_window=window,
                   hold_open=(1 << 30) if frac is None else int(frac * cap))
        B.set_hold(plan, cfg["hold_delta"], window, cfg["hold_open"])
        run()
        ms = _time(run, repeats)
        if best is None or ms < best["ms"]:
            best = dict(cfg, ms=ms)
    B.set_hold(plan, best["hold_delta"], best["hold_window"], best["hold_open"])
    run()
    return best


def budgets(plan: B.Plan, margin=1.25, extra=16, gs=32):
    """Launch budgets for a captured iteration from the last synchronous counts
    (relaxation rounds, adjoint levels and, where the parent graph had cycles,
    the Gauss-Seidel sweeps they needed)."""
    c = B.last_counts(plan)
    info = B.backward_info(plan)
    gs_need = int(math.ceil(info["gs_sweeps"] * margin)) + extra if info["cyclic"] > 0 else 0
    return dict(round_budget=int(math.ceil(c["rounds"] * margin)) + extra,
                level_budget=int(math.ceil(c["levels"] * margin)) + extra, gs_budget=max(gs, gs_need))

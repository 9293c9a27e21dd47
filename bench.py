#!/usr/bin/env python3
"""Geodesic-BP iterations per second on one MI355X.

One step = one full Geodesic-BP iteration on the synthetic 500k-vertex
biventricular shell: cold eikonal solve (active-list relaxation of Alg. 2),
lead-field ECG (12 leads x 500 steps of 1 ms), misfit against a target ECG made
from a hidden seeded parameter set, ECG backward, eikonal adjoint (parents
recomputed, gradients w.r.t. the nodal velocity scale and the root onsets), and
one Adam step on those parameters.  All of it runs in libgbp's HIP kernels on
torch's current stream; inputs are resident in HBM before timing starts.

The timed iterations go through the library's enqueue-only calls: the forward
and the backward take launch budgets (the last synchronous solve's rounds and
levels + 8), no host synchronisation falls inside an iteration, and each
iteration's device-side status is read at its end.  The same iterations through
the synchronous calls are timed first; if any enqueue-only iteration missed its
budgets, the synchronous figure is the one reported.

Prints ONE JSON line.  `python bench.py --gpus 1 --steps 20 --warmup 3`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "Geodesic-BP iters/s (FIM+adjoint+ECG) at 500k nodes; speedup vs plain"
# Nominal FP32 operations of one closed-form local solve (vertex, edge and
# interior KKT candidates, see local_solve.h; an FMA counts as two operations).
FLOP_PER_FACE = 185.0
# Bytes a relaxation round gathers per local problem (not the algorithmic count):
# the incidence entry (4 B), the element's vertex ids (16 B) and Gram record
# (32 B), and the three face values (12 B).
GATHERED_BYTES_PER_FACE = 64.0


def sweep_bytes(n_v, n_e):
    """Algorithmic bytes of one full relaxation sweep over every local problem:
    per element its 4 vertex ids (16 B) and the 6 entries of its metric (24 B),
    4 incidence entries (16 B); per vertex the coordinates (12 B), the time read
    and written (8 B) and the incidence pointer (4 B).  Each element's data counts
    once per sweep although 4 local problems use it."""
    return n_e * (16 + 24) + 4 * n_e * 4 + n_v * (12 + 4 + 4 + 4)


def bytes_per_local_problem(n_v, n_e):
    """A solve's algorithmic bytes per local problem evaluated: the full-sweep
    bytes spread over the sweep's 4 n_e local problems (a solve that evaluates k
    local problems moves k / (4 n_e) full sweeps)."""
    return sweep_bytes(n_v, n_e) / (4.0 * n_e)


def adjoint_bytes(n_v, n_e, want_D=False):
    """Algorithmic bytes of one backward: the parent recompute (one full sweep),
    the lambda pass (per vertex 3 parent ids, 3 weights, lambda and the incoming
    gradient: 32 B), the velocity-scale gradient (4 B per vertex) and, if asked
    for, the tensor gradient (24 B per element)."""
    return sweep_bytes(n_v, n_e) + 32 * n_v + 4 * n_v + (24 * n_e if want_D else 0)


def ecg_bytes(n_v, L):
    """Algorithmic bytes of the ECG forward and backward: T and the lead weights
    read by each (4 + 4 L B per vertex), the gradient written by the backward."""
    return 2 * n_v * (4 + 4 * L) + 4 * n_v
# MI355X peaks: FP32 vector without packed math (256 CU x 64 lanes x 2 x 2.4 GHz)
# and HBM3E bandwidth.
PEAK_FP32_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0   # dense bf16 matrix-core peak


FORMS = ("warm", "points", "leadfield", "fista", "slice", "batched", "learned", "inverse")


# Launch configuration of the plain iteration on this workload: the autotuner's
# search (autotune.tune) followed by finer sweeps of the relaxation grid and the
# hold-back around its pick, timed with this script (16 lanes per vertex, 768
# blocks per relaxation round -- three per CU: 1024 and 896 were 2-3% slower, 640
# and 512 slower still --, convergence read every 16 launches, 2048 blocks per
# adjoint level, queue split over the XCDs; hold-back buckets of 2.5 ms, no window,
# the next bucket opened while fewer than 16384 vertices are queued).  Fixed so
# that a profiled run of the same command times the same kernels; --tune
# searches again.
DEFAULT_LAUNCH = "16,768,16,2048,1"
DEFAULT_HOLD = "2.5,0,16384"


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nodes", type=int, default=500_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel timing pass")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="host threads of the CPU baseline (0: min(16, cores))")
    ap.add_argument("--cpu-only", action="store_true",
                    help="time only the CPU baseline on this host (no GPU) and print it")
    ap.add_argument("--no-tune", action="store_true", help="keep the library's default launch configuration")
    ap.add_argument("--tune", action="store_true", help="run the autotuner instead of the fixed configuration")
    ap.add_argument("--launch", default=DEFAULT_LAUNCH, metavar="LANES,BLOCKS,BATCH,LEVEL_BLOCKS,SPLIT",
                    help="launch configuration (default: the one tuned for the benchmark workload)")
    ap.add_argument("--hold", default=DEFAULT_HOLD, metavar="DELTA,WINDOW,OPEN_BELOW",
                    help="the cold forward's hold-back (bucket width in ms, window, opening threshold; "
                         "delta 0 turns it off)")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip every form beside the plain iteration")
    ap.add_argument("--forms", default=",".join(FORMS), metavar="LIST",
                    help="comma-separated subset of " + ",".join(FORMS) + " (default: all)")
    ap.add_argument("--form-steps", type=int, default=10)
    ap.add_argument("--calibrate-copy", type=float, default=0.0, metavar="MIB",
                    help="run one plain copy of this many MiB first (a known-size kernel for "
                         "scaling rocprofv3 FETCH_SIZE/WRITE_SIZE counters)")
    return ap.parse_args()


PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")


def stored_mfma(kernel):
    """Matrix-core figures of an ECG kernel from the committed counter summary,
    while its source is unchanged (else None)."""
    from paper_2308_08410_amd import profiling
    t = profiling.read_summary(os.path.join(PROFILES, f"{kernel}_shell500k_mfma.md"))
    if not t or t.get("source_hash") != profiling.source_hash(kernel, "ecg.hip"):
        return None
    return t


def stored_valu(kernel):
    """Vector-ALU figures of an ECG kernel (VALU and transcendental instructions
    per launch) from the committed counter summary, while its source is unchanged
    (else None)."""
    from paper_2308_08410_amd import profiling
    t = profiling.read_summary(os.path.join(PROFILES, f"{kernel}_shell500k_valu.md"))
    if not t or t.get("source_hash") != profiling.source_hash(kernel, "ecg.hip"):
        return None
    return t


def stored_traffic(kernel="k_sweep"):
    """Measured HBM bytes per launch of a kernel on this workload, from the
    committed counter summary, while the kernel's source is unchanged since the
    counters were taken (else None)."""
    from paper_2308_08410_amd import profiling
    t = profiling.read_summary(os.path.join(PROFILES, f"{kernel}_shell500k_traffic.md"))
    if not t or t.get("source_hash") != profiling.source_hash(kernel):
        return None
    return t["bytes_per_launch"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_state(prob, dev, torch, gi, B):
    """Plan, device inputs, a target ECG from hidden parameters, and the
    parameters being fitted (velocity scale, root onsets) with Adam moments."""
    plan = B.Plan(prob.xyz, prob.tets)
    # the backward of a step gets the same, unchanged D, scales and onsets as the
    # forward before it: it may keep the element metric that forward built
    B.set_input_reuse(plan, True)
    f32 = lambda a: torch.as_tensor(a, dtype=torch.float32, device=dev).contiguous()
    st = dict(plan=plan, D=f32(prob.D), W=f32(prob.W), rn=torch.as_tensor(prob.root_node, device=dev))
    ap = prob.ap
    st["ap"] = B.make_ap(ap["K0"], ap["K1"], ap["tau"], ap["t0"], ap["dt"], ap["n_steps"])
    # hidden parameter set -> target ECG
    vs_true = f32(gi.smooth_field(prob.xyz, 0.7, 1.3, seed=20))
    rt_true = f32(prob.root_t)
    T_true, _ = B.eikonal_forward(plan, st["D"], vs_true, st["rn"], rt_true)
    st["target"] = B.ecg_forward(T_true, st["W"], st["ap"]).clone()
    # initial guess of the fit
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(21))
    st["vs_start"] = np.ones(prob.n_v, np.float32)
    st["rt_start"] = (prob.root_t + rng.uniform(-5, 5, size=len(prob.root_t))).astype(np.float32)
    st["vs"] = f32(st["vs_start"])
    st["rt"] = f32(st["rt_start"])
    for k in ("vs", "rt"):
        st["m_" + k] = torch.zeros_like(st[k])
        st["v_" + k] = torch.zeros_like(st[k])
    st["k"] = 0
    return st


def gbp_step(st, B):
    st["k"] += 1
    T, stats = B.eikonal_forward(st["plan"], st["D"], st["vs"], st["rn"], st["rt"])
    ecg = B.ecg_forward(T, st["W"], st["ap"])
    loss, G = B.ecg_loss(ecg, st["target"])
    gT = B.ecg_backward(T, st["W"], st["ap"], G)
    _, dvs, drt = B.eikonal_backward(st["plan"], st["D"], st["vs"], st["rn"], st["rt"], T, gT,
                                     want_D=False)
    B.adam_step(st["vs"], dvs, st["m_vs"], st["v_vs"], st["k"], lr=0.01, lo=0.2, hi=5.0)
    B.adam_step(st["rt"], drt, st["m_rt"], st["v_rt"], st["k"], lr=0.5)
    return loss, stats


def enqueue_budgets(st, B, margin=8):
    """Launch budgets of the enqueue-only calls from the last synchronous solve of
    this fit: its rounds and levels + margin; Gauss-Seidel sweeps: 8 when the last
    backward's level walk finished every vertex (no parent-graph cycle longer than
    two), else twice the sweeps it needed (at least 32)."""
    c = B.last_counts(st["plan"])
    info = B.backward_info(st["plan"])
    gs = 8 if info["cyclic"] == 0 else max(32, 2 * info["gs_sweeps"])
    return dict(round_budget=c["rounds"] + margin, level_budget=c["levels"] + margin, gs_budget=gs)


def enqueue_step(st, B, bud):
    """gbp_step through the enqueue-only calls: the forward and the backward take
    fixed launch budgets, so no host synchronisation falls inside the iteration;
    the device-side status is read at its end.  True if the forward converged and
    the adjoint settled within the budgets and no input error was flagged."""
    plan = st["plan"]
    st["k"] += 1
    T = B.eikonal_forward_async(plan, st["D"], st["vs"], st["rn"], st["rt"], bud["round_budget"])
    ecg = B.ecg_forward(T, st["W"], st["ap"])
    loss, G = B.ecg_loss(ecg, st["target"])
    gT = B.ecg_backward(T, st["W"], st["ap"], G)
    _, dvs, drt = B.eikonal_backward_async(plan, st["D"], st["vs"], st["rn"], st["rt"], T, gT,
                                           bud["level_budget"], bud["gs_budget"], want_D=False)
    B.adam_step(st["vs"], dvs, st["m_vs"], st["v_vs"], st["k"], lr=0.01, lo=0.2, hi=5.0)
    B.adam_step(st["rt"], drt, st["m_rt"], st["v_rt"], st["k"], lr=0.5)
    s = B.plan_status(plan)          # synchronises at the end of the iteration
    return loss, s["err"] == 0 and s["forward_converged"] and s["backward_settled"]


def _replay_timed(step, steps, torch):
    step.launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        step.launch()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _warm_accuracy(step, plan, D, vs, rn, rt, T, B, torch):
    """One more replay from saved parameters, then a cold solve with the same
    parameters: max |T_warm - T_cold| / max |T_cold| over reached vertices."""
    vs0, rt0 = vs.clone(), rt.clone()
    step.launch()
    torch.cuda.synchronize()
    st = B.plan_status(plan)
    Tc, _ = B.eikonal_forward(plan, D, vs0, rn, rt0)
    fin = torch.isfinite(Tc)
    err = float((T[fin] - Tc[fin]).abs().max() / Tc[fin].abs().max())
    return err, st


def warm_single_form(st, prob, steps, torch, B, autotune, ordered=False):
    """The same 500k iteration as one HIP-graph replay whose forward starts from
    the previous iteration's activation times: two-sided, or (ordered) a cold
    solve whose hold-back is keyed by them (hold-back searched for that)."""
    plan, dev = st["plan"], st["D"].device
    hold0 = B.get_hold(plan)
    L = prob.W.shape[1]
    S = prob.ap["n_steps"]
    bt = B.Batch([0, prob.n_v], S)
    T = torch.empty(prob.n_v, dtype=torch.float32, device=dev)
    ecg = torch.empty((1, S, L), dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    tgt = st["target"].reshape(1, S, L).contiguous()
    B.eikonal_forward(plan, st["D"], st["vs"], st["rn"], st["rt"], out=T)
    B.eikonal_backward(plan, st["D"], st["vs"], st["rn"], st["rt"], T, torch.ones_like(T), want_D=False)
    hold = None
    if ordered:
        hold = autotune.tune_hold(plan, st["D"], st["vs"], st["rn"], st["rt"], guess=T.clone(), repeats=1)
        B.eikonal_forward(plan, st["D"], st["vs"], st["rn"], st["rt"], T_init=T, out=T)
    # budgets: the ordered (cold) solve's own counts + 8, as the plain iteration's; the
    # two-sided solve is sized from a cold solve and gets room
    bud = (autotune.budgets(plan, margin=1.0, extra=8) if ordered
           else autotune.budgets(plan, margin=1.5, extra=32))
    step = B.Step(plan, bt, st["D"], st["vs"], st["rn"], st["rt"], st["W"], st["ap"], tgt, T, ecg, loss,
                  warm=True, **bud)
    ms = _replay_timed(step, steps, torch)
    work = B.forward_work(plan)
    err, status = _warm_accuracy(step, plan, st["D"], st["vs"], st["rn"], st["rt"], T, B, torch)
    step.close()
    B.set_warm_order(plan, False)
    B.set_hold(plan, *hold0)
    return dict(iters_per_s=1000.0 / ms, ms_per_step=ms, max_rel_T_vs_cold=err,
                converged=bool(status["forward_converged"] and status["backward_settled"]), budgets=bud,
                local_problems_per_step=work["face_solves"], hold=hold)


def point_root_form(st, prob, steps, torch, gi, B, n_points=100, seed=41):
    """The same 500k iteration with its roots at points inside endocardial
    elements (Sec. 2.3 Eq. (upwind_xi); the paper fits 100 root points): the
    points, their onsets and the velocity scale are fitted.  One step: vertex
    onsets of the points, cold forward, ECG, loss, ECG backward, adjoint, the
    chain rule to the points, three Adam updates."""
    import numpy as np
    dev = st["D"].device
    plan, D = st["plan"], st["D"]
    cand = gi.tets_touching(prob.tets, prob.extra["endo"])
    k, X, t = gi.random_point_roots(prob.xyz, prob.tets, cand, n_points, 0.0, 20.0, seed=seed)
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=dev)
    s = dict(k=torch.as_tensor(k, device=dev), X=f32(X), t=f32(t), vs=f32(np.ones(prob.n_v)))
    for name in ("X", "t", "vs"):
        s["m_" + name] = torch.zeros_like(s[name])
        s["v_" + name] = torch.zeros_like(s[name])

    def step(kk):
        node, onset = B.point_roots(plan, D, s["vs"], s["k"], s["X"], s["t"])
        T, stats = B.eikonal_forward(plan, D, s["vs"], node, onset)
        ecg = B.ecg_forward(T, st["W"], st["ap"])
        loss, G = B.ecg_loss(ecg, st["target"])
        gT = B.ecg_backward(T, st["W"], st["ap"], G)
        _, dvs, donset = B.eikonal_backward(plan, D, s["vs"], node, onset, T, gT, want_D=False)
        dt, dx = B.point_roots_backward(plan, D, s["vs"], s["k"], s["X"], donset, dL_dvscale=dvs)
        B.adam_step(s["vs"], dvs, s["m_vs"], s["v_vs"], kk, lr=0.01, lo=0.2, hi=5.0)
        B.adam_step(s["t"], dt, s["m_t"], s["v_t"], kk, lr=0.5)
        B.adam_step(s["X"], dx, s["m_X"], s["v_X"], kk, lr=0.01)
        return loss, stats

    # 400 vertex roots spread the first front over the endocardium: the hold-back
    # tuned for the plain form's 5 roots only adds rounds here (measured), so this
    # form runs in the plain relaxation order
    hold = B.get_hold(plan)
    B.set_hold(plan, 0.0)
    try:
        for kk in range(1, 3):
            step(kk)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for kk in range(3, 3 + steps):
            loss, stats = step(kk)
        e1.record()
        torch.cuda.synchronize()
    finally:
        B.set_hold(plan, *hold)
    ms = e0.elapsed_time(e1) / steps
    return dict(points=n_points, iters_per_s=1000.0 / ms, ms_per_step=ms, rounds=stats["rounds"],
                loss=float(loss[0]))


def fista_form(st, torch, B, n_faces=4_000_000, seed=43):
    """The forward with the paper's own local solver (FISTA, Alg. 1, tightened
    step constant) against the exact predicated solve on the same 500k problem:
    forward time and max relative deviation from the exact solve per iteration
    count, and the cost of one local problem for each solver (a batch of seeded
    random faces)."""
    import numpy as np
    plan, D, vs, rn, rt = st["plan"], st["D"], st["vs"], st["rn"], st["rt"]
    dev = D.device

    def timed(fn, k=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            out = fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k, out

    ms_e, (Te, se) = timed(lambda: B.eikonal_forward(plan, D, vs, rn, rt))
    Te = Te.clone()
    fin = torch.isfinite(Te)
    runs = []
    tuned = B.get_launch(plan)
    try:
        # FISTA rounds are arithmetic-bound: 8 lanes per vertex (three local problems
        # per lane) and a full grid of 2048 blocks
        B.set_launch(plan, 8, 2048, tuned["level_blocks"], tuned["sync_batch"])
        for n_f in (32, 64, 128):
            B.set_local_solver(plan, "fista", n_f, "tight")
            ms, (Tf, sf) = timed(lambda: B.eikonal_forward(plan, D, vs, rn, rt))
            err = float((Tf[fin] - Te[fin]).abs().max() / Te[fin].abs().max())
            runs.append(dict(n_f=n_f, forward_ms=ms, rel_max_vs_exact=err, rounds=sf["rounds"],
                             slowdown_vs_exact=ms / ms_e))
        # per-face iteration counts from the rate Eq. (fista_convergence) for a value
        # tolerance per local problem (ms), capped at 1024
        for tau in (1e-2, 1e-3):
            B.set_local_solver(plan, "fista", 1024, "tight")
            B.set_fista_tolerance(plan, tau)
            ms, (Tf, sf) = timed(lambda: B.eikonal_forward(plan, D, vs, rn, rt))
            err = float((Tf[fin] - Te[fin]).abs().max() / Te[fin].abs().max())
            runs.append(dict(tau_ms=tau, n_f_cap=1024, forward_ms=ms, rel_max_vs_exact=err,
                             rounds=sf["rounds"], slowdown_vs_exact=ms / ms_e))
    finally:
        B.set_fista_tolerance(plan, 0.0)
        B.set_local_solver(plan, "exact")
        B.set_launch(plan, tuned["lanes"], tuned["sweep_blocks"], tuned["level_blocks"], tuned["sync_batch"])
    r = np.random.Generator(np.random.PCG64(seed))
    A = r.normal(size=(n_faces, 3, 3)).astype(np.float32)
    Q = np.einsum("nki,nkj->nij", A, A) + 0.1 * np.eye(3, dtype=np.float32)
    Q6 = torch.as_tensor(np.stack([Q[:, 0, 0], Q[:, 1, 1], Q[:, 2, 2], Q[:, 0, 1], Q[:, 0, 2], Q[:, 1, 2]], 1),
                         device=dev).contiguous()
    Phi = torch.as_tensor(r.uniform(0, 1, size=(n_faces, 3)).astype(np.float32), device=dev)
    lip = B.local_solve(Q6, Phi, "fista", n_f=1, want_alpha=False, want_lip=True)[2]
    per_face = {"exact": timed(lambda: B.local_solve(Q6, Phi, "exact", want_alpha=False))[0] * 1e6 / n_faces}
    for n_f in (16, 32, 64, 128):
        per_face[f"fista_{n_f}"] = timed(lambda: B.local_solve(Q6, Phi, "fista", n_f=n_f, lip=lip,
                                                               want_alpha=False))[0] * 1e6 / n_faces
    return dict(exact_forward_ms=ms_e, exact_rounds=se["rounds"], fista_launch=dict(lanes=8, sweep_blocks=2048),
                runs=runs, ns_per_local_problem=per_face)


def learned_form(st, prob, torch, B, n_train=128, steps=1500, batch=16384, n_test=3, seed=5):
    """The learned warm start on the benchmark mesh: the network (bf16 matrix-core
    kernels) trained on n_train cold solves with random roots (1-8), onsets and
    smooth velocity scales (beyond 128 solves the held-out guess error stops
    improving: 13.3% at 128 and 512 solves, 13.0% at 2048), then on held-out
    cases: the guess error, and the cold solve against the solve warm-started
    from the guess (local problems, rounds, time, agreement)."""
    import numpy as np
    from paper_2308_08410_amd import warmstart as WS
    plan, D = st["plan"], st["D"]
    t0 = time.perf_counter()
    data = WS.make_dataset(plan, prob.xyz, D, prob.extra["endo"], n_train, seed=1000 * seed, scale_bank=32)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    ws = WS.WarmStart(prob.xyz, prob.extra["node_fibre"], max_rows=batch, seed=seed)
    t0 = time.perf_counter()
    hist = WS.train(ws, data, steps, batch=batch, lr=1e-3, log_every=max(1, steps // 5))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del data
    test = WS.make_dataset(plan, prob.xyz, D, prob.extra["endo"], n_test, seed=7_000_000 + seed)
    rows = WS.evaluate(ws, plan, D, test, repeats=2)
    mean = lambda f: float(np.mean([f(r) for r in rows]))
    return dict(
        train_solves=n_train, train_steps=steps, batch=batch, data_seconds=t_data, train_seconds=t_train,
        loss_first=hist[0][1], loss_last=hist[-1][1], held_out=n_test,
        guess_rel_l2=dict(mlp=mean(lambda r: r["guess_rel_l2"]["mlp"]), geo=mean(lambda r: r["guess_rel_l2"]["geo"])),
        local_problems=dict(cold=mean(lambda r: r["cold"]["face_solves"]),
                            warm_mlp=mean(lambda r: r["warm_mlp"]["face_solves"]),
                            warm_mlp_ordered=mean(lambda r: r["warm_mlp_ordered"]["face_solves"])),
        rounds=dict(cold=mean(lambda r: r["cold"]["rounds"]), warm_mlp=mean(lambda r: r["warm_mlp"]["rounds"]),
                    warm_mlp_ordered=mean(lambda r: r["warm_mlp_ordered"]["rounds"])),
        ms=dict(cold=mean(lambda r: r["cold_ms"]), warm_mlp_incl_prediction=mean(lambda r: r["warm_ms"]),
                warm_mlp_ordered_incl_prediction=mean(lambda r: r["ordered_ms"]),
                predict=mean(lambda r: r["predict_ms"])),
        fallbacks=int(sum(r["warm_mlp"]["fallback"] for r in rows)),
        max_rel_T_warm_vs_cold=max(r["warm_vs_cold_rel_max"]["mlp"] for r in rows),
        max_rel_T_ordered_vs_cold=max(r["warm_vs_cold_rel_max"]["mlp_ordered"] for r in rows))


def lead_field_form(st, prob, torch, B, reps=5):
    """Lead weights W = K Z assembled on the device for the benchmark's 12
    electrodes (Sec. 2.4): time per assembly and the largest deviation from the
    weights the benchmark uses (assembled on the host in float64)."""
    import numpy as np
    dev = st["D"].device
    e = torch.as_tensor(np.asarray(prob.extra["electrodes"], np.float32), device=dev)
    W = B.lead_field(st["plan"], e)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        B.lead_field(st["plan"], e, out=W)
    e1.record()
    torch.cuda.synchronize()
    dev_max = float((W - st["W"]).abs().max() / st["W"].abs().max())
    return dict(ms=e0.elapsed_time(e1) / reps, n_leads=int(e.shape[0]), rel_max_vs_host=dev_max)


def slice_form(dev, steps, torch, gi, B, sizes=(2_700, 250_000)):
    """The iteration on triangle meshes (d = 2): the 2-D left-ventricular slice of
    the paper's 2-D study (~2.7k nodes, 8 roots, 7 leads) and a finer slice.  One
    step: forward, ECG, loss, ECG backward, adjoint (scale, onsets), two Adam
    updates, fitting to the ECG of a hidden scale field."""
    import numpy as np
    out = []
    for n in sizes:
        p = gi.annulus_problem(n)
        f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=dev)
        plan = B.TriPlan(p.xyz, p.tets)
        D, W = f32(p.D), f32(p.W)
        rn = torch.as_tensor(p.root_node, device=dev)
        a = p.ap
        ap = B.make_ap(a["K0"], a["K1"], a["tau"], a["t0"], a["dt"], a["n_steps"])
        vs_true = f32(np.random.Generator(np.random.PCG64(8)).uniform(0.8, 1.2, size=p.n_v))
        T_true, _ = B.tri_forward(plan, D, vs_true, rn, f32(p.root_t))
        target = B.ecg_forward(T_true, W, ap).clone()
        vs, rt = f32(np.ones(p.n_v)), f32(p.root_t + 2.0)
        m_vs, v_vs, m_rt, v_rt = (torch.zeros_like(x) for x in (vs, vs, rt, rt))

        def step(k):
            T, st = B.tri_forward(plan, D, vs, rn, rt)
            ecg = B.ecg_forward(T, W, ap)
            loss, G = B.ecg_loss(ecg, target)
            gT = B.ecg_backward(T, W, ap, G)
            _, dvs, drt = B.tri_backward(plan, D, vs, rn, rt, T, gT, want_D=False)
            B.adam_step(vs, dvs, m_vs, v_vs, k, lr=0.01, lo=0.2, hi=5.0)
            B.adam_step(rt, drt, m_rt, v_rt, k, lr=0.5)
            return loss, st

        for k in range(1, 3):
            step(k)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(3, 3 + steps):
            loss, st = step(k)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out.append(dict(n_v=p.n_v, n_tri=p.n_e, iters_per_s=1000.0 / ms, ms_per_step=ms, rounds=st["rounds"],
                        loss=float(loss[0])))
        plan.close()
    return out


def batched_form(dev, steps, torch, gi, B, autotune, n_inst=64, n_meshes=8, seed=31):
    """Many uneven meshes and parameter sets as one union plan, one HIP-graph
    replay per iteration for all instances (forward -- cold, then warm-started
    from the previous iteration -- batched ECG and misfit, adjoint, Adam),
    launch configuration from the autotuner."""
    import numpy as np
    from paper_2308_08410_amd.batch import concat, shift_roots, union_mesh
    t0 = time.time()
    wl = gi.batched_workload(n_inst=n_inst, n_meshes=n_meshes, seed=seed)
    meshes = wl.meshes
    inst = [meshes[k] for k in wl.mesh_of]
    xyz, tets, voff, _ = union_mesh([m.xyz for m in inst], [m.tets for m in inst])
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=dev)
    D, W = f32(concat([m.D for m in inst])), f32(concat([m.W for m in inst]))
    rn = torch.as_tensor(shift_roots(wl.root_node, voff), device=dev)
    rt_true = f32(concat(wl.root_t_true))
    rt = f32(concat(wl.root_t_start))
    vs = f32(np.ones(int(voff[-1])))
    vs_true = wl.vscale_true
    plan = B.Plan(xyz, tets)
    B.set_input_reuse(plan, True)   # each step's backward gets its forward's inputs
    ap = inst[0].ap
    S, L = ap["n_steps"], W.shape[1]
    apc = B.make_ap(ap["K0"], ap["K1"], ap["tau"], ap["t0"], ap["dt"], S)
    bt = B.Batch(voff, S)
    t_setup = time.time() - t0
    T_true, _ = B.eikonal_forward(plan, D, f32(concat(vs_true)), rn, rt_true)
    target = B.ecg_forward_batched(bt, T_true, W, apc).clone()
    tune = autotune.tune(plan, D, vs, rn, rt, use_cache=False, save=False, repeats=1)
    out = dict(instances=n_inst, distinct_meshes=n_meshes, mesh_sizes=[int(m.n_v) for m in meshes],
               total_vertices=int(voff[-1]), total_tets=int(len(tets)), setup_s=t_setup,
               launch=dict(lanes=tune["lanes"], sweep_blocks=tune["sweep_blocks"], split=tune["split"]))
    out["launch"]["hold"] = B.get_hold(plan)
    vs_start, rt_start = vs.clone(), rt.clone()
    hold0 = B.get_hold(plan)
    for mode in ("cold", "warm", "warm_ordered"):
        warm = mode != "cold"
        vs.copy_(vs_start)
        rt.copy_(rt_start)
        T = torch.empty(len(xyz), dtype=torch.float32, device=dev)
        B.eikonal_forward(plan, D, vs, rn, rt, out=T)
        B.eikonal_backward(plan, D, vs, rn, rt, T, torch.ones_like(T), want_D=False)
        hold = None
        if mode == "warm_ordered":
            # the hold-back searched for forwards ordered by the last times
            hold = autotune.tune_hold(plan, D, vs, rn, rt, guess=T.clone(), repeats=1)
            B.eikonal_forward(plan, D, vs, rn, rt, T_init=T, out=T)
        # a two-sided warm solve can need more rounds than the cold one it is sized from;
        # the cold and ordered solves get their own counts + 8, as the plain iteration
        bud = (autotune.budgets(plan, margin=2.0, extra=64) if mode == "warm"
               else autotune.budgets(plan, margin=1.0, extra=8))
        ecg = torch.empty((n_inst, S, L), dtype=torch.float32, device=dev)
        loss = torch.empty(n_inst, dtype=torch.float32, device=dev)
        step = B.Step(plan, bt, D, vs, rn, rt, W, apc, target, T, ecg, loss, warm=warm, **bud)
        ms = _replay_timed(step, steps, torch)
        work = B.forward_work(plan)          # the last replay's forward
        err, status = _warm_accuracy(step, plan, D, vs, rn, rt, T, B, torch)
        step.close()
        B.set_warm_order(plan, False)
        B.set_hold(plan, *hold0)
        # algorithmic bytes of one replayed iteration: the forward's local problems,
        # the backward, the ECG forward and backward (the small misfit and Adam aside)
        nv, ne = int(voff[-1]), int(len(tets))
        alg = (work["face_solves"] * bytes_per_local_problem(nv, ne) + adjoint_bytes(nv, ne)
               + ecg_bytes(nv, L))
        out[mode] = dict(
            hold=hold, ms_per_step=ms, instance_iters_per_s=n_inst * 1000.0 / ms,
            vertex_iters_per_s=int(voff[-1]) * 1000.0 / ms, max_rel_T_vs_cold=err,
            converged=bool(status["forward_converged"] and status["backward_settled"]), status=status,
            budgets=bud, backward=B.backward_info(plan), local_problems_per_step=work["face_solves"],
            roofline=dict(bound="hbm", algorithmic_bytes_per_step=alg,
                          achieved=alg / (ms * 1e-3) / 1e9, peak=PEAK_HBM_GBS, unit="GB/s",
                          frac=alg / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS))
    return out


def inverse_form(dev, torch, gi, B, iters=20, n_nodes=1_000_000, starts=16, seed=5):
    """The inverse problem (Sec. 2.4 Eq. (inverse_ecg)) as the multi-start fit:
    `starts` fits of the 1M-vertex shell (8 roots, hidden smooth scale in
    [0.5, 1.5]) as the instances of one union plan, every iteration one replay of
    the captured step (cold forwards, in the launch configuration and hold-back the
    autotuner picks for the union plan) for all starts; timed over `iters`
    iterations after two untimed ones, the misfit of every start before and after."""
    import numpy as np
    from paper_2308_08410_amd.inverse import MultiStartFit
    t0 = time.time()
    p, vs_true, rt0 = gi.multistart_workload(n_nodes, starts, 8, seed)
    a = p.ap
    f32 = lambda x: torch.as_tensor(np.ascontiguousarray(x, np.float32), device=dev)
    plan1 = B.Plan(p.xyz, p.tets)
    T_true, _ = B.eikonal_forward(plan1, f32(p.D), f32(vs_true), torch.as_tensor(p.root_node, device=dev),
                                  f32(p.root_t))
    apc = B.make_ap(a["K0"], a["K1"], a["tau"], a["t0"], a["dt"], a["n_steps"])
    target = B.ecg_forward(T_true, f32(p.W), apc).cpu().numpy()
    plan1.close()
    vs0 = [np.ones(p.n_v, np.float32) for _ in range(starts)]
    fit = MultiStartFit(p.xyz, p.tets, p.D, p.W, p.root_node, target, a, vs0, rt0, tune=True)
    t_setup = time.time() - t0
    fit.run(2, check_every=0)
    loss0 = fit.loss.detach().cpu().numpy().copy()
    out = fit.run(iters, check_every=iters)
    loss1 = fit.loss.detach().cpu().numpy().copy()
    st = B.plan_status(fit.plan)
    res = dict(nodes=int(p.n_v), tets=int(p.n_e), starts=starts, union_vertices=int(fit.voff[-1]),
               iters=iters, iters_per_s=out["iters_per_s"], start_iters_per_s=out["iters_per_s"] * starts,
               ms_per_iter=1000.0 / out["iters_per_s"], setup_s=t_setup, budgets=fit.budgets,
               launch={k: fit.tuned[k] for k in ("lanes", "sweep_blocks", "level_blocks", "sync_batch", "split",
                                                  "hold_delta", "hold_window", "hold_open")},
               loss_after_2=[float(x) for x in loss0], loss_after_last=[float(x) for x in loss1],
               converged=bool(st["forward_converged"] and st["backward_settled"] and st["err"] == 0))
    fit.step.close()
    fit.plan.close()
    return res


def host_info():
    """CPU model and logical core count of the host this runs on."""
    from paper_2308_08410_amd.runlog import host_info as info
    h = info()
    return dict(cpu_model=h["cpu_model"], nproc=h["nproc"])


def cpu_baseline(prob, vs, rt, threads):
    """The FP64 oracle, as it stands, timed on this host for one complete
    iteration of the benchmark workload itself (same mesh, inputs and seeds): Alg. 2
    (Jacobi), the parent map, the ECG forward, misfit and backward, the sparse
    adjoint and the Adam step.  The oracle's element and vertex loops run on
    `threads` host threads (OpenMP; the results do not depend on the count), numpy
    and scipy with as many BLAS threads."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle as O
    O.set_threads(threads)
    target = np.zeros((prob.ap["n_steps"], prob.W.shape[1]))
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        Minv = O.metric_inverse(prob.D, vs, prob.tets)
        T, st = O.fim(prob.xyz, prob.tets, Minv, prob.root_node, rt)
        t1 = time.perf_counter()
        par = O.parent_map(prob.xyz, prob.tets, Minv, prob.root_node, rt, T)
        t2 = time.perf_counter()
        e = O.ecg_forward(T, prob.W, prob.ap)
        _, G = O.ecg_loss(e, target)
        g = O.ecg_backward(T, prob.W, prob.ap, G)
        t3 = time.perf_counter()
        res = O.adjoint(prob.xyz, prob.tets, prob.D, vs, prob.root_node, rt, T, g, par=par)
        O.adam_step(vs, res["dvscale"], np.zeros_like(vs), np.zeros_like(vs), 1, lr=0.01)
        t4 = time.perf_counter()
    # the same oracle on one thread and on `threads`, over a bounded sample: a full
    # Alg. 2 solve on the 64k-vertex member of the same shell family
    import gbp_inputs as gi
    small = gi.shell_problem(64_000, seed=2, n_roots=5, n_leads=12)
    Minv_s = O.metric_inverse(small.D, None, small.tets)
    solve_s = {}
    for n in sorted({1, threads}):
        O.set_threads(n)
        with threadpool_limits(limits=n):
            ts = time.perf_counter()
            O.fim(small.xyz, small.tets, Minv_s, small.root_node, small.root_t)
            solve_s[str(n)] = time.perf_counter() - ts
    O.set_threads(1)
    total = t4 - t0
    return dict(value=1.0 / total, unit="iter/s", cores=threads, kind="oracle", **host_info(),
                thread_scaling=dict(sample=f"one Alg. 2 solve on the {small.n_v}-vertex member of the same "
                                           f"shell family", seconds=solve_s,
                                    speedup=solve_s["1"] / solve_s[str(threads)]),
                seconds=dict(eikonal=t1 - t0, parents=t2 - t1, ecg=t3 - t2, adjoint_adam=t4 - t3, total=total),
                sample=(f"one full FP64 oracle iteration on the benchmark workload itself ({prob.n_v} vertices, "
                        f"{prob.n_e} tets, same inputs): Alg. 2 Jacobi ({st['sweeps']} sweeps, "
                        f"{st['solves']} local problems), parents, ECG fwd/bwd, sparse adjoint, Adam; "
                        f"{threads} host threads; measured, not scaled"))


def cpu_threads(args):
    return args.cpu_threads if args.cpu_threads > 0 else min(16, os.cpu_count() or 1)


def cpu_only(args):
    """The CPU baseline alone (no GPU): the benchmark workload's inputs, the oracle."""
    import numpy as np
    import gbp_inputs as gi
    prob = gi.shell_problem(args.nodes, seed=2, n_roots=5, n_leads=12)
    rng = np.random.Generator(np.random.PCG64(21))
    rt = (prob.root_t + rng.uniform(-5, 5, size=len(prob.root_t))).astype(np.float32)
    cpu = cpu_baseline(prob, np.ones(prob.n_v, np.float32), rt, cpu_threads(args))
    print(json.dumps(dict(cpu_baseline=cpu, workload=f"shell {prob.n_v} vertices / {prob.n_e} tets")),
          flush=True)


def main():
    args = parse()
    if args.cpu_only:
        cpu_only(args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (the solve of one mesh runs on "
              "one MI355X). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import gbp_inputs as gi
    from paper_2308_08410_amd import binding as B
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t = time.time()
    prob = gi.shell_problem(args.nodes, seed=2, n_roots=5, n_leads=12)
    log(f"[bench] shell n_v={prob.n_v} n_e={prob.n_e} generated in {time.time() - t:.1f}s")
    st = make_state(prob, dev, torch, gi, B)
    tuned = None
    if args.no_tune:
        pass
    elif not args.tune:
        lanes, blocks, batch, lblocks, split = (int(x) for x in args.launch.split(",")[:5])
        B.set_launch(st["plan"], lanes, blocks, lblocks, batch)
        B.set_queue_split(st["plan"], split)
        d, w, o = args.hold.split(",")
        B.set_hold(st["plan"], float(d), int(w), int(o))
        log(f"[bench] launch {args.launch}, hold-back {args.hold}")
    else:
        from paper_2308_08410_amd import autotune
        t = time.time()
        tuned = autotune.tune(st["plan"], st["D"], st["vs"], st["rn"], st["rt"], use_cache=False, save=False)
        log(f"[bench] autotuned launch: lanes={tuned['lanes']} sweep_blocks={tuned['sweep_blocks']} "
            f"sync_batch={tuned['sync_batch']} level_blocks={tuned['level_blocks']} split={tuned['split']} "
            f"hold=({tuned['hold_delta']:.3g} ms, window {tuned['hold_window']}, open below "
            f"{tuned['hold_open']}) ({time.time() - t:.1f}s)")
    if args.calibrate_copy > 0:
        n = int(args.calibrate_copy * (1 << 20)) // 4
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        del x, y
    for w in range(args.warmup):
        loss, stats = gbp_step(st, B)
    torch.cuda.synchronize()
    log(f"[bench] warmup done: loss={float(loss[0]):.4g} rounds={stats['rounds']}")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record()
    face_solves = 0
    for k in range(args.steps):
        loss, stats = gbp_step(st, B)
        face_solves += stats["face_solves"]
    e1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_sync = e0.elapsed_time(e1) / args.steps
    wall_sync = 1e3 * t_wall / args.steps
    log(f"[bench] synchronous calls, timed {args.steps} steps: {ms_sync:.3f} ms/step (wall {wall_sync:.3f}) "
        f"loss={float(loss[0]):.4g}")
    # the same iterations through the enqueue-only calls (budgets from the last
    # synchronous solve); reported when every timed step met its budgets
    bud = enqueue_budgets(st, B)
    enqueue_step(st, B, bud)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record()
    ok = 0
    for k in range(args.steps):
        loss, good = enqueue_step(st, B, bud)
        ok += int(good)
    e1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_enq = e0.elapsed_time(e1) / args.steps
    wall_enq = 1e3 * t_wall / args.steps
    enqueue = ok == args.steps
    log(f"[bench] enqueue-only calls (budgets {bud['round_budget']} rounds, {bud['level_budget']} levels, "
        f"{bud['gs_budget']} sweeps), timed {args.steps} steps: {ms_enq:.3f} ms/step (wall {wall_enq:.3f}), "
        f"{ok}/{args.steps} within budgets")
    ms = ms_enq if enqueue else ms_sync
    # the forward alone at the same parameters: synchronous call, and enqueue-only
    # with the iteration's round budget (status checked after each)
    nf = 10
    e0.record()
    for _ in range(nf):
        B.eikonal_forward(st["plan"], st["D"], st["vs"], st["rn"], st["rt"])
    e1.record()
    torch.cuda.synchronize()
    fwd_sync = e0.elapsed_time(e1) / nf
    fwd_ok = 0
    e0.record()
    for _ in range(nf):
        B.eikonal_forward_async(st["plan"], st["D"], st["vs"], st["rn"], st["rt"], bud["round_budget"])
        fs_ = B.plan_status(st["plan"])
        fwd_ok += int(fs_["err"] == 0 and fs_["forward_converged"])
    e1.record()
    torch.cuda.synchronize()
    fwd_enq = e0.elapsed_time(e1) / nf
    log(f"[bench] forward alone: {fwd_sync:.3f} ms synchronous, {fwd_enq:.3f} ms enqueue-only "
        f"({fwd_ok}/{nf} within {bud['round_budget']} rounds)")
    log(f"[bench] timed {args.steps} steps: {ms:.3f} ms/step ({'enqueue-only' if enqueue else 'synchronous'} "
        f"calls) loss={float(loss[0]):.4g}")

    roofline = None
    hd, hw, ho = B.get_hold(st["plan"])
    detail = dict(launch=dict(B.get_launch(st["plan"]), split=int(B.get_queue_split(st["plan"])),
                              hold_delta_ms=hd, hold_window=hw, hold_open_below=ho),
                  fim_rounds=stats["rounds"],
                  face_solves_per_step=face_solves // args.steps,
                  node_updates=stats["node_updates"],
                  wall_ms_per_step=wall_enq if enqueue else wall_sync,
                  calls="enqueue-only" if enqueue else "synchronous",
                  synchronous_calls=dict(ms_per_step=ms_sync, iters_per_s=1000.0 / ms_sync, wall_ms_per_step=wall_sync),
                  enqueue_only_calls=dict(ms_per_step=ms_enq, iters_per_s=1000.0 / ms_enq, wall_ms_per_step=wall_enq,
                                          steps_within_budgets=ok, **bud),
                  forward_alone=dict(synchronous_ms=fwd_sync, enqueue_only_ms=fwd_enq,
                                     enqueue_only_within_budget=fwd_ok, solves=nf))
    if not args.no_profile:
        # per-kernel HIP-event timing on the launching stream, separate steps
        B.profile_reset()
        B.profile_enable(True)
        nprof = 3
        fs = 0
        for k in range(nprof):
            if enqueue:
                enqueue_step(st, B, bud)
                fs += B.forward_work(st["plan"])["face_solves"]
            else:
                _, s2 = gbp_step(st, B)
                fs += s2["face_solves"]
        torch.cuda.synchronize()
        prof = B.profile_read()
        B.profile_enable(False)
        n_sw, ms_sw = prof["fim_sweep"]
        avg_ms = ms_sw / max(n_sw, 1)
        faces_per_launch = fs / max(n_sw, 1)
        bpl = bytes_per_local_problem(prob.n_v, prob.n_e)
        # The relaxation round is bound by its gathers (memory), not by its arithmetic:
        # report it against HBM bandwidth with the algorithmic bytes per launch (the
        # full-sweep bytes times the fraction of the sweep's local problems the launch
        # evaluates), and keep the arithmetic rate beside it.
        alg = faces_per_launch * bpl
        achieved = alg / (avg_ms * 1e-3) / 1e9
        tflops = faces_per_launch * FLOP_PER_FACE / (avg_ms * 1e-3) / 1e12
        traffic = stored_traffic("k_sweep")
        roofline = dict(kernel="k_sweep (eikonal relaxation round)", bound="hbm", achieved=achieved,
                        peak=PEAK_HBM_GBS, unit="GB/s", frac=achieved / PEAK_HBM_GBS, traffic=traffic,
                        algorithmic_bytes_per_launch=alg, bytes_per_local_problem=bpl,
                        full_sweep_bytes=sweep_bytes(prob.n_v, prob.n_e),
                        local_problems_per_launch=faces_per_launch,
                        gathered_bytes_per_launch=faces_per_launch * GATHERED_BYTES_PER_FACE,
                        traffic_over_algorithmic=None if traffic is None else traffic / alg,
                        avg_launch_ms=avg_ms, launches_per_step=n_sw / nprof,
                        alu_tflops=tflops, alu_frac=tflops / PEAK_FP32_TFLOPS)
        # the whole backward (parent recompute, child lists, level walk, gradients)
        # against its algorithmic bytes; the level launches are latency-bound
        bwd_fams = ("parent", "child_lists", "adj_level", "grad")
        bwd_ms = sum(prof[f][1] for f in bwd_fams if f in prof) / nprof
        ab = adjoint_bytes(prob.n_v, prob.n_e)
        n_lv, ms_lv = prof["adj_level"]
        lv_ms = ms_lv / max(n_lv, 1)
        lv_bytes = stored_traffic("k_adj_level")
        detail["adjoint"] = dict(
            kernels="+".join(bwd_fams), ms_per_step=bwd_ms, algorithmic_bytes=ab,
            achieved_GBps=ab / (bwd_ms * 1e-3) / 1e9, frac=ab / (bwd_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
            level_kernel="k_adj_level", level_avg_launch_ms=lv_ms, level_launches_per_step=n_lv / nprof,
            level_traffic_per_launch=lv_bytes,
            level_traffic_per_backward=None if lv_bytes is None else lv_bytes * n_lv / nprof)
        # ECG contraction on the matrix cores: executed bf16 MFMA flops (counters)
        # over the launch time measured here
        for fam, kern in (("ecg_fwd", "k_ecg_fwd"), ("ecg_bwd", "k_ecg_bwd")):
            n_k, ms_k = prof[fam]
            m = stored_mfma(kern)
            if m and n_k:
                avg = ms_k / n_k
                tf = m["mfma_flops_per_launch"] / (avg * 1e-3) / 1e12
                detail[kern] = dict(avg_launch_ms=avg, mfma_flops_per_launch=m["mfma_flops_per_launch"],
                                    mfma_tflops=tf, peak_tflops=PEAK_BF16_TFLOPS, frac=tf / PEAK_BF16_TFLOPS,
                                    mfma_busy_pct=m["mfma_busy_pct"])
                # the template's exp2/rcp on the VALU: transcendental operations
                # (counters) over the launch time measured here, against the
                # quarter-rate peak
                v = stored_valu(kern)
                if v:
                    rate = v["trans_ops_per_launch"] / (avg * 1e-3)
                    detail[kern].update(valu_insts_per_launch=v["valu_insts_per_launch"],
                                        trans_ops_per_launch=v["trans_ops_per_launch"],
                                        trans_ops_per_s=rate, trans_frac=rate / v["trans_peak_ops_per_s"],
                                        valu_busy_pct=v["valu_busy_pct"])
        detail["kernel_ms_per_step"] = {k: v[1] / nprof for k, v in prof.items() if v[0]}
        detail["kernel_launches_per_step"] = {k: v[0] / nprof for k, v in prof.items() if v[0]}
    forms = set() if args.no_forms else {f for f in args.forms.split(",") if f}
    unknown = forms - set(FORMS)
    if unknown:
        print(f"unknown forms {sorted(unknown)}; choose from {','.join(FORMS)}", file=sys.stderr)
        sys.exit(2)
    from paper_2308_08410_amd import autotune
    if "warm" in forms:
        for ordered in (False, True):
            t = time.time()
            ws = warm_single_form(st, prob, args.form_steps, torch, B, autotune, ordered=ordered)
            ws["speedup_vs_plain"] = ws["iters_per_s"] / (1000.0 / ms)
            name = "ordered" if ordered else "two-sided"
            detail["warm_ordered_single_500k" if ordered else "warm_single_500k"] = ws
            log(f"[bench] warm single form ({name}): {ws['iters_per_s']:.1f} iter/s (x{ws['speedup_vs_plain']:.2f}), "
                f"{ws['local_problems_per_step'] / 1e6:.1f}M local problems, "
                f"max rel T vs cold {ws['max_rel_T_vs_cold']:.1e} ({time.time() - t:.1f}s)")
    if "points" in forms:
        t = time.time()
        pf = point_root_form(st, prob, args.form_steps, torch, gi, B)
        pf["speedup_vs_plain"] = pf["iters_per_s"] / (1000.0 / ms)
        detail["point_roots_500k"] = pf
        log(f"[bench] point-root form ({pf['points']} points): {pf['iters_per_s']:.1f} iter/s "
            f"(x{pf['speedup_vs_plain']:.2f}), {pf['rounds']} rounds ({time.time() - t:.1f}s)")
    if "leadfield" in forms:
        lf = lead_field_form(st, prob, torch, B)
        detail["lead_field_500k"] = lf
        log(f"[bench] lead weights on the device: {lf['ms']:.2f} ms for {lf['n_leads']} leads, "
            f"max rel dev from the host assembly {lf['rel_max_vs_host']:.1e}")
    if "fista" in forms:
        t = time.time()
        fs = fista_form(st, torch, B)
        detail["fista_500k"] = fs
        log("[bench] FISTA local solver: " + ", ".join(
            (f"n_f={x['n_f']}" if "n_f" in x else f"tau={x['tau_ms']:g} ms")
            + f": {x['forward_ms']:.1f} ms (x{x['slowdown_vs_exact']:.1f}), dev {x['rel_max_vs_exact']:.1e}"
            for x in fs["runs"]) + f"; exact {fs['exact_forward_ms']:.2f} ms ({time.time() - t:.1f}s)")
    if "slice" in forms:
        t = time.time()
        sl = slice_form(dev, args.form_steps, torch, gi, B)
        detail["slice_2d"] = sl
        log("[bench] 2-D slice (triangles): " + ", ".join(
            f"{x['n_v']} nodes {x['iters_per_s']:.1f} iter/s" for x in sl) + f" ({time.time() - t:.1f}s)")
    if "batched" in forms:
        t = time.time()
        bw = batched_form(dev, args.form_steps, torch, gi, B, autotune)
        for k in ("cold", "warm", "warm_ordered"):
            f = bw[k]
            f["speedup_vs_plain_vertex_iters"] = f["vertex_iters_per_s"] / (prob.n_v * 1000.0 / ms)
            log(f"[bench] batched form ({k}): {bw['instances']} instances / {bw['total_vertices']} vertices, "
                f"{f['instance_iters_per_s']:.1f} instance-iter/s, x{f['speedup_vs_plain_vertex_iters']:.2f} "
                f"vertex-iter/s vs plain, {f['local_problems_per_step'] / 1e6:.0f}M local problems, "
                f"max rel T vs cold {f['max_rel_T_vs_cold']:.1e}, "
                f"within budgets {f['converged']}")
        detail["batched"] = bw
        log(f"[bench] batched forms done ({time.time() - t:.1f}s)")
    if "learned" in forms:
        t = time.time()
        lf = learned_form(st, prob, torch, B)
        detail["learned_warm_start_500k"] = lf
        log(f"[bench] learned warm start ({lf['train_solves']} solves, {lf['train_steps']} steps, "
            f"{lf['train_seconds']:.1f}s training): guess error {lf['guess_rel_l2']['mlp']:.3f} (geometric "
            f"{lf['guess_rel_l2']['geo']:.3f}); warm {lf['ms']['warm_mlp_incl_prediction']:.2f} ms vs cold "
            f"{lf['ms']['cold']:.2f} ms, local problems x{lf['local_problems']['warm_mlp'] / lf['local_problems']['cold']:.2f}, "
            f"rounds {lf['rounds']['warm_mlp']:.0f} vs {lf['rounds']['cold']:.0f}; ordered "
            f"{lf['ms']['warm_mlp_ordered_incl_prediction']:.2f} ms, local problems "
            f"x{lf['local_problems']['warm_mlp_ordered'] / lf['local_problems']['cold']:.2f} ({time.time() - t:.1f}s)")
    if "inverse" in forms:
        t = time.time()
        inv = inverse_form(dev, torch, gi, B)
        detail["inverse_multistart_1m"] = inv
        log(f"[bench] inverse problem, {inv['starts']} starts x {inv['nodes']} vertices: "
            f"{inv['iters_per_s']:.2f} iter/s ({inv['start_iters_per_s']:.1f} start-iter/s), misfit "
            f"{np.mean(inv['loss_after_2']):.3g} -> {np.mean(inv['loss_after_last']):.3g} over {inv['iters']} "
            f"iterations, within budgets {inv['converged']} (setup {inv['setup_s']:.1f}s, {time.time() - t:.1f}s)")
    cpu = None
    if not args.no_cpu_baseline:
        t = time.time()
        cpu = cpu_baseline(prob, st["vs_start"], st["rt_start"], cpu_threads(args))
        log(f"[bench] cpu baseline {time.time() - t:.1f}s: {cpu['value']:.4g} iter/s on {cpu['cores']} threads")
    out = {
        "metric": METRIC, "value": 1000.0 / ms, "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"biventricular shell {prob.n_v} vertices / {prob.n_e} tets, helix fibres, "
                               f"D=diag(0.36,0.09,0.09), 5 endocardial roots, 12 leads x 500 steps; "
                               f"cold eikonal + ECG + loss + ECG bwd + adjoint + Adam",
                   "n_v": prob.n_v, "n_e": prob.n_e, "leads": 12, "time_steps": 500, "roots": 5,
                   "parallelism": "single GPU", "calls": detail["calls"]},
        "roofline": roofline, "cpu_baseline": cpu, "detail": detail,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

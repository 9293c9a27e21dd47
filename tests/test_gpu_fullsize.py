"""GPU parity at the benchmark's sizes, in the benchmark's launch configuration.

* 64k-vertex shell (same generator and root perturbation as the benchmark; its
  anisotropic parent graph contains cycles): the oracle solves it here.
* 500k-vertex shell, the benchmark workload itself: the oracle's activation times
  were written once by tests/golden/make_shell500k_reference.py (oracle only);
  the GPU forward is compared with them element by element, and the ECG and
  adjoint run on both sides on those stored times.

The oracle only ever sees seeded inputs and its own results."""
import os
import sys

import numpy as np
import pytest

import oracle as O
from test_gpu_parity import B, _dev, i32, rel_l2, rel_max, t32

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
from make_shell500k_reference import OUT as REF_PATH, bench_like, input_hash  # noqa: E402

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


class Big:
    def __init__(self, n, T_ref=None):
        dev = _dev()
        self.p, self.rt, self.vs = bench_like(n)
        p = self.p
        print(f"[case] bench-like shell n_v={p.n_v} n_e={p.n_e}", flush=True)
        self.dev = dev
        self.plan = B().Plan(p.xyz, p.tets)
        self.D, self.W = t32(p.D, dev), t32(p.W, dev)
        self.rn, self.rtt, self.vst = i32(p.root_node, dev), t32(self.rt, dev), t32(self.vs, dev)
        self.T, self.stats = B().eikonal_forward(self.plan, self.D, self.vst, self.rn, self.rtt)
        torch.cuda.synchronize()
        self.Tg = self.T.cpu().numpy()
        if T_ref is None:
            T_ref, _ = O.solve(p.xyz, p.tets, p.D, self.vs, p.root_node, self.rt)
        self.T_ref = np.asarray(T_ref, np.float32)
        self.T_ref_dev = t32(self.T_ref, dev)
        a = p.ap
        self.ap = B().make_ap(a["K0"], a["K1"], a["tau"], a["t0"], a["dt"], a["n_steps"])

    def ecg_and_backward(self):
        p = self.p
        T64 = self.T_ref.astype(np.float64)
        ecg = B().ecg_forward(self.T_ref_dev, self.W, self.ap)
        eo = O.ecg_forward(T64, p.W, p.ap)
        assert np.abs(ecg.cpu().numpy() - eo).max() / np.abs(eo).max() <= 1e-3
        eg = B().ecg_forward(self.T, self.W, self.ap).cpu().numpy()     # GPU's own times
        assert np.abs(eg - eo).max() / np.abs(eo).max() <= 1e-3
        _, Go = O.ecg_loss(eo, 0.8 * eo)
        go = O.ecg_backward(T64, p.W, p.ap, Go)
        gT = B().ecg_backward(self.T_ref_dev, self.W, self.ap, t32(Go, self.dev))
        assert rel_l2(gT.cpu().numpy(), go) <= 1e-3
        dD, dvs, drt = B().eikonal_backward(self.plan, self.D, self.vst, self.rn, self.rtt,
                                            self.T_ref_dev, t32(go, self.dev))
        info = B().backward_info(self.plan)
        res = O.adjoint(p.xyz, p.tets, p.D, self.vs, p.root_node, self.rt, T64, go)
        got = dict(vscale=dvs.cpu().numpy(), root_t=drt.cpu().numpy(), D=dD.cpu().numpy())
        ref = dict(vscale=res["dvscale"], root_t=res["droot_t"], D=res["dD"])
        errs = {k: rel_l2(got[k], ref[k]) for k in got}
        # element by element, relative to the block's largest entry
        emax = {k: float(np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max()) for k in got}
        print(f"[backward] {info} rel L2 errors {errs}, max-norm errors {emax}", flush=True)
        for k in got:
            assert errs[k] <= 1e-3, (k, errs[k])
            assert emax[k] <= 1e-3, (k, emax[k])
        return info


@pytest.fixture(scope="module")
def medium():
    return Big(62_500)


@pytest.fixture(scope="module")
def full():
    if not os.path.exists(REF_PATH):
        pytest.fail(f"missing {REF_PATH}: run tests/golden/make_shell500k_reference.py")
    ref = np.load(REF_PATH)
    big = Big(500_000, T_ref=ref["T"])
    if str(ref["input_sha256"]) != input_hash(big.p, big.rt, big.vs):
        pytest.fail("stored reference does not match the generated inputs: rerun the script")
    return big


def test_medium_forward_parity(medium):
    assert medium.stats["converged"]
    assert rel_max(medium.Tg, medium.T_ref) <= 1e-4


def test_medium_ecg_and_backward_with_cycles(medium):
    medium.ecg_and_backward()


def test_full_forward_parity(full):
    assert full.stats["converged"] and full.stats["unreached"] == 0
    err = rel_max(full.Tg, full.T_ref)
    print(f"[forward 500k] rel max err {err:.3e} rounds {full.stats['rounds']}", flush=True)
    assert err <= 1e-4


def test_full_ecg_and_gradients(full):
    full.ecg_and_backward()


@pytest.mark.parametrize("split", [True, False])
def test_full_forward_with_push_overflow(full, split):
    """A 64-block grid makes every block's LDS push buffer overflow in the first
    rounds of a two-sided warm solve (all 500k vertices queued, ~7.8k per
    block): the overflow path of both queue layouts must keep every vertex it
    queues, so the warm solve (from a perturbed guess) and the cold solve both
    reach the stored oracle times."""
    plan = full.plan
    saved = B().get_launch(plan)
    saved_split = B().get_queue_split(plan)
    B().set_launch(plan, 16, 64, saved["level_blocks"], 16)
    B().set_queue_split(plan, split)
    try:
        r = np.random.Generator(np.random.PCG64(11))
        guess = t32(full.T_ref * (1.0 + 0.02 * r.uniform(-1.0, 1.0, size=len(full.T_ref))), full.dev)
        print(f"[overflow] split={split} warm", flush=True)
        T, st = B().eikonal_forward(plan, full.D, full.vst, full.rn, full.rtt, T_init=guess)
        assert st["converged"]
        assert rel_max(T.cpu().numpy(), full.T_ref) <= 1e-4
        print(f"[overflow] split={split} cold", flush=True)
        T, st = B().eikonal_forward(plan, full.D, full.vst, full.rn, full.rtt)
        assert st["converged"]
        assert rel_max(T.cpu().numpy(), full.T_ref) <= 1e-4
    finally:
        B().set_launch(plan, saved["lanes"], saved["sweep_blocks"], saved["level_blocks"], saved["sync_batch"])
        B().set_queue_split(plan, saved_split)


@pytest.mark.parametrize("launch", [(16, 1024), (8, 2048)])
def test_full_forward_with_fista(full, launch):
    """The forward with FISTA local solves (Alg. 1, 128 iterations, tightened
    step constant) at 500k reaches the stored oracle times within 1e-4 and
    never falls below them by more than the FP32 solve's own error (FISTA
    values are feasible points of each local problem), in the default launch
    (16 lanes per vertex, two local problems per lane) and in the one the
    benchmark's FISTA figures use (8 lanes, three per lane, 2048 blocks)."""
    plan = full.plan
    lanes, blocks = launch
    saved = B().get_launch(plan)
    B().set_local_solver(plan, "fista", 128, "tight")
    B().set_launch(plan, lanes, blocks, saved["level_blocks"], saved["sync_batch"])
    try:
        T, st = B().eikonal_forward(plan, full.D, full.vst, full.rn, full.rtt)
    finally:
        B().set_local_solver(plan, "exact")
        B().set_launch(plan, saved["lanes"], saved["sweep_blocks"], saved["level_blocks"], saved["sync_batch"])
    assert st["converged"]
    Tg = T.cpu().numpy().astype(np.float64)
    err = rel_max(Tg, full.T_ref)
    print(f"[fista 500k] lanes {lanes} blocks {blocks}: rel max err {err:.3e} rounds {st['rounds']}",
          flush=True)
    assert err <= 1e-4
    assert np.all(Tg >= full.T_ref * (1 - 1e-5) - 1e-6)


@pytest.mark.parametrize("launch", [(16, 768, 16, 2048, True, (2.5, 0, 16384)),
                                    (16, 1024, 32, 2048, True, (4.0, 0, 32768)),
                                    (8, 512, 16, 512, False, (0.0, 0, 0)),
                                    (32, 2048, 64, 1024, True, (1.0, 2, 1 << 30))])
def test_full_forward_and_gradients_in_launch_configs(full, launch):
    """The 500k forward against the stored oracle times, and the gradients against
    those of the default configuration, in the benchmark's launch configuration
    (first: the one bench.py times, hold-back included) and others from the
    autotuner's search space."""
    lanes, blocks, batch, lblocks, split, hold = launch
    plan = full.plan
    saved = B().get_launch(plan)
    saved_split = B().get_queue_split(plan)
    saved_hold = B().get_hold(plan)
    g = t32(np.random.Generator(np.random.PCG64(12)).normal(size=full.p.n_v), full.dev)
    ref = B().eikonal_backward(plan, full.D, full.vst, full.rn, full.rtt, full.T_ref_dev, g)
    B().set_launch(plan, lanes, blocks, lblocks, batch)
    B().set_queue_split(plan, split)
    B().set_hold(plan, *hold)
    try:
        print(f"[case] 500k launch {launch}", flush=True)
        T, st = B().eikonal_forward(plan, full.D, full.vst, full.rn, full.rtt)
        assert st["converged"]
        assert rel_max(T.cpu().numpy(), full.T_ref) <= 1e-4
        got = B().eikonal_backward(plan, full.D, full.vst, full.rn, full.rtt, full.T_ref_dev, g)
        for a, b in zip(got, ref):
            assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) <= 1e-5
    finally:
        B().set_launch(plan, saved["lanes"], saved["sweep_blocks"], saved["level_blocks"], saved["sync_batch"])
        B().set_queue_split(plan, saved_split)
        B().set_hold(plan, *saved_hold)

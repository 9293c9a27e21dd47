"""torch.autograd wrappers: one Geodesic-BP iteration through autograd gives the
same gradients as the FP64 oracle chain (loss -> ECG backward -> adjoint) on the
same seeded inputs, and the same as calling the C ABI step by step."""
import numpy as np
import pytest

import gbp_inputs as gi
import oracle as O
from test_gpu_parity import B, _dev, i32, rel_l2, t32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_autograd_iteration_matches_oracle_chain():
    dev = _dev()
    from paper_2308_08410_amd import autograd as A
    p = gi.shell_problem(12_000, seed=11, n_roots=4, vscale_range=(0.6, 1.4))
    r = np.random.Generator(np.random.PCG64(4))
    plan = B().Plan(p.xyz, p.tets)
    a = p.ap
    ap = B().make_ap(a["K0"], a["K1"], a["tau"], a["t0"], a["dt"], a["n_steps"])
    D = t32(p.D, dev).requires_grad_(True)
    vs = t32(p.vscale, dev).requires_grad_(True)
    rt = t32(p.root_t, dev).requires_grad_(True)
    rn = i32(p.root_node, dev)
    W = t32(p.W, dev)
    # target from the oracle's ECG of perturbed onsets (oracle only)
    To_tgt, _ = O.solve(p.xyz, p.tets, p.D, p.vscale, p.root_node, p.root_t + r.uniform(-3, 3, 4))
    target = t32(O.ecg_forward(To_tgt, p.W, a), dev)

    T = A.eikonal(plan, D, vs, rn, rt)
    loss = A.ecg_loss(A.ecg(T, W, ap), target)
    loss.backward()

    # oracle chain on its own activation times
    To, _ = O.solve(p.xyz, p.tets, p.D, p.vscale, p.root_node, p.root_t)
    eo = O.ecg_forward(To, p.W, a)
    lo, Go = O.ecg_loss(eo, target.cpu().numpy())
    go = O.ecg_backward(To, p.W, a, Go)
    res = O.adjoint(p.xyz, p.tets, p.D, p.vscale, p.root_node, p.root_t, To, go)
    assert float(loss.detach()) == pytest.approx(lo, rel=1e-3)
    assert rel_l2(vs.grad.cpu().numpy(), res["dvscale"]) <= 1e-3
    assert rel_l2(rt.grad.cpu().numpy(), res["droot_t"]) <= 1e-3
    assert rel_l2(D.grad.cpu().numpy(), res["dD"]) <= 1e-3


def test_autograd_equals_direct_abi_calls():
    dev = _dev()
    from paper_2308_08410_amd import autograd as A
    p = gi.cube_problem(10, jitter=0.1)
    plan = B().Plan(p.xyz, p.tets)
    a = p.ap
    ap = B().make_ap(a["K0"], a["K1"], a["tau"], a["t0"], a["dt"], a["n_steps"])
    D, vs, rt = t32(p.D, dev), t32(p.vscale, dev), t32(p.root_t, dev)
    rn, W = i32(p.root_node, dev), t32(p.W, dev)
    target = torch.zeros((a["n_steps"], W.shape[1]), device=dev)
    vs_g = vs.clone().requires_grad_(True)
    T = A.eikonal(plan, D, vs_g, rn, rt)
    A.ecg_loss(A.ecg(T, W, ap), target).backward()
    T2, _ = B().eikonal_forward(plan, D, vs, rn, rt)
    e2 = B().ecg_forward(T2, W, ap)
    _, G = B().ecg_loss(e2, target)
    gT = B().ecg_backward(T2, W, ap, G)
    _, dvs, _ = B().eikonal_backward(plan, D, vs, rn, rt, T2, gT)
    assert torch.allclose(vs_g.grad, dvs, rtol=1e-4, atol=1e-6 * float(dvs.abs().max()))

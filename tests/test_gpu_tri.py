"""Triangle meshes (d = 2; the paper's 2-D study, Sec. 3.1) on the GPU against the
triangle oracle (`oracle/tri.py`): activation times on the 2-D left-ventricular
slice and on a jittered anisotropic square, an exact plane wave, the ECG of the
slice, gradients at the oracle's times, and input errors.  Bars as for
tetrahedra: times 1e-4 relative (max norm), ECG 1e-3, gradients 1e-3 relative
L2 per block."""
import numpy as np
import pytest

import gbp_inputs as gi
import oracle as O
from oracle import tri as O2
from conftest import random_spd, rng
from test_gpu_parity import B, _dev, i32, rel_l2, rel_max, t32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slice_case():
    dev = _dev()
    p = gi.annulus_problem(vscale_range=(0.7, 1.3))
    print(f"[case] slice n_v={p.n_v} n_t={p.n_e}", flush=True)
    plan = B().TriPlan(p.xyz, p.tets)
    d = dict(p=p, plan=plan, D=t32(p.D, dev), vs=t32(p.vscale, dev), rn=i32(p.root_node, dev),
             rt=t32(p.root_t, dev), dev=dev)
    d["T"], d["st"] = B().tri_forward(plan, d["D"], d["vs"], d["rn"], d["rt"])
    torch.cuda.synchronize()
    d["To"], _ = O2.solve2(p.xyz, p.tets, p.D, p.vscale, p.root_node, p.root_t)
    return d


def test_slice_forward_matches_oracle(slice_case):
    c = slice_case
    assert c["st"]["converged"] and c["st"]["unreached"] == 0
    assert rel_max(c["T"].cpu().numpy(), c["To"]) <= 1e-4


def test_slice_ecg(slice_case):
    c, p = slice_case, slice_case["p"]
    a = p.ap
    ap = B().make_ap(a["K0"], a["K1"], a["tau"], a["t0"], a["dt"], a["n_steps"])
    ecg = B().ecg_forward(c["T"], t32(p.W, c["dev"]), ap).cpu().numpy()
    eo = O.ecg_forward(c["To"], p.W, p.ap)
    assert np.abs(ecg - eo).max() <= 1e-3 * np.abs(eo).max()


def test_slice_gradients_match_oracle(slice_case):
    c, p = slice_case, slice_case["p"]
    g = np.random.Generator(np.random.PCG64(2)).normal(size=p.n_v)
    T_in = c["To"].astype(np.float32)
    dD, dvs, drt = B().tri_backward(c["plan"], c["D"], c["vs"], c["rn"], c["rt"], t32(T_in, c["dev"]),
                                    t32(g, c["dev"]))
    ref = O2.adjoint2(p.xyz, p.tets, p.D, p.vscale, p.root_node, p.root_t, T_in.astype(np.float64), g)
    info = B().tri_backward_info(c["plan"])
    print(f"[walk] slice: {info}", flush=True)
    # the level walk finishes the adjoint (sweeps only on what cycles leave)
    assert info["levels"] > 10 and info["cyclic"] <= p.n_v // 10
    assert (info["sweeps"] == 0) == (info["cyclic"] == 0)
    assert rel_l2(dD.cpu().numpy(), ref["dD"]) <= 1e-3
    assert rel_l2(dvs.cpu().numpy(), ref["dvscale"]) <= 1e-3
    assert rel_l2(drt.cpu().numpy(), ref["droot_t"]) <= 1e-3
    # the shift identity holds for the GPU's own gradients too
    assert float(drt.sum()) == pytest.approx(float(g.sum()), rel=1e-4, abs=1e-3)


@pytest.mark.parametrize("seed", range(2))
def test_square_anisotropic_matches_oracle(seed):
    dev = _dev()
    r = rng(seed)
    xy, tris = gi.square_tri(100)
    x = gi.jitter_nodes2(xy, 0.01, 0.15, seed)
    D3 = np.stack([O2.pack2(random_spd(r, 2, 6.0)) for _ in range(len(tris))]).astype(np.float32)
    vs = r.uniform(0.6, 1.4, size=len(x)).astype(np.float32)
    rn = r.choice(len(x), size=4, replace=False).astype(np.int32)
    rt = r.uniform(0, 0.3, size=4).astype(np.float32)
    plan = B().TriPlan(x, tris)
    T, st = B().tri_forward(plan, t32(D3, dev), t32(vs, dev), i32(rn, dev), t32(rt, dev))
    To, _ = O2.solve2(x, tris, D3, vs, rn, rt)
    assert st["converged"]
    assert rel_max(T.cpu().numpy(), To) <= 1e-4
    g = r.normal(size=len(x))
    T_in = To.astype(np.float32)
    dD, dvs, drt = B().tri_backward(plan, t32(D3, dev), t32(vs, dev), i32(rn, dev), t32(rt, dev),
                                    t32(T_in, dev), t32(g, dev))
    ref = O2.adjoint2(x, tris, D3, vs, rn, rt, T_in.astype(np.float64), g)
    info = B().tri_backward_info(plan)
    print(f"[walk] anisotropic square seed {seed}: {info}", flush=True)
    assert info["levels"] > 10 and (info["sweeps"] == 0) == (info["cyclic"] == 0)
    assert rel_l2(dD.cpu().numpy(), ref["dD"]) <= 1e-3
    assert rel_l2(dvs.cpu().numpy(), ref["dvscale"]) <= 1e-3
    assert rel_l2(drt.cpu().numpy(), ref["droot_t"]) <= 1e-3


def test_plane_wave_exact_on_gpu():
    dev = _dev()
    r = rng(3)
    xy, tris = gi.square_tri(20)
    x = xy.astype(np.float64)
    Dm = random_spd(r, 2, 8.0)
    u = r.normal(size=2)
    p = u / np.sqrt(u @ Dm @ u)
    vel = Dm @ p
    Tex = 0.3 + x @ p
    roots = np.array([i for i, xi in enumerate(x) if any((xi[d] == 0.0 and vel[d] >= 0) or
                                                          (xi[d] == 1.0 and vel[d] <= 0) for d in range(2))],
                     dtype=np.int32)
    plan = B().TriPlan(xy, tris)
    D3 = np.tile(O2.pack2(Dm), (len(tris), 1)).astype(np.float32)
    T, st = B().tri_forward(plan, t32(D3, dev), None, i32(roots, dev), t32(Tex[roots], dev))
    assert st["converged"]
    assert np.abs(T.cpu().numpy() - Tex).max() <= 1e-5 * np.abs(Tex).max()


def test_tri_input_errors():
    dev = _dev()
    xy, tris = gi.square_tri(2)
    bad = tris.copy()
    bad[0, 0] = len(xy)
    with pytest.raises(B().GbpError):
        B().TriPlan(xy, bad)
    deg = tris.copy()
    deg[0, 1] = deg[0, 0]
    with pytest.raises(B().GbpError):
        B().TriPlan(xy, deg)
    plan = B().TriPlan(xy, tris)
    D3 = t32(np.tile([1.0, 1.0, 0.0], (len(tris), 1)), dev)
    with pytest.raises(B().GbpError):   # root id out of range
        B().tri_forward(plan, D3, None, i32([len(xy)], dev), t32([0.0], dev))
    with pytest.raises(B().GbpError):   # not positive definite
        B().tri_forward(plan, t32(np.tile([1.0, 1.0, 2.0], (len(tris), 1)), dev), None, i32([0], dev),
                        t32([0.0], dev))
    T, st = B().tri_forward(plan, D3, None, i32([0], dev), t32([0.0], dev))
    assert st["converged"] and float(T[0]) == 0.0


def test_slice_through_autograd(slice_case):
    """A full 2-D iteration through torch autograd (TriEikonalFn + ECG + loss)
    gives the explicit C ABI chain's gradients."""
    from paper_2308_08410_amd import autograd as A
    c, p = slice_case, slice_case["p"]
    a = p.ap
    ap = B().make_ap(a["K0"], a["K1"], a["tau"], a["t0"], a["dt"], a["n_steps"])
    W = t32(p.W, c["dev"])
    target = B().ecg_forward(c["T"], W, ap).clone() * 0.9
    vs = c["vs"].clone().requires_grad_(True)
    rt = c["rt"].clone().requires_grad_(True)
    D = c["D"].clone().requires_grad_(True)
    T = A.tri_eikonal(c["plan"], D, vs, c["rn"], rt)
    loss = A.ecg_loss(A.ecg(T, W, ap), target)
    loss.backward()
    T2, _ = B().tri_forward(c["plan"], c["D"], c["vs"], c["rn"], c["rt"])
    ecg = B().ecg_forward(T2, W, ap)
    _, G = B().ecg_loss(ecg, target)
    gT = B().ecg_backward(T2, W, ap, G)
    dD, dvs, drt = B().tri_backward(c["plan"], c["D"], c["vs"], c["rn"], c["rt"], T2, gT)
    for x, y in ((D.grad, dD), (vs.grad, dvs), (rt.grad, drt)):
        assert rel_l2(x.cpu().numpy(), y.cpu().numpy()) <= 1e-5


def test_fine_slice_identities():
    """250k-vertex slice (the benchmark's finer 2-D case): every vertex reached,
    roots hold their onsets, and the GPU's own gradients satisfy the exact
    identities of the scheme at any size: sum_r dL/dt_r = sum_n g_n and
    sum_n s_n dL/ds_n - sum_r t_r dL/dt_r = -g.T."""
    dev = _dev()
    p = gi.annulus_problem(250_000, vscale_range=(0.7, 1.3))
    print(f"[case] fine slice n_v={p.n_v} n_t={p.n_e}", flush=True)
    plan = B().TriPlan(p.xyz, p.tets)
    D, vs, rn, rt = t32(p.D, dev), t32(p.vscale, dev), i32(p.root_node, dev), t32(p.root_t, dev)
    T, st = B().tri_forward(plan, D, vs, rn, rt)
    assert st["converged"] and st["unreached"] == 0
    Tn = T.cpu().numpy().astype(np.float64)
    assert np.all(Tn[p.root_node] <= p.root_t + 1e-6)
    g = np.random.Generator(np.random.PCG64(9)).uniform(0.5, 1.5, size=p.n_v)
    _, dvs, drt = B().tri_backward(plan, D, vs, rn, rt, T, t32(g, dev), want_D=False)
    drt = drt.cpu().numpy().astype(np.float64)
    dvs = dvs.cpu().numpy().astype(np.float64)
    assert drt.sum() == pytest.approx(g.sum(), rel=1e-4)
    lhs = p.vscale.astype(np.float64) @ dvs - p.root_t.astype(np.float64) @ drt
    assert lhs == pytest.approx(-(g @ Tn), rel=1e-3)

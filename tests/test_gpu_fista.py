"""The FISTA local solver (Alg. 1) on the GPU against the oracle's `fista_local`
and Lipschitz constants, the exact batch solve against the oracle's
`local_solve`, unreached face vertices, and the forward solve with FISTA
against the oracle's exact activation times.

Tolerances.  Local values are compared relative to the face's scale
sqrt(tr Q): FP32 against FP64 arithmetic of the same steps, 1e-5 for the exact
solve and 1e-4 for up to 100 FISTA iterations (rounding of each iterate
carries into the next).  Step constants: the bound of Eq. (lipschitz_est)
divides by the smallest eigenvalue of Q, which FP32 rounding of Q moves by up
to cond(Q) * 2^-24 relative, so 5e-3 for the random faces here (condition
numbers up to ~1e4); the tightened constant divides by the minimum of h
(well conditioned), 1e-3.  FISTA values are feasible points, so the forward's
times are never below the exact scheme's by more than the FP32 solve's own
error (1e-5 relative)."""
import numpy as np
import pytest

import gbp_inputs as gi
import oracle as O
from test_gpu_parity import B, _dev, i32, rel_max, t32
from test_oracle_local import random_face

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def faces():
    r = np.random.Generator(np.random.PCG64(1))
    n = 2000
    Q = np.stack([random_face(r) for _ in range(n)])
    Phi = r.uniform(-0.5, 0.5, size=(n, 3)) * np.sqrt(np.trace(Q, axis1=1, axis2=2) / 3)[:, None]
    Q6 = np.stack([Q[:, 0, 0], Q[:, 1, 1], Q[:, 2, 2], Q[:, 0, 1], Q[:, 0, 2], Q[:, 1, 2]], 1)
    return Q, Phi, Q6, np.sqrt(np.trace(Q, axis1=1, axis2=2))


def _obj(Q, Phi, a):
    return (a * Phi).sum(1) + np.sqrt(np.einsum("ni,nij,nj->n", a, Q, a))


def test_exact_batch_matches_oracle(faces):
    dev = _dev()
    Q, Phi, Q6, scale = faces
    v, a, _ = B().local_solve(t32(Q6, dev), t32(Phi, dev), "exact")
    vo = np.array([O.local_solve(Q[i], Phi[i])[0] for i in range(len(Q))])
    assert np.max(np.abs(v.cpu().numpy() - vo) / scale) <= 1e-5
    # the minimiser may differ at ties: check it is one (its objective is the minimum)
    a = a.cpu().numpy().astype(np.float64)
    assert a.min() >= -1e-6 and np.allclose(a.sum(1), 1.0, atol=1e-5)
    assert np.max(np.abs(_obj(Q, Phi, a) - vo) / scale) <= 1e-5


@pytest.mark.parametrize("mode,tol", [("bound", 5e-3), ("tight", 1e-3)])
def test_step_constants_match_oracle(faces, mode, tol):
    dev = _dev()
    Q, Phi, Q6, _ = faces
    f = O.lipschitz_bound if mode == "bound" else O.lipschitz_tight
    Lo = np.array([f(Q[i]) for i in range(len(Q))])
    _, _, L = B().local_solve(t32(Q6, dev), t32(Phi, dev), "fista", n_f=1, lipschitz=mode, want_lip=True)
    assert np.max(np.abs(L.cpu().numpy() - Lo) / Lo) <= tol


@pytest.mark.parametrize("mode", ["bound", "tight"])
@pytest.mark.parametrize("n_f", [1, 5, 20, 100])
def test_fista_matches_oracle(faces, mode, n_f):
    dev = _dev()
    Q, Phi, Q6, scale = faces
    f = O.lipschitz_bound if mode == "bound" else O.lipschitz_tight
    Lo = np.array([f(Q[i]) for i in range(len(Q))])
    res = [O.fista_local(Q[i], Phi[i], Lo[i], n_f) for i in range(len(Q))]
    vo = np.array([x[1] for x in res])
    ao = np.stack([x[0] for x in res])
    v, a, _ = B().local_solve(t32(Q6, dev), t32(Phi, dev), "fista", n_f=n_f, lip=t32(Lo, dev))
    assert np.max(np.abs(v.cpu().numpy() - vo) / scale) <= 1e-4
    assert np.max(np.abs(a.cpu().numpy() - ao)) <= 1e-3


def test_fista_unreached_vertices(faces):
    """Unreached vertices get weight zero; the values are feasible (never below
    the exact masked minimum) and approach it with more iterations."""
    dev = _dev()
    Q, Phi, Q6, scale = faces
    n = len(Q)
    P = Phi.copy()
    P[: n // 2, 0] = np.inf
    P[: n // 4, 1] = np.inf
    P[-10:] = np.inf                                       # nothing reached: +inf
    Qd, Pd = t32(Q6, dev), t32(P, dev)
    vx = B().local_solve(Qd, Pd, "exact")[0].cpu().numpy()
    assert np.all(np.isinf(vx[-10:]))
    gaps = []
    for n_f in (20, 400):
        v, a, _ = B().local_solve(Qd, Pd, "fista", n_f=n_f)
        v, a = v.cpu().numpy(), a.cpu().numpy()
        assert np.all(np.isinf(v[-10:]))
        assert np.all(a[: n // 2, 0] == 0) and np.all(a[: n // 4, 1] == 0)
        g = (v[:-10] - vx[:-10]) / scale[:-10]
        assert g.min() >= -2e-6
        gaps.append(np.median(g))
    assert gaps[1] < gaps[0]
    # one reached vertex: the edge value exactly
    one = slice(0, n // 4)
    v, _, _ = B().local_solve(Qd, Pd, "fista", n_f=3)
    np.testing.assert_allclose(v.cpu().numpy()[one], vx[one], rtol=1e-6)


def test_solver_setting_and_errors():
    dev = _dev()
    p = gi.cube_problem(4)
    plan = B().Plan(p.xyz, p.tets)
    assert B().get_local_solver(plan) == dict(solver="exact", n_f=32, lipschitz="tight")
    B().set_local_solver(plan, "fista", 7, "bound")
    assert B().get_local_solver(plan) == dict(solver="fista", n_f=7, lipschitz="bound")
    with pytest.raises(B().GbpError):
        B()._check(B()._set_solver(plan.handle, 2, 8, 1))
    with pytest.raises(B().GbpError):
        B()._check(B()._set_solver(plan.handle, 1, 0, 1))
    with pytest.raises(B().GbpError):
        B().local_solve(t32(np.zeros((2, 6)), dev), t32(np.zeros((2, 3)), dev), "fista", n_f=0)


def test_fista_forward_converges_to_exact():
    """12k shell: the forward with FISTA local solves (tightened step constant)
    approaches the oracle's exact times from above as n_f grows, and is within
    1e-4 at 128 iterations."""
    dev = _dev()
    p = gi.shell_problem(12_000, seed=81, n_roots=3, vscale_range=(0.7, 1.3))
    To, _ = O.solve(p.xyz, p.tets, p.D, p.vscale, p.root_node, p.root_t, eps_abs=0.0, eps_rel=1e-12)
    plan = B().Plan(p.xyz, p.tets)
    D, vs, rn, rt = t32(p.D, dev), t32(p.vscale, dev), i32(p.root_node, dev), t32(p.root_t, dev)
    errs = []
    for n_f in (16, 128):
        B().set_local_solver(plan, "fista", n_f, "tight")
        T, st = B().eikonal_forward(plan, D, vs, rn, rt)
        assert st["converged"]
        Tg = T.cpu().numpy().astype(np.float64)
        assert np.all(Tg >= To * (1 - 1e-5) - 1e-6)
        errs.append(rel_max(Tg, To))
    print(f"[fista forward] rel max err n_f=16 {errs[0]:.2e}, n_f=128 {errs[1]:.2e}", flush=True)
    assert errs[1] < errs[0] and errs[1] <= 1e-4
    B().set_local_solver(plan, "exact")
    T, _ = B().eikonal_forward(plan, D, vs, rn, rt)
    assert rel_max(T.cpu().numpy(), To) <= 1e-4


@pytest.mark.parametrize("mode", ["bound", "tight"])
def test_fista_iterations_match_oracle(faces, mode):
    """Per-face counts from Eq. (fista_convergence): the device decides them in
    FP32, the oracle in FP64 on the same step constants and the same (FP32)
    tolerance.  The FP32 evaluation of x = sqrt(4 L / (3 tau)) rounds the
    constant 4/3, the product, the quotient and the root, each within one FP32
    ulp, so it is within 8 * 2^-24 * x of the exact x; the counts may then
    differ (by one) only where x lies that close to an integer.  Those faces
    are counted and must be rare; every other face must agree exactly."""
    Q, Phi, Q6, scale = faces
    dev = _dev()
    _, _, lip = B().local_solve(t32(Q6, dev), t32(Phi, dev), "fista", n_f=1, lipschitz=mode,
                                want_alpha=False, want_lip=True)
    L = lip.cpu().numpy().astype(np.float64)
    n_near = 0
    for tau in (1e-1, 1e-3, 1e-5):
        tau32 = float(np.float32(tau))
        x = np.sqrt(4.0 * L / (3.0 * tau32))
        near = np.abs(x - np.round(x)) <= 8.0 * 2.0 ** -24 * x
        for n_max in (100000, 64):
            n = B().fista_iterations(lip, tau, n_max).cpu().numpy()
            no = O.fista_iterations(L, tau32, n_max)
            diff = n != no
            assert not np.any(diff & ~near), (tau, n_max, np.flatnonzero(diff & ~near)[:5])
            assert np.all(np.abs(n[diff] - no[diff]) == 1)
            n_near += int(np.sum(diff))
    print(f"[fista counts] {len(L)} faces x 6 settings: {n_near} differ by one at a "
          f"near-integer bound", flush=True)
    assert n_near <= 1e-3 * 6 * len(L)
    assert np.all(B().fista_iterations(lip, 0.0, 17).cpu().numpy() == 17)


def test_fista_per_face_counts_meet_tolerance(faces):
    """With the step constant of Eq. (lipschitz_est) (a true Lipschitz constant)
    each face's count keeps its value within tau of the exact minimum, up to the
    FP32 solve's own error; faces with up to 100 iterations match the oracle's
    iterates at the same count."""
    Q, Phi, Q6, scale = faces
    dev = _dev()
    m = 400
    Qd, Pd = t32(Q6[:m], dev), t32(Phi[:m], dev)
    _, _, lip = B().local_solve(Qd, Pd, "fista", n_f=1, lipschitz="bound", want_alpha=False,
                                want_lip=True)
    L = lip.cpu().numpy().astype(np.float64)
    exact = np.array([O.local_solve(Q[i], Phi[i])[0] for i in range(m)])
    n_parity = 0
    for tau_rel in (1e-1, 1e-2, 1e-3):
        tau = float(tau_rel * np.median(scale))
        n = B().fista_iterations(lip, tau, 100000).cpu().numpy()
        v = np.empty(m)
        for k in np.unique(n):
            idx = np.flatnonzero(n == k)
            vk, _, _ = B().local_solve(t32(Q6[idx], dev), t32(Phi[idx], dev), "fista", n_f=int(k),
                                       lip=lip[torch.as_tensor(idx, device=dev)], want_alpha=False)
            v[idx] = vk.cpu().numpy()
        slack = 1e-5 * scale[:m]
        assert np.all(v >= exact - slack)
        assert np.all(v - exact <= tau + slack), np.max(v - exact - tau)
        few = np.flatnonzero(n <= 100)
        n_parity += len(few)
        vo = np.array([O.fista_local(Q[i], Phi[i], L[i], int(n[i]))[1] for i in few])
        assert np.all(np.abs(v[few] - vo) <= 1e-4 * scale[few])
    assert n_parity >= 20


def test_fista_tolerance_setting_and_forward():
    """12k shell: the forward with per-face counts for tolerance tau (step
    constant of Eq. (lipschitz_est)) converges to times at or above the exact
    scheme's, at most tau per local problem along the longest chain of rounds
    above them, and closer with a smaller tau."""
    dev = _dev()
    p = gi.shell_problem(12_000, seed=81, n_roots=3, vscale_range=(0.7, 1.3))
    To, _ = O.solve(p.xyz, p.tets, p.D, p.vscale, p.root_node, p.root_t, eps_abs=0.0, eps_rel=1e-12)
    plan = B().Plan(p.xyz, p.tets)
    assert B().get_fista_tolerance(plan) == 0.0
    with pytest.raises(B().GbpError):
        B().set_fista_tolerance(plan, -1.0)
    with pytest.raises(B().GbpError):
        B().set_fista_tolerance(plan, float("nan"))
    D, vs, rn, rt = t32(p.D, dev), t32(p.vscale, dev), i32(p.root_node, dev), t32(p.root_t, dev)
    B().set_local_solver(plan, "fista", 100000, "bound")
    errs = []
    for tau in (1e-2, 1e-3):
        B().set_fista_tolerance(plan, tau)
        assert B().get_fista_tolerance(plan) == pytest.approx(tau)
        print(f"[case] fista tolerance {tau}", flush=True)
        T, st = B().eikonal_forward(plan, D, vs, rn, rt)
        assert st["converged"]
        Tg = T.cpu().numpy().astype(np.float64)
        assert np.all(Tg >= To * (1 - 1e-5) - 1e-6)
        assert np.max(Tg - To) <= tau * st["rounds"] + 1e-5 * To.max()
        errs.append(np.max(Tg - To))
    print(f"[fista tolerance] max err tau=1e-2 {errs[0]:.2e}, tau=1e-3 {errs[1]:.2e}", flush=True)
    assert errs[1] < errs[0]
    B().set_fista_tolerance(plan, 0.0)
    B().set_local_solver(plan, "exact")


def test_fista_forward_same_fixed_point_at_8_lanes():
    """The FISTA round at 8 lanes per vertex (three local problems per lane) reaches
    the same times as at 16 lanes (two per lane): the same local values, another
    order (FISTA values are not exactly monotone in the face values, so the
    fixed points may differ by up to the solver's own error)."""
    dev = _dev()
    p = gi.shell_problem(12_000, seed=81, n_roots=3, vscale_range=(0.7, 1.3))
    plan = B().Plan(p.xyz, p.tets)
    D, vs, rn, rt = t32(p.D, dev), t32(p.vscale, dev), i32(p.root_node, dev), t32(p.root_t, dev)
    B().set_local_solver(plan, "fista", 48, "tight")
    out = []
    for lanes, blocks in ((16, 1024), (8, 2048), (8, 256)):
        B().set_launch(plan, lanes, blocks, 2048, 16)
        T, st = B().eikonal_forward(plan, D, vs, rn, rt)
        assert st["converged"]
        out.append(T.cpu().numpy().astype(np.float64))
    for o in out[1:]:
        assert rel_max(o, out[0]) <= 1e-4

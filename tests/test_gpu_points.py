"""Roots at points inside elements (Sec. 2.3 Eq. (upwind_xi)) on the GPU against
the FP64 oracle: the vertex onsets, the forward solve started from them, the
gradients carried back to the points, onsets, tensors and velocity scales (by
the C ABI calls and through torch autograd), point location, and edge cases.
Bars as in the other parity tests: onsets 1e-6 and activation times 1e-4
relative (max norm), gradients 1e-3 relative (L2 per block).

At the benchmark's size (500k vertices, 100 points) the oracle computes the
onsets one by one, and two exact identities of the scheme that hold at any size
check the gradients: the onset shift sum_i dL/dt_i = sum_n g_n, and the velocity
homogeneity sum_n s_n dL/ds_n - sum_i t_i dL/dt_i = -g.T."""
import numpy as np
import pytest

import gbp_inputs as gi
import oracle as O
from test_gpu_parity import B, _dev, i32, rel_l2, rel_max, t32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


class PointCase:
    def __init__(self, n, n_points, seed):
        dev = _dev()
        self.dev = dev
        p = gi.shell_problem(n, seed=seed, n_roots=1, vscale_range=(0.6, 1.4))
        self.p = p
        cand = gi.tets_touching(p.tets, p.extra["endo"])
        self.k, self.X, self.t = gi.random_point_roots(p.xyz, p.tets, cand, n_points, 0.0, 20.0, seed=seed + 1)
        print(f"[case] point roots n_v={p.n_v} n_e={p.n_e} points={n_points}", flush=True)
        self.plan = B().Plan(p.xyz, p.tets)
        self.D, self.vs = t32(p.D, dev), t32(p.vscale, dev)
        self.kd, self.Xd, self.td = i32(self.k, dev), t32(self.X, dev), t32(self.t, dev)
        self.node, self.onset = B().point_roots(self.plan, self.D, self.vs, self.kd, self.Xd, self.td)
        self.T, _ = B().eikonal_forward(self.plan, self.D, self.vs, self.node, self.onset)
        torch.cuda.synchronize()


@pytest.fixture(scope="module")
def small():
    c = PointCase(12_000, 20, seed=61)
    p = c.p
    c.on_node, c.on_t = O.point_roots(p.xyz, p.tets, p.D, p.vscale, c.k, c.X, c.t)
    c.T_orc, st = O.solve(p.xyz, p.tets, p.D, p.vscale, c.on_node, c.on_t, eps_abs=0.0, eps_rel=1e-12)
    assert st["converged"]
    return c


def test_point_onsets_match_oracle(small):
    assert np.array_equal(small.node.cpu().numpy(), small.on_node)
    np.testing.assert_allclose(small.onset.cpu().numpy(), small.on_t, rtol=1e-6)


def test_forward_from_points_matches_oracle(small):
    assert rel_max(small.T.cpu().numpy(), small.T_orc) <= 1e-4


def _gpu_gradients(c, T_dev, g_dev):
    """The C ABI chain: adjoint down to the vertex roots, then the point rule."""
    dD, dvs, donset = B().eikonal_backward(c.plan, c.D, c.vs, c.node, c.onset, T_dev, g_dev)
    dt, dx = B().point_roots_backward(c.plan, c.D, c.vs, c.kd, c.Xd, donset, dL_dD=dD, dL_dvscale=dvs)
    return dD, dvs, dt, dx


def test_point_gradients_match_oracle(small):
    c, p = small, small.p
    g = np.random.Generator(np.random.PCG64(3)).normal(size=p.n_v)
    T_in = c.T_orc.astype(np.float32)          # both sides differentiate at the oracle's times
    dD, dvs, dt, dx = _gpu_gradients(c, t32(T_in, c.dev), t32(g, c.dev))
    ref = O.point_root_adjoint(p.xyz, p.tets, p.D, p.vscale, c.k, c.X, c.t, T_in.astype(np.float64), g)
    assert rel_l2(dt.cpu().numpy(), ref["dt"]) <= 1e-3
    assert rel_l2(dx.cpu().numpy(), ref["dx"]) <= 1e-3
    assert rel_l2(dD.cpu().numpy(), ref["dD"]) <= 1e-3
    assert rel_l2(dvs.cpu().numpy(), ref["dvscale"]) <= 1e-3


def test_point_gradients_through_autograd(small):
    """PointRootsFn + EikonalFn give the same gradients as the explicit calls."""
    from paper_2308_08410_amd import autograd as A
    c = small
    D = c.D.clone().requires_grad_(True)
    vs = c.vs.clone().requires_grad_(True)
    X = c.Xd.clone().requires_grad_(True)
    t = c.td.clone().requires_grad_(True)
    node, onset = A.point_roots(c.plan, D, vs, c.kd, X, t)
    T = A.eikonal(c.plan, D, vs, node, onset)
    g = t32(np.random.Generator(np.random.PCG64(4)).normal(size=c.p.n_v), c.dev)
    (T * g).sum().backward()
    dD, dvs, dt, dx = _gpu_gradients(c, T.detach(), g)
    for a, b in ((D.grad, dD), (vs.grad, dvs), (t.grad, dt), (X.grad, dx)):
        assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) <= 1e-5


def test_locate_points(small):
    c, p = small, small.p
    loc = B().locate_points(c.plan, c.Xd, tol=1e-5).cpu().numpy()
    # every answer holds its point (FP64 barycentric coordinates within tolerance)
    x = p.xyz.astype(np.float64)
    for r, j in enumerate(loc):
        assert j >= 0
        v = x[p.tets[j]]
        lam = np.linalg.solve((v[1:] - v[0]).T, c.X[r].astype(np.float64) - v[0])
        bary = np.concatenate([[1 - lam.sum()], lam])
        assert bary.min() >= -1e-4, (r, j, bary)
    # points well inside their generating element have it as the unique answer
    inside = O.locate_points(p.xyz, p.tets, c.X, tol=-1e-3)
    ok = inside >= 0
    assert ok.sum() >= 5
    assert np.array_equal(loc[ok], inside[ok])
    far = B().locate_points(c.plan, t32([[1e4, 1e4, 1e4]], c.dev)).cpu().numpy()
    assert far[0] == -1


def test_point_edge_cases(small):
    c, p = small, small.p
    dev = c.dev
    # no points
    node, onset = B().point_roots(c.plan, c.D, c.vs, i32(np.zeros(0), dev), t32(np.zeros((0, 3)), dev),
                                  t32(np.zeros(0), dev))
    assert node.numel() == 0 and onset.numel() == 0
    # an element id out of range is reported by the forward
    bad_k = c.k.copy()
    bad_k[3] = p.n_e
    node, onset = B().point_roots(c.plan, c.D, c.vs, i32(bad_k, dev), c.Xd, c.td)
    assert int(node[12:16].min()) == -1
    with pytest.raises(B().GbpError):
        B().eikonal_forward(c.plan, c.D, c.vs, node, onset)
    # a point on a vertex of its element: finite gradients, dL/dt is the sum
    k = c.k[:1].copy()
    X = p.xyz[p.tets[k[0]]][:1].astype(np.float32)
    node, onset = B().point_roots(c.plan, c.D, c.vs, i32(k, dev), t32(X, dev), c.td[:1])
    assert float(onset[0]) == float(c.td[0])
    g = t32([1.0, 2.0, 3.0, 4.0], dev)
    dt, dx = B().point_roots_backward(c.plan, c.D, c.vs, i32(k, dev), t32(X, dev), g)
    assert float(dt[0]) == 10.0 and torch.isfinite(dx).all()


@pytest.fixture(scope="module")
def full():
    return PointCase(500_000, 100, seed=71)


def test_full_size_point_roots(full):
    """500k vertices, 100 points (the paper fits 100 root points): onsets against
    the oracle, the forward at the roots' vertices, and the two gradient
    identities of the scheme."""
    c, p = full, full.p
    on_node, on_t = O.point_roots(p.xyz, p.tets, p.D, p.vscale, c.k, c.X, c.t)
    assert np.array_equal(c.node.cpu().numpy(), on_node)
    np.testing.assert_allclose(c.onset.cpu().numpy(), on_t, rtol=1e-6)
    T = c.T.cpu().numpy()
    assert np.all(T[on_node] <= on_t.astype(np.float32) * (1 + 1e-6))
    assert np.isfinite(T).all()
    g = np.random.Generator(np.random.PCG64(5)).normal(size=p.n_v).astype(np.float32)
    dD, dvs, dt, dx = _gpu_gradients(c, c.T, t32(g, c.dev))
    dt, dvs = dt.cpu().numpy().astype(np.float64), dvs.cpu().numpy().astype(np.float64)
    assert dt.sum() == pytest.approx(float(g.astype(np.float64).sum()), rel=1e-3, abs=1e-2)
    gT = float(g.astype(np.float64) @ T.astype(np.float64))
    lhs = p.vscale.astype(np.float64) @ dvs - c.t.astype(np.float64) @ dt
    assert lhs == pytest.approx(-gT, rel=1e-3)
    assert torch.isfinite(dx).all() and torch.isfinite(dD).all()

"""Pins of the triangle-mesh oracle (d = 2; the paper's 2-D study, Sec. 3.1):
the local solve against brute force and a bounded scalar minimiser, exact plane
waves, the point source between the continuous distance and edge Dijkstra with
equality on the grid's edge rays, first-order convergence, exact gradient
identities of the scheme, and central finite differences of the adjoint."""
import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra

import gbp_inputs as gi
from oracle import tri as O2
from conftest import random_spd, rng


def _edge_face(r):
    while True:
        E = r.normal(size=(2, 2))
        if abs(np.linalg.det(E)) > 0.2:
            break
    Q = E.T @ random_spd(r, 2, 6.0) @ E
    return Q


@pytest.mark.parametrize("seed", range(12))
def test_local_solve_vs_brute_force_and_bounded_minimiser(seed):
    r = rng(seed)
    Q = _edge_face(r)
    Phi = r.uniform(-0.6, 0.6, size=2) * np.sqrt(np.trace(Q) / 2)
    v, a = O2.local_solve2(Q[0, 0], Q[1, 1], Q[0, 1], Phi[0], Phi[1])
    t = np.linspace(0, 1, 200001)
    f = t * Phi[0] + (1 - t) * Phi[1] + np.sqrt(t * t * Q[0, 0] + 2 * t * (1 - t) * Q[0, 1] + (1 - t) ** 2 * Q[1, 1])
    assert f.min() >= v - 1e-12 and f.min() <= v + 1e-8
    res = so.minimize_scalar(lambda s: s * Phi[0] + (1 - s) * Phi[1] + np.sqrt(
        s * s * Q[0, 0] + 2 * s * (1 - s) * Q[0, 1] + (1 - s) ** 2 * Q[1, 1]), bounds=(0, 1),
        method="bounded", options=dict(xatol=1e-12))
    # the bounded minimiser stops at its own tolerance: never below the exact minimum
    assert float(v) <= res.fun + 1e-12 and res.fun - float(v) < 1e-6
    fa = a * Phi[0] + (1 - a) * Phi[1] + np.sqrt(a * a * Q[0, 0] + 2 * a * (1 - a) * Q[0, 1] + (1 - a) ** 2 * Q[1, 1])
    assert float(fa) == pytest.approx(float(v), abs=1e-12)


def test_local_solve_edge_cases():
    # one unreached vertex: the other vertex's edge value; both unreached: +inf
    v, a = O2.local_solve2(4.0, 9.0, 1.0, np.inf, 2.0)
    assert v == pytest.approx(5.0) and a == 0.0
    v, _ = O2.local_solve2(4.0, 9.0, 1.0, np.inf, np.inf)
    assert np.isinf(v)
    # shift equivariance
    Q = _edge_face(rng(99))
    v1, _ = O2.local_solve2(Q[0, 0], Q[1, 1], Q[0, 1], 0.3, -0.2)
    v2, _ = O2.local_solve2(Q[0, 0], Q[1, 1], Q[0, 1], 5.3, 4.8)
    assert float(v2) == pytest.approx(float(v1) + 5.0, abs=1e-12)


def _homog(tris, Dm):
    return np.tile(O2.pack2(Dm), (len(tris), 1))


@pytest.mark.parametrize("seed", range(3))
def test_plane_wave_exact(seed):
    """T = t0 + p.x with sqrt(p^T D p) = 1 is reproduced exactly when the inflow
    and tangential boundary nodes are roots with exact values."""
    r = rng(seed)
    xy, tris = gi.square_tri(8)
    x = xy.astype(np.float64)
    Dm = random_spd(r, 2, 8.0)
    u = r.normal(size=2)
    p = u / np.sqrt(u @ Dm @ u)
    vel = Dm @ p
    Tex = 0.3 + x @ p
    roots = [i for i, xi in enumerate(x) if any((xi[d] == 0.0 and vel[d] >= 0) or (xi[d] == 1.0 and vel[d] <= 0)
                                              for d in range(2))]
    T, st = O2.solve2(x, tris, _homog(tris, Dm), None, roots, Tex[roots])
    assert st["converged"]
    assert np.abs(T - Tex).max() < 1e-13


def _edge_dijkstra(x, tris, Minv3, roots, rt):
    M = O2.unpack2(Minv3)
    rows, cols, w = [], [], []
    for j, t in enumerate(tris):
        for a in range(3):
            for b in range(3):
                if a != b:
                    e = x[t[b]] - x[t[a]]
                    rows.append(t[a])
                    cols.append(t[b])
                    w.append(np.sqrt(e @ M[j] @ e))
    n = len(x)
    G = sp.csr_matrix((w, (rows, cols)), shape=(n + 1, n + 1))
    G = G.tolil()
    for r_, t_ in zip(roots, rt):
        G[n, r_] = t_ + 1e-300   # super source
    d = dijkstra(G.tocsr(), indices=n)
    return d[:n]


@pytest.mark.parametrize("aniso", [False, True])
def test_point_source_bounds_and_rays(aniso):
    n = 12
    xy, tris = gi.square_tri(n)
    x = xy.astype(np.float64)
    Dm = np.eye(2) if not aniso else random_spd(rng(5), 2, 5.0)
    D3 = _homog(tris, Dm)
    Minv = O2.metric_inverse2(D3, None, tris)
    T, st = O2.fim2(x, tris, Minv, [0], [0.0], eps_rel=1e-15)
    rr = np.sqrt(np.einsum("ni,ij,nj->n", x, np.linalg.inv(Dm), x))
    assert (T - rr).min() > -1e-13
    dj = _edge_dijkstra(x, tris, Minv, [0], [0.0])
    assert (T - dj).max() < 1e-12
    n1 = n + 1
    for i in range(n1):
        for (a, b) in [(i, 0), (0, i), (i, i)]:        # axes and the split diagonal
            k = a + n1 * b
            assert abs(T[k] - rr[k]) < 1e-13
    if not aniso:
        assert T[n1 * n1 - 1] == pytest.approx(np.sqrt(2.0), abs=1e-13)


def test_point_source_first_order():
    p = np.array([0.0, 0.0])
    Dm = random_spd(rng(7), 2, 4.0)
    err = []
    for n in (8, 16, 32):
        xy, tris = gi.square_tri(n)
        x = gi.jitter_nodes2(xy, 1.0 / n, 0.1, 3).astype(np.float64)
        x[0] = p
        T, _ = O2.solve2(x, tris, _homog(tris, Dm), None, [0], [0.0])
        rr = np.sqrt(np.einsum("ni,ij,nj->n", x, np.linalg.inv(Dm), x))
        err.append(np.abs(T - rr).max())
    assert err[0] > err[1] > err[2]
    assert err[2] < 0.75 * err[1] and err[1] < 0.75 * err[0]


def _problem(seed, n=6):
    r = rng(seed)
    xy, tris = gi.square_tri(n)
    x = gi.jitter_nodes2(xy, 1.0 / n, 0.15, seed).astype(np.float64)
    D3 = np.stack([O2.pack2(random_spd(r, 2, 6.0)) for _ in range(len(tris))])
    vs = r.uniform(0.5, 1.5, size=len(x))
    roots = r.choice(len(x), size=3, replace=False)
    rt = r.uniform(0, 0.3, size=3)
    return x, tris, D3, vs, roots, rt


@pytest.mark.parametrize("seed", range(4))
def test_gradient_identities(seed):
    x, tris, D3, vs, roots, rt = _problem(50 + seed)
    T, _ = O2.solve2(x, tris, D3, vs, roots, rt)
    g = rng(seed).normal(size=len(T))
    res = O2.adjoint2(x, tris, D3, vs, roots, rt, T, g)
    gT = g @ T
    assert res["droot_t"].sum() == pytest.approx(g.sum(), rel=1e-10)
    assert vs @ res["dvscale"] - rt @ res["droot_t"] == pytest.approx(-gT, rel=1e-9)
    assert (D3 * res["dD"]).sum() - 0.5 * rt @ res["droot_t"] == pytest.approx(-0.5 * gT, rel=1e-9)


@pytest.mark.parametrize("seed", range(2))
def test_gradient_central_fd(seed):
    x, tris, D3, vs, roots, rt = _problem(60 + seed, n=4)
    T, _ = O2.solve2(x, tris, D3, vs, roots, rt, eps_rel=1e-15)
    r = rng(seed)
    g = r.normal(size=len(T))
    res = O2.adjoint2(x, tris, D3, vs, roots, rt, T, g)
    h = 1e-6

    def L(D3_, vs_, rt_):
        return float(g @ O2.solve2(x, tris, D3_, vs_, roots, rt_, eps_rel=1e-15)[0])

    for k in range(len(rt)):
        e = np.zeros_like(rt)
        e[k] = h
        assert (L(D3, vs, rt + e) - L(D3, vs, rt - e)) / (2 * h) == pytest.approx(res["droot_t"][k], rel=1e-4, abs=1e-6)
    for n_ in r.choice(len(x), size=6, replace=False):
        e = np.zeros_like(vs)
        e[n_] = h
        assert (L(D3, vs + e, rt) - L(D3, vs - e, rt)) / (2 * h) == pytest.approx(res["dvscale"][n_], rel=1e-4, abs=1e-6)
    for j in r.choice(len(tris), size=4, replace=False):
        for c in range(3):
            e = np.zeros_like(D3)
            e[j, c] = h
            assert (L(D3 + e, vs, rt) - L(D3 - e, vs, rt)) / (2 * h) == pytest.approx(res["dD"][j, c], rel=1e-4, abs=1e-6)


def test_annulus_slice():
    """The 2-D slice workload: every vertex reached, roots hold their onsets or
    less, activation spreads over tens of ms."""
    p = gi.annulus_problem()
    T, st = O2.solve2(p.xyz, p.tets, p.D, p.vscale, p.root_node, p.root_t)
    assert st["converged"] and np.isfinite(T).all()
    assert np.all(T[p.root_node] <= p.root_t + 1e-6)
    assert 10.0 < T.max() < 120.0

"""Pins of the oracle's roots at points inside elements (Sec. 2.3 Eq. (upwind_xi))
and of their gradients: a point on a vertex reduces to a node root, the exact
lower bound of a point source in homogeneous media, first-order convergence to
the continuous distance, exact identities of the scheme, and central finite
differences through the whole solve."""
import numpy as np
import pytest

import gbp_inputs as gi
import oracle as O
from conftest import random_spd, rng
from test_oracle_fim import jittered_problem


def _homogeneous(n, seed, aniso=4.0):
    xyz, tets = gi.kuhn_cube(n)
    x = xyz.astype(np.float64)
    D = O.pack_sym(random_spd(rng(seed), 3, aniso))
    D6 = np.tile(D, (len(tets), 1))
    return x, tets, D6


def _solve_points(x, tets, D6, vs, k, X, t, eps_rel=1e-14):
    nodes, onset = O.point_roots(x, tets, D6, vs, k, X, t)
    T, st = O.solve(x, tets, D6, vs, nodes, onset, eps_abs=0.0, eps_rel=eps_rel)
    assert st["converged"]
    return T


def test_locate_points_finds_the_generating_element():
    xyz, tets = gi.kuhn_cube(4)
    k, X, _ = gi.random_point_roots(xyz, tets, np.arange(len(tets)), 20, 0.0, 1.0, seed=3)
    loc = O.locate_points(xyz, tets, X, tol=1e-6)
    # interior points lie in exactly one element
    assert np.array_equal(loc, k)
    assert O.locate_points(xyz, tets, [[2.0, 0.5, 0.5]])[0] == -1


@pytest.mark.parametrize("seed", range(3))
def test_point_on_a_vertex_is_a_node_root(seed):
    """With x_i at vertex a of its element and homogeneous D, Eq. (upwind_xi)
    gives the element's other vertices t_i + |v - v_a|_M, which is also what
    Alg. 2 computes from a node root at a (the straight edge is the geodesic,
    and the scheme never goes below the continuous distance), so both solves
    reach the same fixed point."""
    x, tets, D6 = _homogeneous(6, seed)
    r = rng(seed)
    k = int(r.integers(len(tets)))
    a = int(r.integers(4))
    t0 = float(r.uniform(0, 1))
    Tp = _solve_points(x, tets, D6, None, [k], x[tets[k, a]][None], [t0])
    Tn, _ = O.solve(x, tets, D6, None, [tets[k, a]], [t0], eps_abs=0.0, eps_rel=1e-14)
    assert np.abs(Tp - Tn).max() <= 1e-12 * np.abs(Tn).max()


@pytest.mark.parametrize("seed", range(3))
def test_point_source_lower_bound(seed):
    """Homogeneous medium: T >= t + |x - x_i|_M everywhere (the P1 interpolant of
    the convex distance lies above it and each local step obeys the triangle
    inequality), with equality on the element's own vertices."""
    x, tets, D6 = _homogeneous(6, 10 + seed)
    k, X, t = gi.random_point_roots(x, tets, np.arange(len(tets)), 1, 0.0, 1.0, seed=seed)
    X = X.astype(np.float64)
    T = _solve_points(x, tets, D6, None, k, X, t)
    M = np.linalg.inv(O.unpack_sym(D6[0]))
    e = x - X[0]
    r = float(t[0]) + np.sqrt(np.einsum("ni,ij,nj->n", e, M, e))
    assert np.all(T >= r - 1e-12)
    assert np.allclose(T[tets[k[0]]], r[tets[k[0]]], rtol=0, atol=1e-13)


def test_point_source_first_order_convergence():
    """max |T - r| falls with h (Bornemann-Rasch: O(h) for the linear scheme)
    for one physical point in nested Kuhn meshes."""
    p = np.array([[0.37, 0.41, 0.29]])
    D = O.pack_sym(random_spd(rng(7), 3, 4.0))
    M = np.linalg.inv(O.unpack_sym(D))
    err = []
    for n in (4, 8, 16):
        xyz, tets = gi.kuhn_cube(n)
        x = xyz.astype(np.float64)
        D6 = np.tile(D, (len(tets), 1))
        k = O.locate_points(x, tets, p)
        T = _solve_points(x, tets, D6, None, k, p, [0.0], eps_rel=1e-12)
        e = x - p[0]
        err.append(np.abs(T - np.sqrt(np.einsum("ni,ij,nj->n", e, M, e))).max())
    assert err[0] > err[1] > err[2]
    assert err[2] < 0.65 * err[1] and err[1] < 0.65 * err[0]


def _point_problem(seed, n=3, R=2):
    x, tets, D6, vs, _, _ = jittered_problem(seed, n=n)
    k, X, t = gi.random_point_roots(x, tets, np.arange(len(tets)), R, 0.0, 0.3, seed=seed)
    return x, tets, D6, vs, k, X.astype(np.float64), t.astype(np.float64)


@pytest.mark.parametrize("seed", range(3))
def test_point_root_identities(seed):
    """For L = g.T with roots at points:
       shift:     sum_i dL/dt_i = sum_n g_n over reached nodes;
       velocity:  sum_n s_n dL/ds_n - sum_i t_i dL/dt_i = -g.T   (T(cs, t/c) = T/c);
       tensor:    sum_j <D_j, dL/dD_j> - 1/2 sum_i t_i dL/dt_i = -1/2 g.T.
    (The point gradient has no such identity on a fixed mesh; finite
    differences pin it.)"""
    x, tets, D6, vs, k, X, t = _point_problem(100 + seed, n=4, R=3)
    T = _solve_points(x, tets, D6, vs, k, X, t)
    g = rng(seed).normal(size=len(T))
    res = O.point_root_adjoint(x, tets, D6, vs, k, X, t, T, g)
    gT = g @ T
    assert res["dt"].sum() == pytest.approx(g.sum(), rel=1e-10)
    assert vs @ res["dvscale"] - t @ res["dt"] == pytest.approx(-gT, rel=1e-9)
    assert (D6 * res["dD"]).sum() - 0.5 * t @ res["dt"] == pytest.approx(-0.5 * gT, rel=1e-9)


def _loss(x, tets, D6, vs, k, X, t, g):
    return float(g @ _solve_points(x, tets, D6, vs, k, X, t, eps_rel=1e-15))


@pytest.mark.parametrize("seed", range(2))
def test_point_root_gradient_central_fd(seed):
    x, tets, D6, vs, k, X, t = _point_problem(200 + seed)
    T = _solve_points(x, tets, D6, vs, k, X, t, eps_rel=1e-15)
    r = rng(seed)
    g = r.normal(size=len(T))
    res = O.point_root_adjoint(x, tets, D6, vs, k, X, t, T, g)
    h = 1e-6

    def fd(**kw):
        up = dict(D6=D6, vs=vs, X=X, t=t)
        dn = dict(up)
        for name, delta in kw.items():
            up[name] = up[name] + delta
            dn[name] = dn[name] - delta
        return (_loss(x, tets, up["D6"], up["vs"], k, up["X"], up["t"], g)
                - _loss(x, tets, dn["D6"], dn["vs"], k, dn["X"], dn["t"], g)) / (2 * h)

    for i in range(len(k)):
        e = np.zeros_like(t)
        e[i] = h
        assert fd(t=e) == pytest.approx(res["dt"][i], rel=1e-4, abs=1e-6)
        for c in range(3):
            e = np.zeros_like(X)
            e[i, c] = h
            assert fd(X=e) == pytest.approx(res["dx"][i, c], rel=1e-4, abs=1e-6)
        # the element holding the point: its tensor and its nodes' scales
        for c in range(6):
            e = np.zeros_like(D6)
            e[k[i], c] = h
            assert fd(D6=e) == pytest.approx(res["dD"][k[i], c], rel=1e-4, abs=1e-6)
        for n in tets[k[i]]:
            e = np.zeros_like(vs)
            e[n] = h
            assert fd(vs=e) == pytest.approx(res["dvscale"][n], rel=1e-4, abs=1e-6)


def test_point_root_gradient_sign():
    """A point moved towards a vertex reaches it earlier: dT_v/dx_i points away
    from v (the paper's -D (v - x)/|v - x|_D, Sec. 2.3)."""
    x, tets, D6 = _homogeneous(3, 5)
    k, X, t = gi.random_point_roots(x, tets, np.arange(len(tets)), 1, 0.0, 0.0, seed=5)
    X = X.astype(np.float64)
    v = tets[k[0], 0]
    T = _solve_points(x, tets, D6, None, k, X, t)
    g = np.zeros(len(T))
    g[v] = 1.0
    res = O.point_root_adjoint(x, tets, D6, None, k, X, t, T, g)
    assert res["dx"][0] @ (x[v] - X[0]) < 0

"""Pins of the oracle's global iteration (Alg. 2) against closed forms, graph
bounds, brute-force local minima and invariants of the fixed point."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra

import gbp_inputs as gi
import oracle as O
from conftest import rng, random_spd
from test_oracle_local import brute


def homogeneous(tets, Dm):
    D6 = O.pack_sym(Dm)
    return np.tile(D6[None, :], (len(tets), 1)).astype(np.float64)


def edge_dijkstra(xyz, tets, Minv6, root_node, root_t):
    """Shortest paths over mesh edges; an edge costs its smallest metric length
    among the elements that contain it.  A virtual source feeds the roots."""
    x = np.asarray(xyz, dtype=np.float64)
    M = O.unpack_sym(Minv6)
    n = len(x)
    cost = {}
    for j, t in enumerate(tets):
        for a in range(4):
            for b in range(a + 1, 4):
                u, v = int(t[a]), int(t[b])
                e = x[v] - x[u]
                c = np.sqrt(e @ M[j] @ e)
                key = (min(u, v), max(u, v))
                cost[key] = min(cost.get(key, np.inf), c)
    rt = np.asarray(root_t, dtype=np.float64)
    off = rt.min()
    rows = [k[0] for k in cost] + [k[1] for k in cost] + [n] * len(root_node)
    cols = [k[1] for k in cost] + [k[0] for k in cost] + list(root_node)
    vals = list(cost.values()) * 2 + list(rt - off + 1e-300)
    G = sp.csr_matrix((vals, (rows, cols)), shape=(n + 1, n + 1))
    d = dijkstra(G, directed=True, indices=n)
    return d[:n] + off


# ------------------------------------------------------------------ P2
@pytest.mark.parametrize("seed", range(4))
def test_plane_wave_exact(seed):
    """T(x) = t0 + p.x with sqrt(p^T D p) = 1 is reproduced exactly when every
    inflow or tangential boundary node is a root with its exact value."""
    r = rng(seed)
    xyz, tets = gi.kuhn_cube(6)
    x = xyz.astype(np.float64)
    Dm = random_spd(r, 3, 8.0)
    u = r.normal(size=3)
    p = u / np.sqrt(u @ Dm @ u)
    vel = Dm @ p
    t0 = 0.3
    Tex = t0 + x @ p
    roots = []
    for i, xi in enumerate(x):
        for d in range(3):
            if (xi[d] == 0.0 and vel[d] >= 0) or (xi[d] == 1.0 and vel[d] <= 0):
                roots.append(i)
                break
    roots = np.array(sorted(set(roots)), dtype=np.int32)
    D6 = homogeneous(tets, Dm)
    T, st = O.solve(x, tets, D6, None, roots, Tex[roots])
    assert st["converged"]
    assert np.abs(T - Tex).max() < 1e-13


# ------------------------------------------------------------------ P3
@pytest.mark.parametrize("aniso", [False, True])
def test_point_source_kuhn(aniso):
    n = 10
    xyz, tets = gi.kuhn_cube(n)
    x = xyz.astype(np.float64)
    Dm = np.eye(3) if not aniso else random_spd(rng(5), 3, 5.0)
    D6 = homogeneous(tets, Dm)
    Minv = O.metric_inverse(D6, None, tets)
    T, st = O.fim(x, tets, Minv, [0], [0.0], eps_abs=1e-14, eps_rel=0.0)
    Dinv = np.linalg.inv(Dm)
    rr = np.sqrt(np.einsum("ni,ij,nj->n", x, Dinv, x))
    # lower bound: the continuous distance
    assert (T - rr).min() > -1e-13
    # upper bound: shortest paths along mesh edges
    dj = edge_dijkstra(x, tets, Minv, [0], [0.0])
    assert (T - dj).max() < 1e-13
    # equality on the rays from the corner along mesh edge directions
    n1 = n + 1
    for i in range(n1):
        for (a, b, c) in [(i, 0, 0), (0, i, 0), (0, 0, i), (i, i, 0), (i, 0, i), (0, i, i), (i, i, i)]:
            k = a + n1 * (b + n1 * c)
            assert abs(T[k] - rr[k]) < 1e-13
    if not aniso:
        h = 1.0 / n
        assert T[n] == pytest.approx(n * h, abs=1e-14)
        assert T[n1 ** 3 - 1] == pytest.approx(np.sqrt(3.0), abs=1e-13)


# ------------------------------------------------------------------ P4
def test_first_order_convergence():
    """Mesh refinement (Hopf-Lax convergence to the viscosity solution, Sec. 2.1)."""
    errs = []
    for n in (5, 10, 20):
        xyz, tets = gi.kuhn_cube(n)
        x = xyz.astype(np.float64)
        D6 = homogeneous(tets, np.eye(3))
        T, _ = O.solve(x, tets, D6, None, [0], [0.0], eps_abs=1e-14, eps_rel=0)
        errs.append(np.abs(T - np.linalg.norm(x, axis=1)).max())
    # a point source converges at the first-order rate with the logarithmic
    # factor of the source singularity: err ~ C h log(1/h)
    hs = np.array([1 / 5, 1 / 10, 1 / 20])
    c = np.array(errs) / (hs * np.log(1 / hs))
    assert errs[0] > errs[1] > errs[2]
    assert c.max() / c.min() < 1.1, (errs, c)


# ------------------------------------------------------------------ P6
def jittered_problem(seed, n=4, aniso=6.0):
    r = rng(seed)
    xyz, tets = gi.kuhn_cube(n)
    x = gi.jitter_nodes(xyz, 1.0 / n, 0.12, seed).astype(np.float64)
    D6 = np.stack([O.pack_sym(random_spd(r, 3, aniso)) for _ in range(len(tets))])
    vs = r.uniform(0.5, 1.5, size=len(x))
    roots = r.choice(len(x), size=3, replace=False).astype(np.int32)
    rt = r.uniform(0, 0.3, size=3)
    return x, tets, D6, vs, roots, rt


@pytest.mark.parametrize("seed", range(3))
def test_jacobi_gauss_seidel_same_fixed_point(seed):
    x, tets, D6, vs, roots, rt = jittered_problem(seed)
    Tj, sj = O.solve(x, tets, D6, vs, roots, rt, mode="jacobi")
    Tg, sg = O.solve(x, tets, D6, vs, roots, rt, mode="gauss_seidel")
    assert sj["converged"] and sg["converged"]
    assert np.abs(Tj - Tg).max() < 1e-11 * np.abs(Tj).max()
    assert sg["sweeps"] <= sj["sweeps"]


@pytest.mark.parametrize("seed", range(3))
def test_warm_two_sided_converges_from_any_guess(seed):
    x, tets, D6, vs, roots, rt = jittered_problem(10 + seed)
    T, _ = O.solve(x, tets, D6, vs, roots, rt)
    r = rng(seed)
    guesses = [0.5 * T, 1.5 * T + 0.3, T * (1 + 0.05 * r.normal(size=len(T))), np.zeros_like(T),
               np.full_like(T, 5.0)]
    for gss in guesses:
        Tw, st = O.solve(x, tets, D6, vs, roots, rt, mode="warm", T_init=gss)
        assert st["converged"]
        assert np.abs(Tw - T).max() < 1e-10 * np.abs(T).max()


def test_min_update_from_low_guess_is_stuck():
    """Why warm starts need the two-sided update: a guess below the solution is
    a subsolution (every face value exceeds it), so min(T, F(T)) leaves it."""
    x, tets, D6, vs, roots, rt = jittered_problem(21)
    T, _ = O.solve(x, tets, D6, vs, roots, rt)
    low = 0.5 * T
    Minv = O.metric_inverse(D6, vs, tets)
    par = O.parent_map(x, tets, Minv, roots, rt, low)
    nonroot = np.ones(len(T), bool)
    nonroot[roots] = False
    assert np.all(par["best"][nonroot] >= low[nonroot])
    assert np.abs(low - T).max() > 0.1 * np.abs(T).max()


@pytest.mark.parametrize("seed", range(2))
def test_fixed_point_residual_bruteforce(seed):
    """Every node equals min(onset, min over its faces of the local minimum), the
    local minima taken by brute force on a barycentric grid (no KKT solver)."""
    x, tets, D6, vs, roots, rt = jittered_problem(30 + seed, n=2)
    T, _ = O.solve(x, tets, D6, vs, roots, rt)
    Minv = O.metric_inverse(D6, vs, tets)
    tr = np.full(len(x), np.inf)
    for n_, t_ in zip(roots, rt):
        tr[n_] = min(tr[n_], t_)
    for i in range(len(x)):
        best = tr[i]
        for j, tet in enumerate(tets):
            ks = np.nonzero(tet == i)[0]
            if len(ks) == 0:
                continue
            Q, fv = O.face_Q(x, tet, Minv[j], int(ks[0]))
            bval, _ = brute(Q, T[fv], N=200)
            best = min(best, bval)
        lip = np.abs(T).max() + 3.0
        assert T[i] <= best + 1e-12
        assert best - T[i] <= 2 * lip / 200


def test_edge_dijkstra_upper_bound_random():
    x, tets, D6, vs, roots, rt = jittered_problem(40, n=5)
    Minv = O.metric_inverse(D6, vs, tets)
    T, _ = O.fim(x, tets, Minv, roots, rt)
    dj = edge_dijkstra(x, tets, Minv, roots, rt)
    assert (T - dj).max() < 1e-12


def test_duplicate_roots_take_min_and_unreached_is_inf():
    xyz, tets = gi.kuhn_cube(2)
    x = xyz.astype(np.float64)
    n = len(x)
    # add a disconnected element far away
    x = np.vstack([x, x[:4] + 10.0])
    tets2 = np.vstack([tets, np.array([[n, n + 1, n + 2, n + 3]])]).astype(np.int32)
    D6 = homogeneous(tets2, np.eye(3))
    T1, _ = O.solve(x, tets2, D6, None, [0, 0, 5], [0.4, 0.1, 0.9])
    T2, _ = O.solve(x, tets2, D6, None, [0, 5], [0.1, 0.9])
    assert np.array_equal(T1, T2)
    assert T1[0] == pytest.approx(0.1)
    assert np.all(np.isinf(T1[n:])) and np.all(np.isfinite(T1[:n]))


def test_cube_config_sweeps_and_values():
    """The 21^3-node cube workload: converges, exact on the diagonal rays."""
    p = gi.cube_problem(20)
    T, st = O.solve(p.xyz, p.tets, p.D, p.vscale, p.root_node, p.root_t, eps_abs=1e-10, eps_rel=0)
    assert st["converged"]
    assert T[20] == pytest.approx(1.0, abs=1e-12)
    assert T[-1] == pytest.approx(np.sqrt(3.0), abs=1e-12)

"""Brute-force pin of the eikonal scheme (Sec. 2.1): shortest paths on a
Steiner-refined graph (``oracle/steiner.py``) approach the exact geodesic
distance of a metric that is constant per element, and the oracle's Hopf-Lax
fixed point approaches the same limit as the mesh is refined.  The graph shares
nothing with the scheme (no local problem, no interpolation)."""
import numpy as np
import pytest

import gbp_inputs as gi
import oracle as O
from conftest import rng, random_spd
from oracle import steiner as S
from test_oracle_fim import edge_dijkstra, homogeneous


def blocks_problem(n, seed=3):
    """Unit cube, n^3 Kuhn cells, a velocity tensor per octant (2x2x2 blocks of
    random SPD tensors, anisotropy up to 6): the medium is the same for every n
    divisible by 2, so the exact geodesic distance does not depend on n."""
    r = rng(seed)
    Ds = [O.pack_sym(random_spd(r, 3, 6.0)) for _ in range(8)]
    xyz, tets = gi.kuhn_cube(n)
    x = xyz.astype(np.float64)
    c = x[tets].mean(axis=1)
    b = (c[:, 0] > 0.5).astype(int) + 2 * (c[:, 1] > 0.5) + 4 * (c[:, 2] > 0.5)
    D6 = np.stack([Ds[k] for k in b])
    return x, tets, O.metric_inverse(D6, None, tets)


def probe(n):
    """Vertices of the 5^3 grid of spacing 1/4 (present in every mesh with 4 | n)."""
    n1, s = n + 1, n // 4
    g = np.arange(0, n1, s)
    k, j, i = np.meshgrid(g, g, g, indexing="ij")
    return (i + n1 * (j + n1 * k)).ravel()


def test_level_zero_is_edge_dijkstra():
    x, tets, Minv = blocks_problem(4)
    roots, rt = np.array([0, 77], np.int32), np.array([0.0, 0.25])
    d0, _, _ = S.steiner_distance(x, tets, Minv, roots, rt, 0)
    assert np.abs(d0 - edge_dijkstra(x, tets, Minv, roots, rt)).max() < 1e-12


def test_homogeneous_converges_to_closed_form():
    """Homogeneous anisotropic medium, vertex source on a jittered mesh: every
    graph path is an admissible path, so d >= the straight-line distance
    sqrt(x^T D^-1 x) at every graph point; nested levels never increase d; the
    error shrinks with the level and the finest is within 1% of the exact value."""
    xyz, tets = gi.kuhn_cube(3)
    x = gi.jitter_nodes(xyz, 1.0 / 3, 0.12, 5).astype(np.float64)
    x[0] = 0.0
    Dm = random_spd(rng(7), 3, 6.0)
    Minv = O.metric_inverse(homogeneous(tets, Dm), None, tets)
    Dinv = np.linalg.inv(Dm)
    errs, prev = [], None
    for m in (0, 1, 3, 7):
        dv, d, pts = S.steiner_distance(x, tets, Minv, [0], [0.0], m)
        exact = np.sqrt(np.einsum("ni,ij,nj->n", pts, Dinv, pts))
        assert np.all(d >= exact - 1e-12)
        if prev is not None:
            assert np.all(dv <= prev + 1e-12)
        prev = dv
        ev = exact[: len(x)]
        errs.append(np.max(dv - ev) / ev.max())
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < 0.01, errs


def test_fim_converges_to_the_steiner_limit():
    """Piecewise-constant anisotropic medium (one tensor per octant), source at a
    corner.  The graph distance of the 4^3 mesh at level 7 stands for the exact
    geodesic distance: levels 1, 3, 7 decrease by ~2.6% and ~1% of the largest
    time (so level 7 is within about 1% above the limit; the 8^3 mesh at level 7
    agrees with it to ~1e-3).  The oracle's fixed point on meshes of 4^3 to 32^3
    cells approaches it at the first-order rate of a point source (error
    ~ h log(1/h): a factor of ~0.63-0.75 per halving of h), never falling below
    it by more than the reference's own uncertainty."""
    x, tets, Minv = blocks_problem(4)
    d3, _, _ = S.steiner_distance(x, tets, Minv, [0], [0.0], 3)
    d7, _, _ = S.steiner_distance(x, tets, Minv, [0], [0.0], 7)
    ref = d7[probe(4)]
    scale = ref.max()
    assert np.all(d7 <= d3 + 1e-12)
    gap = np.max(d3 - d7)
    assert gap <= 0.015 * scale
    errs = []
    for n in (4, 8, 16, 32):
        xn, tn, Mn = blocks_problem(n)
        T, st = O.fim(xn, tn, Mn, [0], [0.0], eps_abs=1e-14, eps_rel=0.0)
        assert st["converged"]
        e = T[probe(n)] - ref
        assert e.min() >= -gap
        errs.append(np.abs(e).max() / scale)
    print(f"[steiner] FIM vs graph limit, 4^3..32^3 cells: {np.round(errs, 4)}", flush=True)
    for a, b in zip(errs, errs[1:]):
        assert b <= 0.8 * a
    assert errs[-1] < 0.015

"""Brute-force geodesic distances on a Steiner-refined graph.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``).  It is a reference for
the eikonal scheme that shares nothing with it: no local problem, no
interpolation, only straight segments and Dijkstra's algorithm.

Sec. 2.1 defines the activation time as the shortest travel time from the
initial conditions in the metric ||e||_D, and the Hopf-Lax scheme converges to
that viscosity solution as the mesh is refined.  With the metric constant in
each element (D_eff,j), a shortest path is straight inside every element and
bends only where it crosses element boundaries.  Placing points on those
boundaries and joining every pair of points of one element by a straight segment
of cost sqrt(d^T D_eff,j^-1 d) gives a graph whose shortest paths are
admissible paths of the continuous problem, so its distances are upper bounds of
the exact geodesic distance; as the points fill the boundaries they converge to
it (the Steiner-point method for weighted-region shortest paths).

Points of the graph, for a refinement level m >= 0:
  * the mesh vertices;
  * m points on every edge (u, v): u + k/(m+1) (v - u), k = 1..m;
  * on every triangular face (a, b, c) the interior lattice points
    (i a + j b + l c)/(m+1) with i, j, l >= 1 and i + j + l = m + 1.
Levels m with m + 1 = 1, 2, 4, 8, ... give nested point sets, so their distances
can only decrease from one such level to the next.  m = 0 is the graph of mesh
edges.  A segment lying in a face shared by two elements is present once per
element; the cheaper copy is kept.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra


def _unpack(M6):
    M6 = np.asarray(M6, np.float64)
    M = np.empty(M6.shape[:-1] + (3, 3))
    M[..., 0, 0], M[..., 1, 1], M[..., 2, 2] = M6[..., 0], M6[..., 1], M6[..., 2]
    M[..., 0, 1] = M[..., 1, 0] = M6[..., 3]
    M[..., 0, 2] = M[..., 2, 0] = M6[..., 4]
    M[..., 1, 2] = M[..., 2, 1] = M6[..., 5]
    return M


def _lattice(m):
    """Interior lattice (i, j, l), i + j + l = m + 1, all >= 1, as weights / (m+1)."""
    pts = [(i, j, m + 1 - i - j) for i in range(1, m + 1) for j in range(1, m + 1 - i)]
    return np.array(pts, np.float64).reshape(-1, 3) / (m + 1)


def steiner_graph(xyz, tets, Minv6, m):
    """The refined graph: (coordinates [N, 3], csr matrix of segment costs [N, N])."""
    x = np.asarray(xyz, np.float64)
    tets = np.asarray(tets, np.int64)
    n_v, n_e = len(x), len(tets)
    # unique edges and faces, each with its vertices in increasing order
    loc_edges = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    loc_faces = [(a, b, c) for a in range(4) for b in range(a + 1, 4) for c in range(b + 1, 4)]
    st = np.sort(tets, axis=1)
    E = np.concatenate([st[:, [a, b]] for a, b in loc_edges])
    F = np.concatenate([st[:, [a, b, c]] for a, b, c in loc_faces])
    edges, e_of = np.unique(E, axis=0, return_inverse=True)
    faces, f_of = np.unique(F, axis=0, return_inverse=True)
    e_of = e_of.reshape(len(loc_edges), n_e).T          # [n_e, 6] edge index per local edge
    f_of = f_of.reshape(len(loc_faces), n_e).T          # [n_e, 4] face index per local face
    k = np.arange(1, m + 1, dtype=np.float64) / (m + 1)
    lat = _lattice(m)
    n_ep, n_fp = m, len(lat)
    e_base = n_v
    f_base = n_v + len(edges) * n_ep
    N = f_base + len(faces) * n_fp
    coords = np.empty((N, 3))
    coords[:n_v] = x
    if n_ep:
        u, v = x[edges[:, 0]], x[edges[:, 1]]
        coords[e_base:f_base] = (u[:, None, :] + k[None, :, None] * (v - u)[:, None, :]).reshape(-1, 3)
    if n_fp:
        coords[f_base:] = np.einsum("pk,fkd->fpd", lat, x[faces]).reshape(-1, 3)
    # boundary points of every element (global ids), [n_e, P]
    ids = [st]
    if n_ep:
        ids.append((e_base + e_of[:, :, None] * n_ep + np.arange(n_ep)[None, None, :]).reshape(n_e, -1))
    if n_fp:
        ids.append((f_base + f_of[:, :, None] * n_fp + np.arange(n_fp)[None, None, :]).reshape(n_e, -1))
    ids = np.concatenate(ids, axis=1)
    P = ids.shape[1]
    ia, ib = np.triu_indices(P, k=1)
    M = _unpack(Minv6)
    rows, cols, vals = [], [], []
    for a0 in range(0, n_e, 256):
        sl = slice(a0, min(n_e, a0 + 256))
        d = coords[ids[sl][:, ib]] - coords[ids[sl][:, ia]]          # [b, pairs, 3]
        c = np.sqrt(np.einsum("bpi,bij,bpj->bp", d, M[sl], d))
        rows.append(ids[sl][:, ia].ravel())
        cols.append(ids[sl][:, ib].ravel())
        vals.append(c.ravel())
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    w = np.concatenate(vals)
    lo, hi = np.minimum(r, c), np.maximum(r, c)
    key = lo * N + hi
    order = np.lexsort((w, key))                     # by key, cheapest first
    key, w = key[order], w[order]
    first = np.ones(len(key), bool)
    first[1:] = key[1:] != key[:-1]
    key, w = key[first], w[first]
    lo, hi = key // N, key % N
    G = sp.csr_matrix((np.concatenate([w, w]), (np.concatenate([lo, hi]), np.concatenate([hi, lo]))),
                      shape=(N, N))
    return coords, G


def steiner_distance(xyz, tets, Minv6, root_node, root_t, m):
    """Shortest travel times from the roots (onset root_t at vertex root_node)
    over the Steiner graph of level m.  Returns (distance at the mesh vertices
    [n_v], distance at every graph point [N], coordinates [N, 3])."""
    n_v = len(xyz)
    coords, G = steiner_graph(xyz, tets, Minv6, m)
    rn = np.atleast_1d(np.asarray(root_node, np.int64))
    rt = np.atleast_1d(np.asarray(root_t, np.float64))
    best = {}
    for n, t in zip(rn, rt):
        best[int(n)] = min(best.get(int(n), np.inf), float(t))
    nodes = np.array(sorted(best), np.int64)
    times = np.array([best[n] for n in nodes])
    # a virtual source feeds the roots with their onsets, shifted to be >= 1 so
    # that no edge has cost zero (sparse storage would drop it)
    off = times.min() - 1.0
    N = G.shape[0]
    src = sp.csr_matrix((times - off, (np.full(len(nodes), N), nodes)), shape=(N + 1, N + 1))
    G1 = (sp.bmat([[G, None], [None, sp.csr_matrix((1, 1))]], format="csr") + src).tocsr()
    d = dijkstra(G1, directed=True, indices=N)[:N] + off
    return d[:n_v], d, coords

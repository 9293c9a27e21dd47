"""FP64 CPU oracle for triangle meshes (d = 2), the setting of the paper's 2-D
study (Sec. 3.1).

TEST INFRASTRUCTURE ONLY: only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library.

* ``local_solve2``  the local problem of Sec. 2.2 Eq. (upwind_eq_lsqr) with d = 2:
                    min over the segment of <alpha, Phi> + sqrt(alpha^T Q alpha),
                    written out as its three KKT candidates (two vertices, one
                    interior point), vectorised over faces
* ``fim2``          Alg. 2 (Jacobi) on a triangle mesh
* ``parent_map2``   the minimising triangle and weights of every vertex
* ``adjoint2``      Sec. 2.3 along the frozen parents, one sparse solve

Conventions: ``xy`` [n_v, 2], ``tris`` [n_t, 3], ``D3`` [n_t, 3] the velocity
tensor packed (xx, yy, xy); the step cost in triangle j is sqrt(e^T D_eff^-1 e)
with D_eff = sbar^2 D, sbar the mean of the three nodal velocity scales.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import active_roots


def unpack2(D3):
    D3 = np.asarray(D3, dtype=np.float64)
    M = np.empty(D3.shape[:-1] + (2, 2))
    M[..., 0, 0] = D3[..., 0]
    M[..., 1, 1] = D3[..., 1]
    M[..., 0, 1] = M[..., 1, 0] = D3[..., 2]
    return M


def pack2(M):
    return np.stack([M[..., 0, 0], M[..., 1, 1], M[..., 0, 1]], axis=-1)


def mean_scale2(vscale, tris):
    return np.asarray(vscale, dtype=np.float64)[np.asarray(tris)].mean(axis=1)


def metric_inverse2(D3, vscale, tris):
    """Per-triangle D_eff^-1 packed (xx, yy, xy)."""
    D = unpack2(D3)
    sbar = mean_scale2(vscale, tris) if vscale is not None else np.ones(len(D))
    return pack2(np.linalg.inv(D * (sbar ** 2)[:, None, None]))


def local_solve2(qaa, qbb, qab, pa, pb):
    """Vectorised local solve on faces (a, b) seen from a target vertex: Q is the
    2x2 Gram E^T D_eff^-1 E of the edges to a and b, Phi = (pa, pb).  Candidates
    (as the general KKT construction with supports {a}, {b}, {a, b}):
      {a}: pa + sqrt(qaa);  {b}: pb + sqrt(qbb);
      {a, b}: with Phi' = Phi - m (m = min Phi), a~ = 1^T Q^-1 1, b~ = 1^T Q^-1 Phi',
              c~ = Phi'^T Q^-1 Phi', disc = b~^2 - a~ (c~ - 1): if disc > 0 the
              point alpha = Q^-1 (mu 1 - Phi') / sqrt(disc), mu = (b~ + sqrt(disc))/a~,
              if alpha >= 0, with value m + mu.
    Unreached vertices (+inf) leave only the other vertex's candidate.  Ties: the
    first candidate in the order {a}, {b}, {a, b}.  Returns (value, alpha_a)."""
    qaa, qbb, qab, pa, pb = (np.asarray(v, dtype=np.float64) for v in (qaa, qbb, qab, pa, pb))
    fa, fb = np.isfinite(pa), np.isfinite(pb)
    va = np.where(fa, pa + np.sqrt(qaa), np.inf)
    vb = np.where(fb, pb + np.sqrt(qbb), np.inf)
    best = va.copy()
    alpha = np.where(fa, 1.0, 0.0)
    take = vb < best
    best = np.where(take, vb, best)
    alpha = np.where(take, 0.0, alpha)
    both = fa & fb
    m = np.where(both, np.minimum(pa, pb), 0.0)
    Pa, Pb = np.where(both, pa - m, 0.0), np.where(both, pb - m, 0.0)
    det = qaa * qbb - qab * qab
    ia, ib, iab = qbb / det, qaa / det, -qab / det          # Q^-1
    at = ia + ib + 2 * iab
    ya, yb = ia * Pa + iab * Pb, iab * Pa + ib * Pb          # Q^-1 Phi'
    bt = ya + yb
    ct = Pa * ya + Pb * yb
    disc = bt * bt - at * (ct - 1.0)
    ok = both & (disc > 0)
    sd = np.sqrt(np.where(ok, disc, 1.0))
    mu = (bt + sd) / at
    xa = ((ia + iab) * mu - ya) / sd
    xb = ((iab + ib) * mu - yb) / sd
    ok &= (xa >= 0) & (xb >= 0)
    vi = np.where(ok, m + mu, np.inf)
    take = vi < best
    best = np.where(take, vi, best)
    alpha = np.where(take, xa / np.where(ok, xa + xb, 1.0), alpha)
    return best, alpha


def _faces(xy, tris, Minv3):
    """All (triangle, target slot) local problems: target, the two face vertices
    (in increasing local order) and the Gram entries."""
    x = np.asarray(xy, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    M = unpack2(Minv3)
    tgt, fa, fb, qaa, qbb, qab, tri = [], [], [], [], [], [], []
    for k in range(3):
        o = [n for n in range(3) if n != k]
        i, a, b = tris[:, k], tris[:, o[0]], tris[:, o[1]]
        ea, eb = x[a] - x[i], x[b] - x[i]
        tgt.append(i)
        fa.append(a)
        fb.append(b)
        qaa.append(np.einsum("ni,nij,nj->n", ea, M, ea))
        qbb.append(np.einsum("ni,nij,nj->n", eb, M, eb))
        qab.append(np.einsum("ni,nij,nj->n", ea, M, eb))
        tri.append(np.arange(len(tris)))
    return tuple(np.concatenate(v) for v in (tgt, fa, fb, qaa, qbb, qab, tri))


def fim2(xy, tris, Minv3, root_node, root_t, eps_rel=1e-12, max_sweeps=None):
    """Alg. 2 on a triangle mesh, Jacobi: every sweep evaluates every local
    problem from the previous values and takes T_i <- min(T_i, min over faces);
    roots start at their onset (the smallest onset of a node).  Stops when no
    value decreased by more than eps_rel max(1, |T|).  Returns (T, stats)."""
    n_v = len(xy)
    tgt, fa, fb, qaa, qbb, qab, _ = _faces(xy, tris, Minv3)
    T = np.full(n_v, np.inf)
    np.minimum.at(T, np.atleast_1d(np.asarray(root_node)), np.atleast_1d(np.asarray(root_t, np.float64)))
    max_sweeps = 10 * n_v if max_sweeps is None else max_sweeps
    for sweep in range(1, max_sweeps + 1):
        v, _ = local_solve2(qaa, qbb, qab, T[fa], T[fb])
        new = T.copy()
        np.minimum.at(new, tgt, v)
        changed = np.isfinite(new) & (new < T - eps_rel * np.maximum(1.0, np.abs(np.where(np.isfinite(T), T, 0))))
        T = new
        if not changed.any():
            return T, dict(sweeps=sweep, converged=True)
    return T, dict(sweeps=max_sweeps, converged=False)


def solve2(xy, tris, D3, vscale, root_node, root_t, eps_rel=1e-12):
    return fim2(xy, tris, metric_inverse2(D3, vscale, tris), root_node, root_t, eps_rel=eps_rel)


def parent_map2(xy, tris, Minv3, root_node, root_t, T):
    """At a fixed point: for every vertex the minimising local problem (lowest
    triangle index among values within 1e-12 max(1, T_i) of the minimum), its
    face vertices and weights; a vertex is its own parent (a root) when its
    smallest onset does not exceed that minimum."""
    n_v = len(xy)
    T = np.asarray(T, dtype=np.float64)
    tgt, fa, fb, qaa, qbb, qab, tri = _faces(xy, tris, Minv3)
    v, al = local_solve2(qaa, qbb, qab, T[fa], T[fb])
    best = np.full(n_v, np.inf)
    np.minimum.at(best, tgt, v)
    tol = 1e-12 * np.maximum(1.0, np.abs(np.where(np.isfinite(T), T, 0.0)))
    cand = np.isfinite(v) & (v <= best[tgt] + tol[tgt])
    par_tri = np.full(n_v, -1, dtype=np.int64)
    order = np.lexsort((tri[cand], tgt[cand]))            # by vertex, then triangle
    ci = np.nonzero(cand)[0][order]
    first = np.ones(len(ci), bool)
    first[1:] = tgt[ci][1:] != tgt[ci][:-1]
    pick = ci[first]
    par_tri[tgt[pick]] = tri[pick]
    par_node = np.full((n_v, 2), -1, dtype=np.int64)
    par_alpha = np.zeros((n_v, 2))
    par_node[tgt[pick], 0] = fa[pick]
    par_node[tgt[pick], 1] = fb[pick]
    par_alpha[tgt[pick], 0] = al[pick]
    par_alpha[tgt[pick], 1] = 1.0 - al[pick]
    troot = np.full(n_v, np.inf)
    np.minimum.at(troot, np.atleast_1d(np.asarray(root_node)), np.atleast_1d(np.asarray(root_t, np.float64)))
    root_self = np.isfinite(troot) & (troot <= best)
    par_tri[root_self] = -1
    par_node[root_self] = -1
    par_alpha[root_self] = 0.0
    return dict(par_tri=par_tri, par_node=par_node, par_alpha=par_alpha, best=best, root_self=root_self)


def adjoint2(xy, tris, D3, vscale, root_node, root_t, T, g, par=None):
    """Gradients of L = g.T w.r.t. the triangle tensors D (packed, off-diagonal
    doubled), the nodal scales and the onsets, with the parents frozen: solve
    (I - P^T) lam = g, then for vertex i with parent triangle j, weights alpha,
    e = sum_k alpha_k (x_k - x_i) and h = sqrt(e^T D_eff,j^-1 e):
      dL/dD_j += lam_i (-sbar_j^-2 D_j^-1 e e^T D_j^-1 / (2h)),
      dL/dsbar_j += lam_i (-h / sbar_j),  d sbar_j / d s_n = 1/3 on its nodes,
    and dL/dt_r = lam at the root's vertex for active roots."""
    x = np.asarray(xy, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    n_v = len(x)
    vs = np.ones(n_v) if vscale is None else np.asarray(vscale, dtype=np.float64)
    Minv = metric_inverse2(D3, vs, tris)
    if par is None:
        par = parent_map2(x, tris, Minv, root_node, root_t, T)
    c = np.nonzero(par["par_tri"] >= 0)[0]
    rows = np.repeat(c, 2)
    cols = par["par_node"][c].reshape(-1)
    vals = par["par_alpha"][c].reshape(-1)
    keep = vals > 0
    P = sp.csr_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n_v, n_v))
    g = np.asarray(g, dtype=np.float64).copy()
    g[~np.isfinite(np.asarray(T, dtype=np.float64))] = 0.0
    A = (sp.identity(n_v, format="csr") - P.T.tocsr()).tocsc()
    lam = np.asarray(spla.spsolve(A, g)).reshape(-1)
    D = unpack2(D3)
    Dinv = np.linalg.inv(D)
    sbar = mean_scale2(vs, tris)
    M = unpack2(Minv)
    i = np.nonzero((par["par_tri"] >= 0) & (lam != 0.0))[0]
    j = par["par_tri"][i]
    e = par["par_alpha"][i, 0][:, None] * (x[par["par_node"][i, 0]] - x[i]) + \
        par["par_alpha"][i, 1][:, None] * (x[par["par_node"][i, 1]] - x[i])
    h = np.sqrt(np.einsum("ni,nij,nj->n", e, M[j], e))
    u = np.einsum("nij,nj->ni", Dinv[j], e)
    coef = lam[i] / (sbar[j] ** 2 * 2.0 * h)
    dD = np.zeros((len(tris), 2, 2))
    np.add.at(dD, j, -coef[:, None, None] * u[:, :, None] * u[:, None, :])
    dsbar = np.zeros(len(tris))
    np.add.at(dsbar, j, lam[i] * (-h / sbar[j]))
    dvs = np.zeros(n_v)
    np.add.at(dvs, tris.reshape(-1), np.repeat(dsbar / 3.0, 3))
    dD3 = pack2(dD)
    dD3[:, 2] *= 2.0
    act = active_roots(root_node, root_t, par["root_self"])
    rn = np.atleast_1d(np.asarray(root_node))
    return dict(lam=lam, dD=dD3, dvscale=dvs, droot_t=np.where(act, lam[rn], 0.0), par=par)

"""Alg. 2 transcribed with PyTorch autograd on the CPU, float64, for tiny meshes.

TEST INFRASTRUCTURE ONLY.  This is the paper's own differentiation strategy
(Sec. 2.3 and Sec. 2.5: run the global iteration "with enabled gradient
computations" and back-propagate through every sweep) written as plainly as
possible.  The tests compare its gradients with ``oracle.adjoint`` (the frozen
parent system), which checks that back-propagation through the iteration equals
back-tracking along the geodesic parents.

The local problem is solved in closed form (KKT point of every face of the
simplex, then the minimum); autograd through the selected closed form gives the
derivative of the local minimum value.  The vertex update keeps the previous
value as a candidate (first index wins at ties), so at ties the gradient follows
the older value, which is what the paper's change mask is for (Sec. 2.5).
"""
from __future__ import annotations

import numpy as np
import torch

_SUBSETS = [(0,), (1,), (2,), (0, 1), (0, 2), (1, 2), (0, 1, 2)]


def _sym(D6):
    row0 = torch.stack([D6[:, 0], D6[:, 3], D6[:, 4]], dim=1)
    row1 = torch.stack([D6[:, 3], D6[:, 1], D6[:, 5]], dim=1)
    row2 = torch.stack([D6[:, 4], D6[:, 5], D6[:, 2]], dim=1)
    return torch.stack([row0, row1, row2], dim=1)


def _local_values(Q, Phi):
    """Q [F,3,3], Phi [F,3] (may hold +inf) -> min value [F]."""
    fin = torch.isfinite(Phi)
    Phis = torch.where(fin, Phi, torch.zeros_like(Phi))
    big = torch.where(fin, Phis, torch.full_like(Phis, float("inf")))
    m = big.min(dim=1).values
    m_safe = torch.where(torch.isfinite(m), m, torch.zeros_like(m))
    P = Phis - m_safe[:, None]
    cands = []
    for S in _SUBSETS:
        idx = list(S)
        ok = fin[:, idx].all(dim=1)
        if len(S) == 1:
            v = P[:, idx[0]] + torch.sqrt(Q[:, idx[0], idx[0]])
            cands.append(torch.where(ok, v, torch.full_like(v, float("inf"))))
            continue
        Qs = Q[:, idx][:, :, idx]
        Ps = P[:, idx]
        ones = torch.ones_like(Ps)
        y1 = torch.linalg.solve(Qs, ones)
        yP = torch.linalg.solve(Qs, Ps)
        a = y1.sum(dim=1)
        b = yP.sum(dim=1)
        c = (Ps * yP).sum(dim=1)
        disc = b * b - a * (c - 1.0)
        good = ok & (disc > 0)
        sd = torch.sqrt(torch.where(good, disc, torch.ones_like(disc)))
        mu = (b + sd) / a
        alpha = (mu[:, None] * y1 - yP) / sd[:, None]
        good = good & (alpha >= 0).all(dim=1)
        cands.append(torch.where(good, mu, torch.full_like(mu, float("inf"))))
    C = torch.stack(cands, dim=1)
    v = C.min(dim=1).values
    return torch.where(torch.isfinite(v), m_safe + v, v)


def solve_autograd(xyz, tets, D6, vscale, root_node, root_t, eps=1e-13, max_sweeps=10000):
    """Returns T (torch float64 tensor, differentiable w.r.t. D6, vscale and root_t
    when those are tensors with requires_grad)."""
    x = torch.as_tensor(np.asarray(xyz, dtype=np.float64))
    tets_np = np.asarray(tets, dtype=np.int64)
    n_v, n_e = len(x), len(tets_np)
    t_ = torch.as_tensor(tets_np)
    sbar = vscale[t_].mean(dim=1)
    Deff = _sym(D6) * (sbar ** 2)[:, None, None]
    Minv = torch.linalg.inv(Deff)
    # faces: (element j, local vertex k) -> face vertices = other locals in order
    fj, fk, fv = [], [], []
    for j in range(n_e):
        for k in range(4):
            fj.append(j)
            fk.append(tets_np[j, k])
            fv.append([tets_np[j, n] for n in range(4) if n != k])
    fj = torch.as_tensor(fj)
    tgt = torch.as_tensor(fk)
    fv = torch.as_tensor(np.asarray(fv))
    E = x[fv] - x[tgt][:, None, :]                 # [F,3,3] rows = edges
    Q = E @ Minv[fj] @ E.transpose(1, 2)
    # incident faces per node, padded
    deg = np.bincount(tgt.numpy(), minlength=n_v)
    W = int(deg.max()) + 1
    slot = np.zeros(len(fj), dtype=np.int64)
    cnt = np.ones(n_v, dtype=np.int64)
    for f, i in enumerate(tgt.numpy()):
        slot[f] = cnt[i]
        cnt[i] += 1
    slot = torch.as_tensor(slot)
    # roots
    inf = torch.tensor(float("inf"), dtype=torch.float64)
    rn = np.atleast_1d(np.asarray(root_node))
    phi = [inf] * n_v
    for r in range(len(rn)):
        i = int(rn[r])
        phi[i] = root_t[r] if not torch.isfinite(torch.as_tensor(phi[i])) else torch.minimum(phi[i], root_t[r])
    phi_km1 = torch.stack([p if torch.is_tensor(p) else torch.tensor(p) for p in phi])
    phi_km2 = torch.full((n_v,), float("inf"), dtype=torch.float64)
    for _ in range(max_sweeps):
        with torch.no_grad():
            old2, old1 = phi_km2, phi_km1
            changed = torch.isfinite(old1) & (~torch.isfinite(old2) | (old1 < old2 - eps))
            mask = changed[fv].any(dim=1)
        Phi = phi_km1[fv[mask]]
        vals = _local_values(Q[mask], Phi)
        cand = torch.full((n_v, W), float("inf"), dtype=torch.float64)
        cand = cand.index_put((tgt[mask], slot[mask]), vals)
        cand = torch.cat([phi_km1[:, None], cand[:, 1:]], dim=1)
        phi_k = cand.min(dim=1).values
        with torch.no_grad():
            done = not bool((torch.isfinite(phi_k) & (~torch.isfinite(phi_km1) |
                                                      (phi_k < phi_km1 - eps))).any())
        phi_km2, phi_km1 = phi_km1, phi_k
        if done:
            break
    return phi_km1

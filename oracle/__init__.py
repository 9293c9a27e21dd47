"""FP64 CPU oracle for the Geodesic-BP hot path (arXiv 2308.08410).

TEST INFRASTRUCTURE ONLY: only ``tests/``, the smoke check and the CPU-baseline
leg of the benchmark import this package.  It shares no code with the HIP
library (``paper_2308_08410_amd``) and never imports it.

Pieces
------
* ``local_solve``      exact minimum of the local problem, Sec. 2.2
                       Eq. (upwind_eq_lsqr)                       [C, gbp_oracle.c]
* ``fim``              Alg. 2 (Jacobi / Gauss-Seidel / two-sided warm start)
                                                                  [C, gbp_oracle.c]
* ``parent_map``       minimising element + barycentric weights per node
                                                                  [C, gbp_oracle.c]
* ``adjoint``          Sec. 2.3: back-propagation along the frozen geodesic parents,
                       Eq. (dto_grad), solved as one sparse linear system
* ``point_roots`` / ``point_roots_grad`` / ``point_root_adjoint``
                       roots at points inside elements, Sec. 2.3 Eq. (upwind_xi),
                       and the chain rule to the point, onset, D and velocity scale
* ``p1_stiffness`` / ``lead_field``
                       the lead weights B = K Z of Sec. 2.4 (P1 stiffness times the
                       point-electrode lead fields)
* ``ecg_forward`` / ``ecg_backward`` / ``ecg_loss``
                       Sec. 2.4: V_l(t) = sum_n B[n,l] U(t - phi_n) with the tanh
                       template, and the objective Eq. (inverse_ecg)
* ``fista_local``      Alg. 1 (FISTA on the local problem) with the Lipschitz
                       bound Eq. (lipschitz_est) and its tightened variant (Sec. 2.5)
* ``fista_iterations`` per-face iteration counts from the rate Eq. (fista_convergence)
* ``adam_step``        the optimiser used for the inverse problem (Sec. 2.4)

All arithmetic is float64.  Inputs may be float32 arrays (they are upcast).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gbp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (plain -O2, IEEE semantics;
    OpenMP only spreads independent elements or nodes over threads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu99", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                               _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def set_threads(n: int) -> int:
    """Host threads for the C loops of Alg. 2 (Jacobi and warm modes) and the
    parent map; 1 by default.  The results are the same for any count (the
    scatter-min is order-independent); only the time changes."""
    return int(_load().orc_set_threads(int(n)))


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_longlong)
        lib.orc_local_solve.argtypes = [dp, dp, dp, dp]
        lib.orc_local_solve.restype = ctypes.c_int
        lib.orc_fim.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, dp, ctypes.c_int, ip, dp,
                                ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, lp]
        lib.orc_fim.restype = ctypes.c_int
        lib.orc_parent_map.argtypes = [ctypes.c_int, dp, ctypes.c_int, ip, dp, ctypes.c_int, ip, dp,
                                       dp, ip, ip, dp, dp, dp, ip]
        lib.orc_parent_map.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


# --------------------------------------------------------------------------
# metric
# --------------------------------------------------------------------------
def unpack_sym(D6):
    D6 = np.asarray(D6, dtype=np.float64)
    M = np.empty(D6.shape[:-1] + (3, 3))
    M[..., 0, 0] = D6[..., 0]
    M[..., 1, 1] = D6[..., 1]
    M[..., 2, 2] = D6[..., 2]
    M[..., 0, 1] = M[..., 1, 0] = D6[..., 3]
    M[..., 0, 2] = M[..., 2, 0] = D6[..., 4]
    M[..., 1, 2] = M[..., 2, 1] = D6[..., 5]
    return M


def pack_sym(M):
    return np.stack([M[..., 0, 0], M[..., 1, 1], M[..., 2, 2], M[..., 0, 1], M[..., 0, 2],
                     M[..., 1, 2]], axis=-1)


def mean_scale(vscale, tets):
    """Per-element velocity scale: arithmetic mean of the four nodal scales."""
    return np.asarray(vscale, dtype=np.float64)[np.asarray(tets)].mean(axis=1)


def metric_inverse(D6, vscale, tets):
    """Per-element inverse of the effective velocity tensor,
    D_eff = sbar^2 D (sbar = mean nodal velocity scale), packed.  The local
    step cost is sqrt(e^T D_eff^{-1} e) (the norm of Sec. 2.1 with the paper's
    D = M^{-1})."""
    D = unpack_sym(D6)
    sbar = mean_scale(vscale, tets) if vscale is not None else np.ones(len(D))
    Deff = D * (sbar ** 2)[:, None, None]
    return pack_sym(np.linalg.inv(Deff))


# --------------------------------------------------------------------------
# local problem, Alg. 2 and parents (C)
# --------------------------------------------------------------------------
def local_solve(Q, Phi):
    """Exact min over the 2-simplex of <alpha, Phi> + sqrt(alpha^T Q alpha)
    (Sec. 2.2, Eq. (upwind_eq_lsqr)).  Returns (value, alpha[3], support mask)."""
    lib = _load()
    Q, qp = _d(np.asarray(Q, dtype=np.float64).reshape(9))
    Phi, pp = _d(Phi)
    val = np.zeros(1)
    alpha = np.zeros(3)
    mask = lib.orc_local_solve(qp, pp, val.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               alpha.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return float(val[0]), alpha, int(mask)


def face_Q(xyz, tet, Minv6, k):
    """Q = E^T Minv E for the face of element ``tet`` opposite its local vertex k
    (face vertices: the other three in increasing local order)."""
    x = np.asarray(xyz, dtype=np.float64)
    M = unpack_sym(Minv6)
    others = [n for n in range(4) if n != k]
    E = np.stack([x[tet[n]] - x[tet[k]] for n in others], axis=1)
    return E.T @ M @ E, [int(tet[n]) for n in others]


def fim(xyz, tets, Minv6, root_node, root_t, eps_abs=0.0, eps_rel=1e-12, max_sweeps=None,
        mode="jacobi", T_init=None):
    """Alg. 2.  mode: 'jacobi' (as written), 'gauss_seidel', or 'warm' (two-sided
    update from T_init).  Returns (T float64 [n_v], stats dict)."""
    lib = _load()
    xyz, xp = _d(xyz)
    tets, tp = _i(tets)
    Minv6, mp = _d(Minv6)
    rn, rp = _i(np.atleast_1d(root_node))
    rt, rtp = _d(np.atleast_1d(root_t))
    n_v, n_e = len(xyz), len(tets)
    if max_sweeps is None:
        max_sweeps = 10 * n_v
    m = {"jacobi": 0, "gauss_seidel": 1, "warm": 2}[mode]
    T = np.full(n_v, np.inf) if T_init is None else np.array(T_init, dtype=np.float64)
    T, Tp = _d(T)
    st = np.zeros(5, dtype=np.int64)
    rc = lib.orc_fim(n_v, xp, n_e, tp, mp, len(rn), rp, rtp, float(eps_abs), float(eps_rel),
                     int(max_sweeps), m, Tp, st.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)))
    stats = dict(sweeps=int(st[0]), solves=int(st[1]), decreases=int(st[2]), converged=bool(st[3]),
                 increases=int(st[4]), rc=rc)
    return T, stats


def parent_map(xyz, tets, Minv6, root_node, root_t, T):
    """Geodesic parents at a fixed point (see gbp_oracle.c).  Returns a dict with
    par_tet, par_node [n_v,3], par_alpha [n_v,3], best, gap, root_self."""
    lib = _load()
    xyz, xp = _d(xyz)
    tets, tp = _i(tets)
    Minv6, mp = _d(Minv6)
    rn, rp = _i(np.atleast_1d(root_node))
    rt, rtp = _d(np.atleast_1d(root_t))
    T, Tp = _d(T)
    n_v = len(xyz)
    par_tet = np.zeros(n_v, np.int32)
    par_node = np.zeros((n_v, 3), np.int32)
    par_alpha = np.zeros((n_v, 3))
    best = np.zeros(n_v)
    gap = np.zeros(n_v)
    root_self = np.zeros(n_v, np.int32)
    ip = ctypes.POINTER(ctypes.c_int)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.orc_parent_map(n_v, xp, len(tets), tp, mp, len(rn), rp, rtp, Tp,
                       par_tet.ctypes.data_as(ip), par_node.ctypes.data_as(ip),
                       par_alpha.ctypes.data_as(dp), best.ctypes.data_as(dp),
                       gap.ctypes.data_as(dp), root_self.ctypes.data_as(ip))
    return dict(par_tet=par_tet, par_node=par_node, par_alpha=par_alpha, best=best, gap=gap,
                root_self=root_self.astype(bool))


def solve(xyz, tets, D6, vscale, root_node, root_t, eps_abs=0.0, eps_rel=1e-12, mode="jacobi",
          T_init=None):
    """Convenience: metric + Alg. 2."""
    Minv = metric_inverse(D6, vscale, tets)
    return fim(xyz, tets, Minv, root_node, root_t, eps_abs=eps_abs, eps_rel=eps_rel, mode=mode,
               T_init=T_init)


# --------------------------------------------------------------------------
# adjoint (Sec. 2.3)
# --------------------------------------------------------------------------
def active_roots(root_node, root_t, root_self):
    """Root r is active iff its node is its own parent and r carries that node's
    smallest onset (lowest index among equal onsets)."""
    rn = np.atleast_1d(np.asarray(root_node))
    rt = np.atleast_1d(np.asarray(root_t, dtype=np.float64))
    act = np.zeros(len(rn), bool)
    seen = {}
    for r in range(len(rn)):
        n = int(rn[r])
        if n not in seen or rt[r] < rt[seen[n]]:
            seen[n] = r
    for n, r in seen.items():
        act[r] = bool(root_self[n])
    return act


def parent_matrix(par, n_v):
    """P[c, k] = alpha^c_k: the weights of node c's value on its parents
    (Eq. (dto_grad): the gradient of a node value is the alpha-weighted sum of
    the gradients of the face values it was computed from)."""
    c = np.nonzero(par["par_tet"] >= 0)[0]
    rows = np.repeat(c, 3)
    cols = par["par_node"][c].reshape(-1)
    vals = par["par_alpha"][c].reshape(-1)
    keep = vals > 0
    return sp.csr_matrix((vals[keep], (rows[keep], cols[keep])), shape=(n_v, n_v))


def adjoint(xyz, tets, D6, vscale, root_node, root_t, T, g, par=None):
    """Gradients of L = g . T with respect to the per-element velocity tensor D,
    the nodal velocity scales s and the root onsets t_r, holding the geodesic
    parents fixed (first variation: d alpha is neglected, Sec. 2.3).

    With P the parent-weight matrix, dT = P dT + b where b holds the explicit
    derivatives of each node's upwind value, so g.dT = lam.b with
    (I - P^T) lam = g.  For node i with parent element j and weights alpha,
    e = sum_k alpha_k (v_k - v_i), h = sqrt(e^T D_eff^-1 e) and
      dh/dD_j   = - sbar_j^-2 D_j^-1 e e^T D_j^-1 / (2 h),
      dh/dsbar_j = - h / sbar_j,   d sbar_j / d s_n = 1/4 for the 4 nodes of j,
    and dT_r/dt_r = 1 for active roots.
    Returns dict(lam, dD [n_e,6] (off-diagonals doubled), dvscale [n_v],
    droot_t [n_roots], par)."""
    x = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets)
    n_v = len(x)
    vs = np.ones(n_v) if vscale is None else np.asarray(vscale, dtype=np.float64)
    Minv = metric_inverse(D6, vs, tets)
    if par is None:
        par = parent_map(x, tets, Minv, root_node, root_t, T)
    P = parent_matrix(par, n_v)
    g = np.asarray(g, dtype=np.float64).copy()
    g[~np.isfinite(np.asarray(T, dtype=np.float64))] = 0.0
    A = (sp.identity(n_v, format="csr") - P.T.tocsr())
    # Order unknowns by decreasing T: a parent is (almost always) earlier than its
    # child, so the permuted system is nearly triangular and the direct solve
    # stays sparse.  The solution does not depend on the ordering.
    Tn = np.asarray(T, dtype=np.float64)
    order = np.argsort(-np.where(np.isfinite(Tn), Tn, np.inf), kind="stable")
    Ap = A[order][:, order].tocsc()
    lam = np.empty(n_v)
    lam[order] = np.asarray(spla.spsolve(Ap, g[order], permc_spec="NATURAL")).reshape(-1)

    D = unpack_sym(D6)
    Dinv = np.linalg.inv(D)
    sbar = mean_scale(vs, tets)
    Minv3 = unpack_sym(Minv)
    dD = np.zeros((len(tets), 3, 3))
    dsbar = np.zeros(len(tets))
    i = np.nonzero((par["par_tet"] >= 0) & (lam != 0.0))[0]
    j = par["par_tet"][i]
    e = np.zeros((len(i), 3))
    for k in range(3):
        e += par["par_alpha"][i, k][:, None] * (x[par["par_node"][i, k]] - x[i])
    hh = np.sqrt(np.einsum("ni,nij,nj->n", e, Minv3[j], e))
    u = np.einsum("nij,nj->ni", Dinv[j], e)
    coef = lam[i] / (sbar[j] ** 2 * 2.0 * hh)
    np.add.at(dD, j, -coef[:, None, None] * u[:, :, None] * u[:, None, :])
    np.add.at(dsbar, j, lam[i] * (-hh / sbar[j]))
    dvs = np.zeros(n_v)
    np.add.at(dvs, tets.reshape(-1), np.repeat(dsbar / 4.0, 4))
    dD6 = pack_sym(dD)
    dD6[:, 3:] *= 2.0
    act = active_roots(root_node, root_t, par["root_self"])
    rn = np.atleast_1d(np.asarray(root_node))
    droot = np.where(act, lam[rn], 0.0)
    return dict(lam=lam, dD=dD6, dvscale=dvs, droot_t=droot, par=par)


# --------------------------------------------------------------------------
# roots at points inside elements (Sec. 2.3 Eq. (upwind_xi))
# --------------------------------------------------------------------------
def locate_points(xyz, tets, points, tol=1e-12):
    """Index of an element containing each point (barycentric coordinates all
    >= -tol; the lowest such index), or -1.  Brute force over all elements."""
    x = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets)
    P = np.asarray(points, dtype=np.float64).reshape(-1, 3)
    v0 = x[tets[:, 0]]
    E = np.stack([x[tets[:, k]] - v0 for k in (1, 2, 3)], axis=2)      # [n_e,3,3] columns
    Einv = np.linalg.inv(E)
    out = np.full(len(P), -1, dtype=np.int64)
    for r, p in enumerate(P):
        lam = np.einsum("nij,nj->ni", Einv, p - v0)
        bary = np.concatenate([1.0 - lam.sum(1, keepdims=True), lam], axis=1)
        hit = np.nonzero((bary >= -tol).all(axis=1))[0]
        if len(hit):
            out[r] = hit[0]
    return out


def point_roots(xyz, tets, D6, vscale, root_tet, root_xyz, root_t):
    """Eq. (upwind_xi): a root at the point x_i of element E_k with onset t_i
    gives each vertex v of E_k the value t_i + ||v - x_i|| in the metric of E_k
    (D_eff^-1 of that element, the step cost of Alg. 2).  Returned as node
    roots (node ids [4R], onsets [4R]): root i's vertices at 4i..4i+3 in the
    element's vertex order.  Alg. 2 then keeps the smallest onset of a node."""
    x = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets)
    k = np.asarray(root_tet).reshape(-1)
    X = np.asarray(root_xyz, dtype=np.float64).reshape(-1, 3)
    t = np.asarray(root_t, dtype=np.float64).reshape(-1)
    Minv = unpack_sym(metric_inverse(D6, vscale, tets))[k]            # [R,3,3]
    e = x[tets[k]] - X[:, None, :]                                     # [R,4,3]
    h = np.sqrt(np.einsum("rni,rij,rnj->rn", e, Minv, e))
    return tets[k].reshape(-1), (t[:, None] + h).reshape(-1)


def point_roots_grad(xyz, tets, D6, vscale, root_tet, root_xyz, root_t, g_onset):
    """Chain rule of Eq. (upwind_xi) for a loss with dL/d(onset) = g_onset [4R]
    on the node roots of ``point_roots``.  With e = v_n - x_i and
    h = sqrt(e^T D_eff^-1 e) in element k:
      dL/dt_i  = sum_n g_n,
      dL/dx_i  = sum_n g_n (-D_eff^-1 e / h)          (the gradient of Sec. 2.3),
      dL/dD_k += g_n (-sbar^-2 D^-1 e e^T D^-1 / (2h)),
      dL/dsbar_k += g_n (-h / sbar),  d sbar / d s = 1/4 on the element's nodes.
    A vertex at the point itself (h = 0) contributes to t_i only.
    Returns dict(dt [R], dx [R,3], dD [n_e,6] (off-diagonals doubled), dvscale [n_v])."""
    x = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets)
    n_v = len(x)
    vs = np.ones(n_v) if vscale is None else np.asarray(vscale, dtype=np.float64)
    k = np.asarray(root_tet).reshape(-1)
    R = len(k)
    X = np.asarray(root_xyz, dtype=np.float64).reshape(-1, 3)
    g = np.asarray(g_onset, dtype=np.float64).reshape(R, 4)
    D = unpack_sym(D6)
    Dinv = np.linalg.inv(D[k])                                          # [R,3,3]
    sbar = mean_scale(vs, tets)[k]                                      # [R]
    Minv = Dinv / (sbar ** 2)[:, None, None]
    e = x[tets[k]] - X[:, None, :]                                     # [R,4,3]
    h = np.sqrt(np.einsum("rni,rij,rnj->rn", e, Minv, e))               # [R,4]
    pos = h > 0
    hs = np.where(pos, h, 1.0)
    dx = -np.einsum("rn,rij,rnj->ri", np.where(pos, g / hs, 0.0), Minv, e)
    u = np.einsum("rij,rnj->rni", Dinv, e)                              # D^-1 e
    coef = np.where(pos, g / (sbar[:, None] ** 2 * 2.0 * hs), 0.0)      # [R,4]
    dD = np.zeros((len(tets), 3, 3))
    np.add.at(dD, k, -np.einsum("rn,rni,rnj->rij", coef, u, u))
    dsbar = np.zeros(len(tets))
    np.add.at(dsbar, k, (g * (-h / sbar[:, None])).sum(axis=1))
    dvs = np.zeros(n_v)
    np.add.at(dvs, tets.reshape(-1), np.repeat(dsbar / 4.0, 4))
    dD6 = pack_sym(dD)
    dD6[:, 3:] *= 2.0
    return dict(dt=g.sum(axis=1), dx=dx, dD=dD6, dvscale=dvs)


def point_root_adjoint(xyz, tets, D6, vscale, root_tet, root_xyz, root_t, T, g):
    """Gradients of L = g.T when the roots are points (Eq. (upwind_xi)): the
    adjoint along the geodesic parents down to the node roots of the containing
    elements, then the chain rule of ``point_roots_grad``.
    Returns dict(lam, dD, dvscale, dt, dx)."""
    nodes, onset = point_roots(xyz, tets, D6, vscale, root_tet, root_xyz, root_t)
    a = adjoint(xyz, tets, D6, vscale, nodes, onset, T, g)
    c = point_roots_grad(xyz, tets, D6, vscale, root_tet, root_xyz, root_t, a["droot_t"])
    return dict(lam=a["lam"], dD=a["dD"] + c["dD"], dvscale=a["dvscale"] + c["dvscale"],
                dt=c["dt"], dx=c["dx"])


# --------------------------------------------------------------------------
# lead-field weights (Sec. 2.4)
# --------------------------------------------------------------------------
def p1_stiffness(xyz, tets):
    """P1 stiffness with unit conductivity, K_ab = sum over elements of
    |E| grad(l_a) . grad(l_b): the barycentric functions of an element are
    l = C^-1 [1, x, y, z]^T with C the 4x4 matrix whose columns are
    [1, x_a, y_a, z_a], so their gradients are the last three columns of C^-1."""
    x = np.asarray(xyz, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    n_e = len(tets)
    C = np.ones((n_e, 4, 4))
    C[:, 1:, :] = np.transpose(x[tets], (0, 2, 1))
    Ci = np.linalg.inv(C)                       # row a: coefficients of l_a
    G = Ci[:, :, 1:]                             # [n_e, 4, 3] gradients
    vol = np.abs(np.linalg.det(C)) / 6.0
    Ke = vol[:, None, None] * np.einsum("eai,ebi->eab", G, G)
    rows = np.repeat(tets, 4, axis=1).reshape(-1)
    cols = np.tile(tets, (1, 4)).reshape(-1)
    return sp.csr_matrix((Ke.reshape(-1), (rows, cols)), shape=(len(x), len(x)))


def lead_field(xyz, tets, electrodes):
    """Lead weights B = K Z (Sec. 2.4, with G_i = I): Z[n, l] = 1 / |x_n - e_l|, the
    lead field of a point electrode in an unbounded unit-conductivity medium,
    and K the P1 stiffness.  Returns float64 [n_v, L]."""
    x = np.asarray(xyz, dtype=np.float64)
    e = np.asarray(electrodes, dtype=np.float64).reshape(-1, 3)
    Z = 1.0 / np.linalg.norm(x[:, None, :] - e[None, :, :], axis=2)
    return np.asarray(p1_stiffness(x, tets) @ Z)


# --------------------------------------------------------------------------
# ECG (Sec. 2.4)
# --------------------------------------------------------------------------
def ap_template(xi, K0, K1, tau, **_):
    """Template action potential, Sec. 2.4 Eq. (tanh_waveform) read with
    minimum K0 and maximum K1: U = K0 + (K1-K0)/2 (1 + tanh(2 xi / tau))."""
    return K0 + 0.5 * (K1 - K0) * (1.0 + np.tanh(2.0 * xi / tau))


def ap_template_deriv(xi, K0, K1, tau, **_):
    th = np.tanh(2.0 * xi / tau)
    return 0.5 * (K1 - K0) * (2.0 / tau) * (1.0 - th * th)


def time_grid(ap):
    return ap["t0"] + ap["dt"] * np.arange(ap["n_steps"], dtype=np.float64)


def ecg_forward(T, W, ap, chunk=8192):
    """V_l(t_s) = sum_n B[n,l] U(t_s - phi_n)  (Sec. 2.4), B = W [n_v, L].
    Unreached nodes (phi = +inf) sit at rest (U = K0)."""
    T = np.asarray(T, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    t = time_grid(ap)
    out = np.zeros((len(t), W.shape[1]))
    for a in range(0, len(T), chunk):
        xi = t[:, None] - T[None, a:a + chunk]
        out += ap_template(xi, **ap) @ W[a:a + chunk]
    return out


def ecg_backward(T, W, ap, G, chunk=8192):
    """d/dphi_n of sum_{s,l} G[s,l] V_l(t_s):  - sum_s U'(t_s - phi_n) sum_l G[s,l] B[n,l]."""
    T = np.asarray(T, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    t = time_grid(ap)
    out = np.zeros(len(T))
    for a in range(0, len(T), chunk):
        xi = t[:, None] - T[None, a:a + chunk]
        H = G @ W[a:a + chunk].T                     # [S, chunk]
        out[a:a + chunk] = -(ap_template_deriv(xi, **ap) * H).sum(axis=0)
    return out


def ecg_loss(ecg, target):
    """Eq. (inverse_ecg) with the time integral as a rectangle rule:
    L = 1/(N_leads * S) sum (V - V_hat)^2.  Returns (loss, dL/dV)."""
    e = np.asarray(ecg, dtype=np.float64)
    d = e - np.asarray(target, dtype=np.float64)
    n = d.size
    return float((d * d).sum() / n), 2.0 * d / n


# --------------------------------------------------------------------------
# Alg. 1: FISTA on the local problem (Sec. 2.2)
# --------------------------------------------------------------------------
def simplex_projection(y):
    """Euclidean projection onto {a >= 0, sum a = 1} (sort-based, Duchi et al.)."""
    y = np.asarray(y, dtype=np.float64)
    u = np.sort(y)[::-1]
    css = np.cumsum(u)
    j = np.arange(1, len(y) + 1)
    cond = u - (css - 1.0) / j > 0
    rho = j[cond][-1]
    theta = (css[rho - 1] - 1.0) / rho
    return np.maximum(y - theta, 0.0)


def lipschitz_bound(Q, d=3):
    """Eq. (lipschitz_est): L <= ||A^T A|| / h_ (1 + ||A|| / h_),
    h_ = sigma_min(A) / (d sqrt(d)); with Q = A^T A."""
    ev = np.linalg.eigvalsh(np.asarray(Q, dtype=np.float64))
    h_ = np.sqrt(max(ev[0], 0.0)) / (d * np.sqrt(d))
    return ev[-1] / h_ * (1.0 + np.sqrt(ev[-1]) / h_)


def lipschitz_tight(Q, d=3):
    """Sec. 2.5: h_ from the minimiser at Phi = 0, h_ = h(alpha*)/1.1, then the
    same formula.  (alpha* from the exact local solver.)"""
    ev = np.linalg.eigvalsh(np.asarray(Q, dtype=np.float64))
    _, a, _ = local_solve(Q, np.zeros(3))
    h_ = np.sqrt(a @ Q @ a) / 1.1
    return ev[-1] / h_ * (1.0 + np.sqrt(ev[-1]) / h_)


def fista_local(Q, Phi, L, n_f):
    """Alg. 1: FISTA on <alpha,Phi> + ||A alpha|| over the simplex.
    alpha_hat_0 = 1/d, alpha_0 = alpha_hat_0, beta_k = (k-1)/(k+1).
    Returns (alpha_{n_f}, objective value, per-iteration values)."""
    Q = np.asarray(Q, dtype=np.float64)
    Phi = np.asarray(Phi, dtype=np.float64)
    d = len(Phi)
    a_hat = np.full(d, 1.0 / d)
    a_prev = a_hat.copy()
    hist = []
    a_k = a_hat
    for k in range(1, n_f + 1):
        h = np.sqrt(a_hat @ Q @ a_hat)
        grad = Q @ a_hat / h
        a_tilde = (a_hat - grad / L) - Phi / L
        a_k = simplex_projection(a_tilde)
        beta = (k - 1.0) / (k + 1.0)
        a_hat = a_k + beta * (a_k - a_prev)
        a_prev = a_k
        hist.append(a_k @ Phi + np.sqrt(a_k @ Q @ a_k))
    return a_k, float(a_k @ Phi + np.sqrt(a_k @ Q @ a_k)), np.asarray(hist)


def fista_iterations(L, tau, n_max, d=3):
    """Per-face iteration count from the rate Eq. (fista_convergence), as Sec. 2.5
    suggests (n_f on an element basis): after k iterations from alpha_0 = 1/d the
    error is at most 2 L ||alpha_0 - alpha*||^2 / (k+1)^2, and ||alpha_0 - alpha||^2
    <= (d-1)/d over the simplex (its farthest points from the barycentre are the
    vertices), so the least k >= 1 with (k+1)^2 >= 2 (d-1)/d L / tau guarantees an
    error <= tau whenever L is a Lipschitz constant of grad h.  At most n_max;
    n_max for tau <= 0 or a non-finite bound.  Float64 throughout: the square
    root gives a first guess, then the defining inequality, d tau (k+1)^2 >=
    2 (d-1) L, is checked on the neighbouring integers."""
    L = np.asarray(L, dtype=np.float64)
    out = np.full(L.shape, int(n_max), dtype=np.int64)
    tau = float(tau)
    if not tau > 0:
        return out
    flat_L = L.reshape(-1)
    flat = out.reshape(-1)
    for i, Li in enumerate(flat_L):
        if not np.isfinite(Li):
            continue
        need = 2.0 * (d - 1) * Li               # the bound holds iff d tau (k+1)^2 >= need
        x = np.sqrt(need / (d * tau))
        if not x < n_max + 2:
            continue                           # capped
        k = max(int(np.ceil(x)) - 1, 1)
        while k > 1 and d * tau * float(k) ** 2 >= need:        # k - 1 iterations suffice
            k -= 1
        while d * tau * float(k + 1) ** 2 < need:               # k iterations do not
            k += 1
        flat[i] = min(k, int(n_max))
    return out


# --------------------------------------------------------------------------
# Adam (Sec. 2.4)
# --------------------------------------------------------------------------
def adam_step(p, g, m, v, step, lr=0.5, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), step counted from 1.  Returns (p, m, v)."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

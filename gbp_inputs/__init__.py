"""Seeded synthetic inputs for the Geodesic-BP hot path.

This module only *makes data*: meshes, conduction tensors, activation sites,
velocity-scale fields, electrode positions and lead-field weights.  It holds
none of the method's arithmetic (no local solve, no eikonal iteration, no ECG
contraction), so both the FP64 oracle and the HIP path can consume the same
arrays without sharing any code.

Every generator is deterministic given its seed (numpy PCG64).  Arrays that
feed the solvers are returned in float32 / int32; the oracle upcasts them to
float64 so that both sides solve exactly the same discrete problem.

Conventions
-----------
* ``xyz``   float32 [n_v, 3]        node coordinates
* ``tets``  int32   [n_e, 4]        vertex ids of each tetrahedron
* ``D``     float32 [n_e, 6]        symmetric velocity tensor per tet,
  components (xx, yy, zz, xy, xz, yz); the eikonal cost of a step e inside
  tet j is sqrt(e^T D_j^{-1} e).  (The paper's metric M of its Eq. (1); its
  norm tensor is D_p = M^{-1}, Sec. 2.1.)
* ``W``     float32 [n_v, L]        lead weights, W = K Z_l with K the P1
  stiffness matrix (unit conductivity) and Z_l(x) = 1/|x - e_l| (the
  discretised lead-field operator of Sec. 2.4 with analytic lead fields).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

__all__ = [
    "kuhn_cube", "shell_mesh", "Shell", "mlp_params", "mlp_rows", "MLP_SIZES", "fibre_tensor", "endocardial_nodes",
    "random_roots", "random_point_roots", "tets_touching", "smooth_field", "sphere_electrodes", "lead_weights",
    "jitter_nodes", "Problem", "cube_problem", "shell_problem", "AP_CUBE",
    "AP_SHELL", "tet_volumes", "square_tri", "jitter_nodes2", "fibre_tensor2", "annulus_mesh",
    "circle_electrodes", "lead_weights2", "annulus_problem", "AP_SLICE", "batched_workload",
    "multistart_workload",
]

# Action-potential template parameters (U(xi) = K0 + (K1-K0)*sigmoid(4 xi/tau)
# is the corrected reading of the tanh template, Sec. 2.4).  The shell values
# are the ones the paper uses for its rabbit experiment (Sec. 3.2): K0 = -85 mV,
# K1 = 30 mV, tau = 1 ms.  The cube values give 0.5 (1 + tanh((t - T)/0.5)).
AP_CUBE = dict(K0=0.0, K1=1.0, tau=1.0, t0=0.0, dt=0.01, n_steps=200)
AP_SHELL = dict(K0=-85.0, K1=30.0, tau=1.0, t0=0.0, dt=1.0, n_steps=500)


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
_KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def _kuhn_tets_of_cells(cells_ijk: np.ndarray, node_id) -> np.ndarray:
    """Split each unit cell (lower corner ijk) into the 6 Kuhn tetrahedra
    (0, e_a, e_a+e_b, 1) for every permutation (a, b, c) of the axes.  Using the
    same split in every cell makes the mesh conforming."""
    out = []
    eye = np.eye(3, dtype=np.int64)
    for (a, b, _c) in _KUHN_PERMS:
        p0 = cells_ijk
        p1 = p0 + eye[a]
        p2 = p1 + eye[b]
        p3 = p0 + 1
        out.append(np.stack([node_id(p0), node_id(p1), node_id(p2), node_id(p3)], axis=1))
    t = np.stack(out, axis=1).reshape(-1, 4)
    return t


def kuhn_cube(n_cells: int, length: float = 1.0):
    """Structured tet mesh of the cube [0, length]^3 with n_cells^3 cubes split
    into 6 Kuhn tets each: (n_cells+1)^3 nodes, 6 n_cells^3 tets.  Node id of
    grid point (i, j, k) is i + (n+1) (j + (n+1) k)."""
    n1 = n_cells + 1
    g = np.arange(n1, dtype=np.float64) * (length / n_cells)
    k, j, i = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
    c = np.arange(n_cells)
    ck, cj, ci = np.meshgrid(c, c, c, indexing="ij")
    cells = np.stack([ci.ravel(), cj.ravel(), ck.ravel()], axis=1).astype(np.int64)

    def node_id(p):
        return p[:, 0] + n1 * (p[:, 1] + n1 * p[:, 2])

    tets = _kuhn_tets_of_cells(cells, node_id)
    return xyz.astype(np.float32), tets.astype(np.int32)


def tet_volumes(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    x = np.asarray(xyz, dtype=np.float64)
    a = x[tets[:, 1]] - x[tets[:, 0]]
    b = x[tets[:, 2]] - x[tets[:, 0]]
    c = x[tets[:, 3]] - x[tets[:, 0]]
    return np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0


def jitter_nodes(xyz: np.ndarray, h: float, amp: float, seed: int) -> np.ndarray:
    """Smooth random displacement (sum of a few random sine modes) of relative
    amplitude ``amp`` x h.  Breaks the exact ties of a structured grid while
    keeping every Kuhn tet positively oriented for amp <= 0.15."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.asarray(xyz, dtype=np.float64)
    disp = np.zeros_like(x)
    span = np.ptp(x, axis=0).max()
    for _ in range(6):
        k = rng.normal(size=3)
        k *= (2 * np.pi / span) * rng.uniform(2.0, 6.0) / np.linalg.norm(k)
        ph = rng.uniform(0, 2 * np.pi)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        disp += np.sin(x @ k + ph)[:, None] * d[None, :]
    disp *= amp * h / 6.0 * 2.0
    return (x + disp).astype(np.float32)


@dataclasses.dataclass
class Shell:
    xyz: np.ndarray          # float32 [n_v, 3] (mm)
    tets: np.ndarray         # int32 [n_e, 4]
    h: float                 # grid spacing (mm)
    fibre: np.ndarray        # float32 [n_e, 3] unit fibre direction per tet
    endo: np.ndarray         # int32 node ids on the endocardial surfaces
    radius: float            # max distance of a node from the bbox centre
    node_fibre: np.ndarray = None   # float32 [n_v, 3] the same fibre field at the nodes


# Geometry of the synthetic biventricular shell (mm).  LV: truncated prolate
# ellipsoidal shell; RV: thinner crescent wrapped on the -x side and joined
# to the LV epicardium.
_LV_ENDO = (20.0, 20.0, 45.0)
_LV_EPI = (30.0, 30.0, 52.0)
_RV_C = (-40.0, 0.0, 0.0)
_RV_ENDO = (12.0, 28.0, 40.0)
_RV_EPI = (16.0, 32.0, 43.0)
_Z_BASE = 12.0
_SHELL_VOLUME = 1.0023e5   # mm^3, measured on a 1 mm voxel grid


def _in_ell(p, c, ax):
    return (((p[..., 0] - c[0]) / ax[0]) ** 2 + ((p[..., 1] - c[1]) / ax[1]) ** 2
            + ((p[..., 2] - c[2]) / ax[2]) ** 2) < 1.0


def _shell_mask(p):
    lv_epi = _in_ell(p, (0, 0, 0), _LV_EPI)
    lv_endo = _in_ell(p, (0, 0, 0), _LV_ENDO)
    rv_endo = _in_ell(p, _RV_C, _RV_ENDO)
    rv_epi = _in_ell(p, _RV_C, _RV_EPI)
    myo = (lv_epi & ~lv_endo & ~rv_endo) | (rv_epi & ~rv_endo & ~lv_epi)
    return myo & (p[..., 2] < _Z_BASE)


def _wall_coordinate(p, c, ax_in, ax_out):
    """Transmural coordinate w in [0,1] (0 endo, 1 epi): p lies on the
    ellipsoid whose semi-axes interpolate linearly between the two surfaces.
    Found by bisection (the level function is monotone in w)."""
    lo = np.zeros(len(p))
    hi = np.ones(len(p))
    ai = np.asarray(ax_in)
    ao = np.asarray(ax_out)
    q = p - np.asarray(c)
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        ax = ai[None, :] + mid[:, None] * (ao - ai)[None, :]
        f = ((q / ax) ** 2).sum(axis=1)
        inside = f < 1.0
        hi = np.where(inside, mid, hi)
        lo = np.where(inside, lo, mid)
    return 0.5 * (lo + hi)


def _fibres(p, c, ax_in, ax_out, helix_endo_deg, helix_epi_deg):
    w = _wall_coordinate(p, c, ax_in, ax_out)
    q = p - np.asarray(c)
    ax = np.asarray(ax_in)[None, :] + w[:, None] * (np.asarray(ax_out) - np.asarray(ax_in))[None, :]
    # outward normal of the ellipsoid through q
    nrm = q / ax ** 2
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True) + 1e-30
    circ = np.stack([-q[:, 1], q[:, 0], np.zeros(len(q))], axis=1)
    circ -= (circ * nrm).sum(1, keepdims=True) * nrm
    cn = np.linalg.norm(circ, axis=1, keepdims=True)
    fallback = np.tile(np.array([[1.0, 0.0, 0.0]]), (len(q), 1))
    circ = np.where(cn > 1e-9, circ / np.maximum(cn, 1e-30), fallback)
    long_ = np.cross(nrm, circ)
    long_ /= np.linalg.norm(long_, axis=1, keepdims=True) + 1e-30
    ang = np.deg2rad(helix_endo_deg + (helix_epi_deg - helix_endo_deg) * w)
    f = np.cos(ang)[:, None] * circ + np.sin(ang)[:, None] * long_
    f /= np.linalg.norm(f, axis=1, keepdims=True)
    return f


def shell_mesh(target_nodes: int, seed: int = 2, jitter: float = 0.1) -> Shell:
    """Ellipsoidal biventricular-like shell: masked structured grid of cubes,
    each split into 6 Kuhn tets (conforming), smoothly jittered.  The grid
    spacing is chosen so that the node count is close to ``target_nodes``.
    Fibres rotate linearly from +60 deg (endocardium) to -60 deg
    (epicardium) in the local circumferential/longitudinal frame."""
    h = (_SHELL_VOLUME / (target_nodes / 1.07)) ** (1.0 / 3.0)
    for _ in range(4):
        sh = _shell_grid(h)
        n = sh[0]
        ratio = n / target_nodes
        if abs(ratio - 1.0) < 0.03:
            break
        h *= ratio ** (1.0 / 3.0)
    _, xyz, tets, cell_centres = sh
    # tet centroids (before jitter) carry the fibre field
    cen = xyz[tets].mean(axis=1)
    lv_side = _in_ell(cen, (0, 0, 0), tuple(a * 1.0001 for a in _LV_EPI))
    f = np.empty((len(tets), 3))
    if lv_side.any():
        f[lv_side] = _fibres(cen[lv_side], (0, 0, 0), _LV_ENDO, _LV_EPI, 60.0, -60.0)
    if (~lv_side).any():
        f[~lv_side] = _fibres(cen[~lv_side], _RV_C, _RV_ENDO, _RV_EPI, 60.0, -60.0)
    # endocardial nodes: within 1.5 h of an endocardial surface, inside the wall
    lv_e = _in_ell(xyz, (0, 0, 0), tuple(a + 1.5 * h for a in _LV_ENDO))
    rv_e = _in_ell(xyz, _RV_C, tuple(a + 1.5 * h for a in _RV_ENDO))
    endo = np.nonzero(lv_e | rv_e)[0].astype(np.int32)
    centre = 0.5 * (xyz.min(0) + xyz.max(0))
    radius = float(np.linalg.norm(xyz - centre, axis=1).max())
    lv_n = _in_ell(xyz, (0, 0, 0), tuple(a * 1.0001 for a in _LV_EPI))
    fn = np.empty((len(xyz), 3))
    if lv_n.any():
        fn[lv_n] = _fibres(xyz[lv_n], (0, 0, 0), _LV_ENDO, _LV_EPI, 60.0, -60.0)
    if (~lv_n).any():
        fn[~lv_n] = _fibres(xyz[~lv_n], _RV_C, _RV_ENDO, _RV_EPI, 60.0, -60.0)
    xyz_j = jitter_nodes(xyz, h, jitter, seed) if jitter > 0 else xyz.astype(np.float32)
    return Shell(xyz=xyz_j, tets=tets.astype(np.int32), h=float(h),
                 fibre=f.astype(np.float32), endo=endo, radius=radius,
                 node_fibre=fn.astype(np.float32))


def _shell_grid(h):
    lo = np.array([_RV_C[0] - _RV_EPI[0] - h, -_LV_EPI[1] - h, -_LV_EPI[2] - h])
    hi = np.array([_LV_EPI[0] + h, _LV_EPI[1] + h, _Z_BASE + h])
    n = np.ceil((hi - lo) / h).astype(np.int64)
    ci = np.arange(n[0])
    cj = np.arange(n[1])
    ck = np.arange(n[2])
    K, J, I = np.meshgrid(ck, cj, ci, indexing="ij")
    cells = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    centres = lo[None, :] + (cells + 0.5) * h
    keep = _shell_mask(centres)
    cells = cells[keep]
    n1 = n + 1

    def gid(p):
        return p[:, 0] + n1[0] * (p[:, 1] + n1[1] * p[:, 2])

    tets_g = _kuhn_tets_of_cells(cells, gid)
    used, inv = np.unique(tets_g.ravel(), return_inverse=True)
    tets = inv.reshape(-1, 4)
    gi = used % n1[0]
    gj = (used // n1[0]) % n1[1]
    gk = used // (n1[0] * n1[1])
    xyz = lo[None, :] + np.stack([gi, gj, gk], axis=1) * h
    return len(used), xyz, tets, centres[keep]


def fibre_tensor(fibre: np.ndarray, v_fibre: float = 0.6, v_cross: float = 0.3) -> np.ndarray:
    """Velocity tensor D = v_c^2 I + (v_f^2 - v_c^2) f f^T (i.e.
    diag(v_f^2, v_c^2, v_c^2) in the fibre frame), packed (xx,yy,zz,xy,xz,yz)."""
    f = np.asarray(fibre, dtype=np.float64)
    c2 = v_cross ** 2
    d2 = v_fibre ** 2 - c2
    D = np.empty((len(f), 6))
    D[:, 0] = c2 + d2 * f[:, 0] * f[:, 0]
    D[:, 1] = c2 + d2 * f[:, 1] * f[:, 1]
    D[:, 2] = c2 + d2 * f[:, 2] * f[:, 2]
    D[:, 3] = d2 * f[:, 0] * f[:, 1]
    D[:, 4] = d2 * f[:, 0] * f[:, 2]
    D[:, 5] = d2 * f[:, 1] * f[:, 2]
    return D.astype(np.float32)


def endocardial_nodes(shell: Shell) -> np.ndarray:
    return shell.endo


def random_roots(candidates: np.ndarray, n_roots: int, t_lo: float, t_hi: float, seed: int):
    """n_roots distinct nodes drawn uniformly from ``candidates`` with onset
    times t ~ U[t_lo, t_hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nodes = rng.choice(np.asarray(candidates), size=n_roots, replace=False)
    t = rng.uniform(t_lo, t_hi, size=n_roots)
    return nodes.astype(np.int32), t.astype(np.float32)


def random_point_roots(xyz: np.ndarray, tets: np.ndarray, candidate_tets: np.ndarray, n_roots: int,
                       t_lo: float, t_hi: float, seed: int):
    """Activation sites at points inside elements: n_roots distinct elements
    drawn from ``candidate_tets``, a point in each with uniform random
    barycentric coordinates (Dirichlet(1,1,1,1)), onsets t ~ U[t_lo, t_hi].
    Returns (root_tet int32 [R], root_xyz float32 [R,3], root_t float32 [R])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = rng.choice(np.asarray(candidate_tets), size=n_roots, replace=False)
    w = rng.dirichlet(np.ones(4), size=n_roots)
    p = np.einsum("rn,rni->ri", w, np.asarray(xyz, dtype=np.float64)[np.asarray(tets)[k]])
    t = rng.uniform(t_lo, t_hi, size=n_roots)
    return k.astype(np.int32), p.astype(np.float32), t.astype(np.float32)


def tets_touching(tets: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    """Indices of the elements with at least one vertex in ``nodes``."""
    mark = np.zeros(int(np.asarray(tets).max()) + 1, bool)
    mark[np.asarray(nodes)] = True
    return np.nonzero(mark[np.asarray(tets)].any(axis=1))[0].astype(np.int32)


def smooth_field(xyz: np.ndarray, lo: float, hi: float, seed: int, n_modes: int = 8) -> np.ndarray:
    """Smooth random scalar field with values in [lo, hi] (random sine modes,
    rescaled to the interval)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.asarray(xyz, dtype=np.float64)
    span = max(np.ptp(x, axis=0).max(), 1e-12)
    f = np.zeros(len(x))
    for _ in range(n_modes):
        k = rng.normal(size=3)
        k *= (2 * np.pi / span) * rng.uniform(0.5, 3.0) / np.linalg.norm(k)
        f += rng.normal() * np.sin(x @ k + rng.uniform(0, 2 * np.pi))
    f = (f - f.min()) / max(np.ptp(f), 1e-30)
    return (lo + (hi - lo) * f).astype(np.float32)


def sphere_electrodes(centre, radius: float, n: int, seed: int) -> np.ndarray:
    """n points uniform on a sphere (normalised Gaussian draws)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.normal(size=(n, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return (np.asarray(centre, dtype=np.float64)[None, :] + radius * g)


def stiffness_matrix(xyz: np.ndarray, tets: np.ndarray) -> sp.csr_matrix:
    """P1 stiffness matrix with unit conductivity, K_ab = sum_T |T| grad l_a . grad l_b."""
    x = np.asarray(xyz, dtype=np.float64)
    t = np.asarray(tets, dtype=np.int64)
    P = x[t]                                     # [n_e,4,3]
    E = P[:, 1:, :] - P[:, :1, :]                # rows: edges from vertex 0
    det = np.linalg.det(E)
    vol = np.abs(det) / 6.0
    Einv = np.linalg.inv(E)                      # columns: grads of l1..l3
    g123 = np.transpose(Einv, (0, 2, 1))         # [n_e,3,3] grad of l1,l2,l3
    g0 = -g123.sum(axis=1, keepdims=True)
    G = np.concatenate([g0, g123], axis=1)       # [n_e,4,3]
    Ke = vol[:, None, None] * np.einsum("eai,ebi->eab", G, G)
    rows = np.repeat(t, 4, axis=1).ravel()
    cols = np.tile(t, (1, 4)).ravel()
    n = len(x)
    return sp.csr_matrix((Ke.ravel(), (rows, cols)), shape=(n, n))


def lead_weights(xyz: np.ndarray, tets: np.ndarray, electrodes: np.ndarray) -> np.ndarray:
    """W[:, l] = K Z_l with Z_l(x) = 1/|x - e_l| (analytic lead fields, unit
    conductivity, no Wilson terminal).  Assembled in float64, returned float32.
    Column sums vanish up to rounding because K 1 = 0."""
    x = np.asarray(xyz, dtype=np.float64)
    K = stiffness_matrix(x, tets)
    Z = 1.0 / np.linalg.norm(x[:, None, :] - electrodes[None, :, :], axis=2)
    return np.asarray(K @ Z).astype(np.float32)


# --------------------------------------------------------------------------
# triangle meshes (d = 2)
# --------------------------------------------------------------------------
def square_tri(n_cells: int, length: float = 1.0):
    """Structured triangle mesh of the square [0, length]^2: n_cells^2 cells,
    each split along its (i, j)-(i+1, j+1) diagonal into two counter-clockwise
    triangles.  Node id of grid point (i, j) is i + (n+1) j."""
    n1 = n_cells + 1
    g = np.arange(n1, dtype=np.float64) * (length / n_cells)
    j, i = np.meshgrid(g, g, indexing="ij")
    xy = np.stack([i.ravel(), j.ravel()], axis=1)
    c = np.arange(n_cells)
    cj, ci = np.meshgrid(c, c, indexing="ij")
    a = (ci + n1 * cj).ravel()
    b, d, e = a + 1, a + 1 + n1, a + n1
    tris = np.concatenate([np.stack([a, b, d], 1), np.stack([a, d, e], 1)])
    return xy.astype(np.float32), tris.astype(np.int32)


def jitter_nodes2(xy: np.ndarray, h: float, amp: float, seed: int) -> np.ndarray:
    """Smooth random 2-D displacement of relative amplitude ``amp`` x h (random
    sine modes), as ``jitter_nodes`` in the plane."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.asarray(xy, dtype=np.float64)
    disp = np.zeros_like(x)
    span = np.ptp(x, axis=0).max()
    for _ in range(6):
        k = rng.normal(size=2)
        k *= (2 * np.pi / span) * rng.uniform(2.0, 6.0) / np.linalg.norm(k)
        ph = rng.uniform(0, 2 * np.pi)
        d = rng.normal(size=2)
        d /= np.linalg.norm(d)
        disp += np.sin(x @ k + ph)[:, None] * d[None, :]
    disp *= amp * h / 6.0 * 2.0
    return (x + disp).astype(np.float32)


def fibre_tensor2(fibre: np.ndarray, v_fibre: float = 0.6, v_cross: float = 0.3) -> np.ndarray:
    """2-D velocity tensor per triangle, packed (xx, yy, xy):
    D = v_cross^2 I + (v_fibre^2 - v_cross^2) f f^T."""
    f = np.asarray(fibre, dtype=np.float64)
    d1, d2 = v_fibre ** 2, v_cross ** 2
    return np.stack([d2 + (d1 - d2) * f[:, 0] ** 2, d2 + (d1 - d2) * f[:, 1] ** 2,
                     (d1 - d2) * f[:, 0] * f[:, 1]], axis=1).astype(np.float32)


def annulus_mesh(target_nodes: int, r_in: float = 20.0, r_out: float = 30.0, seed: int = 5,
                 jitter: float = 0.1):
    """Ring r_in <= r <= r_out (mm), a short-axis slice of a left ventricle: a
    polar grid of n_r x n_theta nodes (periodic in theta, cells of roughly unit
    aspect) split into triangles, smooth node jitter.  Fibres lie in the plane at
    an angle to the circumferential direction rotating linearly from +60 deg at
    the inner (endocardial) to -60 deg at the outer boundary.
    Returns (xy, tris, inner node ids, fibre per triangle, grid spacing)."""
    r_mid = 0.5 * (r_in + r_out)
    ratio = 2 * np.pi * r_mid / (r_out - r_in)
    n_r = max(2, int(round(np.sqrt(target_nodes / ratio))))
    n_t = max(8, int(round(target_nodes / n_r)))
    r = np.linspace(r_in, r_out, n_r)
    th = np.arange(n_t) * (2 * np.pi / n_t)
    R, TH = np.meshgrid(r, th, indexing="ij")
    xy = np.stack([(R * np.cos(TH)).ravel(), (R * np.sin(TH)).ravel()], axis=1)
    h = min(r[1] - r[0], 2 * np.pi * r_in / n_t)
    xy = jitter_nodes2(xy, h, jitter, seed).astype(np.float64)

    def nid(ir, it):
        return ir * n_t + (it % n_t)
    ir, it = np.meshgrid(np.arange(n_r - 1), np.arange(n_t), indexing="ij")
    a, b = nid(ir, it).ravel(), nid(ir, it + 1).ravel()
    c, d = nid(ir + 1, it + 1).ravel(), nid(ir + 1, it).ravel()
    tris = np.concatenate([np.stack([a, c, b], 1), np.stack([a, d, c], 1)])
    # orient counter-clockwise
    P = xy[tris]
    cr = (P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1]) - (P[:, 1, 1] - P[:, 0, 1]) * (P[:, 2, 0] - P[:, 0, 0])
    tris[cr < 0] = tris[cr < 0][:, [0, 2, 1]]
    cen = xy[tris].mean(axis=1)
    rc = np.linalg.norm(cen, axis=1)
    w = np.clip((rc - r_in) / (r_out - r_in), 0, 1)
    ang = np.deg2rad(60.0 - 120.0 * w)
    e_t = np.stack([-cen[:, 1], cen[:, 0]], 1) / rc[:, None]
    e_r = cen / rc[:, None]
    fib = np.cos(ang)[:, None] * e_t + np.sin(ang)[:, None] * e_r
    return (xy.astype(np.float32), tris.astype(np.int32), np.arange(n_t, dtype=np.int32),
            fib.astype(np.float32), float(h))


def circle_electrodes(centre, radius: float, n: int, seed: int) -> np.ndarray:
    """n points at uniform random angles on a circle."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.uniform(0, 2 * np.pi, size=n)
    return np.asarray(centre, dtype=np.float64)[None, :] + radius * np.stack([np.cos(a), np.sin(a)], 1)


def lead_weights2(xy: np.ndarray, tris: np.ndarray, electrodes: np.ndarray) -> np.ndarray:
    """W[:, l] = K Z_l on a triangle mesh (P1 stiffness, unit conductivity,
    Z_l(x) = 1/|x - e_l|).  Assembled in float64, returned float32."""
    x = np.asarray(xy, dtype=np.float64)
    t = np.asarray(tris, dtype=np.int64)
    P = x[t]
    E = P[:, 1:, :] - P[:, :1, :]
    det = E[:, 0, 0] * E[:, 1, 1] - E[:, 0, 1] * E[:, 1, 0]
    area = np.abs(det) / 2.0
    Einv = np.linalg.inv(E)
    g12 = np.transpose(Einv, (0, 2, 1))
    G = np.concatenate([-g12.sum(axis=1, keepdims=True), g12], axis=1)
    Ke = area[:, None, None] * np.einsum("eai,ebi->eab", G, G)
    n = len(x)
    K = sp.csr_matrix((Ke.ravel(), (np.repeat(t, 3, axis=1).ravel(), np.tile(t, (1, 3)).ravel())), shape=(n, n))
    Z = 1.0 / np.linalg.norm(x[:, None, :] - np.asarray(electrodes)[None, :, :], axis=2)
    return np.asarray(K @ Z).astype(np.float32)


AP_SLICE = dict(K0=-85.0, K1=30.0, tau=1.0, t0=0.0, dt=1.0, n_steps=120)


def annulus_problem(target_nodes: int = 2700, seed: int = 5, n_roots: int = 8, n_leads: int = 7,
                    vscale_range=None) -> "Problem":
    """2-D left-ventricular slice (stands in for the paper's 2-D study: ~2,700
    nodes, 8 roots, 7 leads): ``annulus_mesh``, D = diag(0.6^2, 0.3^2) (mm/ms)^2 in
    the fibre frame, roots on the inner boundary with onsets U[0, 20] ms,
    electrodes on a circle of 3x the outer radius, 120 steps of 1 ms."""
    xy, tris, inner, fib, h = annulus_mesh(target_nodes, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    rn = rng.choice(inner, size=n_roots, replace=False).astype(np.int32)
    rt = rng.uniform(0.0, 20.0, size=n_roots).astype(np.float32)
    if vscale_range is None:
        vs = np.ones(len(xy), dtype=np.float32)
    else:
        r2 = np.random.Generator(np.random.PCG64(seed + 2))
        vs = r2.uniform(vscale_range[0], vscale_range[1], size=len(xy)).astype(np.float32)
    el = circle_electrodes(np.zeros(2), 90.0, n_leads, seed + 3)
    return Problem(name=f"annulus{len(xy)}", xyz=xy, tets=tris, D=fibre_tensor2(fib), vscale=vs,
                   root_node=rn, root_t=rt, W=lead_weights2(xy, tris, el), ap=dict(AP_SLICE), h=h,
                   extra=dict(electrodes=el, inner=inner, fibre=fib))


# --------------------------------------------------------------------------
# complete problems
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Problem:
    name: str
    xyz: np.ndarray
    tets: np.ndarray
    D: np.ndarray
    vscale: np.ndarray
    root_node: np.ndarray
    root_t: np.ndarray
    W: np.ndarray
    ap: dict
    h: float
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n_v(self):
        return len(self.xyz)

    @property
    def n_e(self):
        return len(self.tets)


def cube_problem(n_cells: int = 20, seed: int = 1, n_leads: int = 8, jitter: float = 0.0,
                 D=None, vscale=None) -> Problem:
    """Unit-cube Kuhn mesh, isotropic D = I, unit speed, one root at the
    origin corner with T = 0; 8 electrodes on a radius-3 sphere around the
    cube centre; U = 0.5 (1 + tanh((t - T)/0.5)), 200 steps of 0.01."""
    xyz, tets = kuhn_cube(n_cells)
    h = 1.0 / n_cells
    if jitter > 0:
        xyz = jitter_nodes(xyz, h, jitter, seed + 100)
    if D is None:
        D = np.tile(np.array([[1, 1, 1, 0, 0, 0]], dtype=np.float32), (len(tets), 1))
    if vscale is None:
        vscale = np.ones(len(xyz), dtype=np.float32)
    el = sphere_electrodes((0.5, 0.5, 0.5), 3.0, n_leads, seed)
    W = lead_weights(xyz, tets, el)
    nf = np.tile(np.array([[1.0, 0.0, 0.0]], np.float32), (len(xyz), 1))
    return Problem("cube", xyz, tets, np.asarray(D, np.float32), np.asarray(vscale, np.float32),
                   np.array([0], np.int32), np.array([0.0], np.float32), W, dict(AP_CUBE), h,
                   extra=dict(electrodes=el, node_fibre=nf))


def shell_problem(target_nodes: int = 500_000, seed: int = 2, n_roots: int = 5, n_leads: int = 12,
                  vscale_range=None, jitter: float = 0.1) -> Problem:
    """Biventricular-like shell with helix fibres, D = diag(0.6^2, 0.3^2, 0.3^2)
    (mm/ms)^2 in the fibre frame, ``n_roots`` endocardial roots with onsets
    U[0, 20] ms, 12 electrodes on a sphere of 3x the shell radius, S = 500
    steps of 1 ms, K0 = -85, K1 = 30, tau = 1."""
    sh = shell_mesh(target_nodes, seed=seed, jitter=jitter)
    D = fibre_tensor(sh.fibre, 0.6, 0.3)
    rn, rt = random_roots(sh.endo, n_roots, 0.0, 20.0, seed + 1)
    if vscale_range is None:
        vs = np.ones(len(sh.xyz), dtype=np.float32)
    else:
        vs = smooth_field(sh.xyz, vscale_range[0], vscale_range[1], seed + 2)
    centre = 0.5 * (sh.xyz.min(0) + sh.xyz.max(0))
    el = sphere_electrodes(centre, 3.0 * sh.radius, n_leads, seed + 3)
    W = lead_weights(sh.xyz, sh.tets, el)
    return Problem("shell", sh.xyz, sh.tets, D, vs, rn, rt, W, dict(AP_SHELL), sh.h,
                   extra=dict(electrodes=el, endo=sh.endo, fibre=sh.fibre, node_fibre=sh.node_fibre))


@dataclasses.dataclass
class BatchedWorkload:
    """Many uneven meshes and parameter sets solved together.  Instance i uses
    mesh ``meshes[mesh_of[i]]`` with roots ``root_node[i]`` (local vertex ids), a
    hidden velocity scale ``vscale_true[i]`` and onsets ``root_t_true[i]`` that
    make its target ECG, and fit start values ``root_t_start[i]`` (the velocity
    scale starts at 1)."""
    meshes: list
    mesh_of: list
    root_node: list
    root_t_true: list
    root_t_start: list
    vscale_true: list


def batched_workload(n_inst: int = 64, n_meshes: int = 8, seed: int = 31) -> BatchedWorkload:
    """The batched form: ``n_meshes`` shells of seeded sizes in [10k, 200k]
    vertices, each used by n_inst / n_meshes instances (instance i on mesh
    i % n_meshes); per instance 1-8 endocardial roots with onsets U[0, 20] ms, a
    hidden smooth velocity scale in [0.5, 1.5], and start onsets perturbed by
    U[-3, 3] ms."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.sort(rng.integers(10_000, 200_001, size=n_meshes))
    meshes = [shell_problem(int(n), seed=seed + 7 * k, n_roots=1, n_leads=12) for k, n in enumerate(sizes)]
    mesh_of = [i % n_meshes for i in range(n_inst)]
    rns, rts, vst = [], [], []
    for i in range(n_inst):
        m = meshes[mesh_of[i]]
        R = int(rng.integers(1, 9))
        rn, rt = random_roots(m.extra["endo"], R, 0.0, 20.0, seed=seed + 1000 + i)
        rns.append(rn)
        rts.append(rt)
        vst.append(smooth_field(m.xyz, 0.5, 1.5, seed=seed + 2000 + i))
    pert = rng.uniform(-3, 3, size=sum(len(r) for r in rns)).astype(np.float32)
    starts, o = [], 0
    for rt in rts:
        starts.append((rt + pert[o:o + len(rt)]).astype(np.float32))
        o += len(rt)
    return BatchedWorkload(meshes, mesh_of, rns, rts, starts, vst)


def multistart_workload(n_nodes: int = 1_000_000, n_starts: int = 16, n_roots: int = 8, seed: int = 5):
    """The inverse problem: a shell with hidden parameters (a smooth velocity
    scale in [0.5, 1.5] and ``n_roots`` endocardial onsets) whose ECG is the
    target, and ``n_starts`` fit starts (velocity scale 1, onsets U[0, 20] ms).
    Returns (problem, vscale_true, [start onsets])."""
    p = shell_problem(n_nodes, seed=seed, n_roots=n_roots, n_leads=12)
    vs_true = smooth_field(p.xyz, 0.5, 1.5, seed=seed + 10)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    rt0 = [rng.uniform(0.0, 20.0, size=n_roots).astype(np.float32) for _ in range(n_starts)]
    return p, vs_true, rt0


# ---------------------------------------------------------------- warm-start network
MLP_SIZES = (("W1", (256, 16)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)),
             ("W3", (256, 256)), ("b3", (256,)), ("W4", (256, 256)), ("b4", (256,)),
             ("w5", (256,)), ("b5", (1,)))


def mlp_params(seed: int, bias_scale: float = 0.1) -> np.ndarray:
    """Random parameter vector for the 16 -> 4x256 -> 1 network in its flat order
    (W1, b1, ..., W4, b4, w5, b5): He-normal weights (fan-in 15 for W1, whose
    16th column is zero), normal biases of std ``bias_scale``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, shape in MLP_SIZES:
        if name == "W1":
            w = rng.normal(0.0, np.sqrt(2.0 / 15.0), size=shape)
            w[:, 15] = 0.0
        elif name[0] == "W":
            w = rng.normal(0.0, np.sqrt(2.0 / shape[1]), size=shape)
        elif name == "w5":
            w = rng.normal(0.0, np.sqrt(1.0 / 256.0), size=shape)
        else:
            w = rng.normal(0.0, bias_scale, size=shape)
        parts.append(w.ravel())
    return np.concatenate(parts).astype(np.float32)


def mlp_rows(m: int, seed: int, scale: float = 1.0):
    """m random network input rows of 16 bfloat16 numbers (the last one 0):
    normal draws times ``scale`` stored as float32, of which the upper 16 bits
    are kept.  Returns (bit patterns as int16 [m, 16], values as float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = (rng.normal(size=(m, 16)) * scale).astype(np.float32)
    x[:, 15] = 0.0
    bits = (x.view(np.uint32) >> 16).astype(np.uint16)
    vals = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return bits.view(np.int16), vals

"""FP64 reference of the learned warm-start network.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): used by ``tests/`` to
check the bf16 matrix-core kernels; shares no code with the HIP library.

The network is not part of the paper (which solves every forward from scratch);
it maps per-vertex features to a guess of the activation time that seeds the
two-sided warm-started solve.  Parity is pinned by the tests in
``tests/test_oracle_mlp.py``: the forward equals ``torch.nn`` Linear/ReLU layers
in float64, the gradient equals autograd and central differences, and the
features equal hand-computed rows.

Network: 16 -> 256 -> 256 -> 256 -> 256 -> 1, ReLU after each hidden layer.
Everything here is float64 and nothing is rounded to a narrower format: the
library's bf16 storage of weights, features and activations is an error that
the GPU tests bound from the rounding unit of bf16, not something this
reference imitates.  ``forward(..., cache=True)`` and ``loss_and_gradient(...,
cache=True)`` also return the intermediate arrays those bounds are built from,
and the optional ``perturb`` callable lets a test sample the standard model of
rounding error (every stored value times 1 + delta with |delta| <= u): it is
applied to the hidden weights W1..W4 where they are used, to each hidden
activation H_l and to each back-propagated dZ_l.  With ``perturb=None`` (the
default) the network is evaluated exactly in float64.
"""
from __future__ import annotations

import numpy as np

SIZES = (("W1", (256, 16)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)),
         ("W3", (256, 256)), ("b3", (256,)), ("W4", (256, 256)), ("b4", (256,)),
         ("w5", (256,)), ("b5", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(params):
    """Flat parameter vector -> dict of float64 arrays."""
    p = np.asarray(params, dtype=np.float64)
    if p.shape != (N_PARAMS,):
        raise ValueError(f"expected {N_PARAMS} parameters")
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SIZES])


def features(xyz, fibre, vscale, rows, root_xyz, root_t, norm, T=None):
    """Feature rows: (x - c)/len_scale, fibre, the per-root values
    |x - x_r|/len_scale + t_r/time_scale over 8 roots (fewer roots: root 0
    repeated) sorted ascending, vscale, 0.  Returns X [m,16] (and T[rows] /
    time_scale when T is given)."""
    xyz = np.asarray(xyz, np.float64)
    rows = np.arange(len(xyz)) if rows is None else np.asarray(rows)
    cx, cy, cz, ls, ts = (float(v) for v in norm)
    rx = np.asarray(root_xyz, np.float64).reshape(-1, 3)
    rt = np.asarray(root_t, np.float64).ravel()
    R = len(rt)
    if not 1 <= R <= 8:
        raise ValueError("1..8 roots")
    idx = [k if k < R else 0 for k in range(8)]
    x = xyz[rows]
    a = np.stack([np.linalg.norm(x - rx[q], axis=1) / ls + rt[q] / ts for q in idx], axis=1)
    a.sort(axis=1)
    vs = np.ones(len(rows)) if vscale is None else np.asarray(vscale, np.float64)[rows]
    X = np.zeros((len(rows), 16))
    X[:, 0:3] = (x - np.array([cx, cy, cz])) / ls
    X[:, 3:6] = np.asarray(fibre, np.float64)[rows]
    X[:, 6:14] = a
    X[:, 14] = vs
    if T is None:
        return X
    return X, np.asarray(T, np.float64)[rows] / ts


def _keep(name, a):
    return a


def forward(params, X, cache=False, perturb=None):
    """y = w5 . H4 + b5 with H_l = relu(Z_l), Z_l = W_l H_{l-1} + b_l, H_0 = X.
    cache=True returns (y, Z [Z_1..Z_4], H [H_0..H_4])."""
    pt = _keep if perturb is None else perturb
    P = unpack(params)
    H = np.asarray(X, np.float64)
    hs, zs = [H], []
    for l in range(1, 5):
        Z = H @ pt(f"W{l}", P[f"W{l}"]).T + P[f"b{l}"]
        H = pt(f"H{l}", np.maximum(Z, 0.0))
        zs.append(Z)
        hs.append(H)
    y = H @ P["w5"] + P["b5"][0]
    return (y, zs, hs) if cache else y


def loss_and_gradient(params, X, target, cache=False, perturb=None):
    """Mean squared error and its gradient with respect to the flat parameter
    vector (back-propagation through the layers above).  cache=True also
    returns dict(y, Z, H, dy, dZ) with dZ[l-1] the gradient of the loss with
    respect to Z_l."""
    pt = _keep if perturb is None else perturb
    P = unpack(params)
    Wq = {l: pt(f"W{l}", P[f"W{l}"]) for l in range(1, 5)}

    def same_weights(name, a):      # the forward and the backward use one set of weights
        return Wq[int(name[1])] if name.startswith("W") else pt(name, a)

    y, zs, hs = forward(params, X, cache=True, perturb=same_weights)
    t = np.asarray(target, np.float64)
    m = len(t)
    d = y - t
    loss = float(np.mean(d * d))
    dy = 2.0 * d / m
    G = {"w5": hs[4].T @ dy, "b5": np.array([dy.sum()])}
    dZ = pt("dZ4", np.outer(dy, P["w5"]) * (zs[3] > 0))
    dzs = [None] * 4
    for l in range(4, 0, -1):
        dzs[l - 1] = dZ
        G[f"W{l}"] = dZ.T @ hs[l - 1]
        G[f"b{l}"] = dZ.sum(axis=0)
        if l > 1:
            dZ = pt(f"dZ{l - 1}", (dZ @ Wq[l]) * (zs[l - 2] > 0))
    if cache:
        return loss, pack(G), dict(y=y, Z=zs, H=hs, dy=dy, dZ=dzs)
    return loss, pack(G)

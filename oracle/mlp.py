"""FP64 reference of the learned warm-start network.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): used by ``tests/`` to
check the bf16 matrix-core kernels; shares no code with the HIP library.

The network is not part of the paper (which solves every forward from scratch);
it maps per-vertex features to a guess of the activation time that seeds the
two-sided warm-started solve.  Parity is pinned by the tests in
``tests/test_oracle_mlp.py``: the forward equals ``torch.nn`` Linear/ReLU layers
in float64, the gradient equals autograd and central differences, and the bf16
rounding equals torch's float32 -> bfloat16 conversion.

Network: 16 -> 256 -> 256 -> 256 -> 256 -> 1, ReLU after each hidden layer.
With ``bf16=True`` the same quantities are rounded to bfloat16 as in the
library: the hidden weights W1..W4, each hidden activation H_l, and each
back-propagated pre-activation gradient dZ_l; everything else is float64.
"""
from __future__ import annotations

import numpy as np

SIZES = (("W1", (256, 16)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)),
         ("W3", (256, 256)), ("b3", (256,)), ("W4", (256, 256)), ("b4", (256,)),
         ("w5", (256,)), ("b5", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def bf16_round(x):
    """Round float64 values to the nearest bfloat16 value (8 significant bits,
    ties to even); the result is returned as float64.  Subnormal and overflow
    ranges are not handled (no value here comes near them)."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                      # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0), e - 8)   # np.round: half to even


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


def features(xyz, fibre, vscale, rows, root_xyz, root_t, norm, T=None, bf16=True):
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
    if bf16:
        X = bf16_round(X)
    if T is None:
        return X
    return X, np.asarray(T, np.float64)[rows] / ts


def forward(params, X, bf16=True, cache=False):
    """y = w5 . H4 + b5 with H_l = relu(W_l H_{l-1} + b_l), H_0 = X."""
    P = unpack(params)
    H = np.asarray(X, np.float64)
    hs = [H]
    for l in range(1, 5):
        W = P[f"W{l}"]
        if bf16:
            W = bf16_round(W)
        H = np.maximum(H @ W.T + P[f"b{l}"], 0.0)
        if bf16:
            H = bf16_round(H)
        hs.append(H)
    y = H @ P["w5"] + P["b5"][0]
    return (y, hs) if cache else y


def loss_and_gradient(params, X, target, bf16=True):
    """Mean squared error and its gradient with respect to the flat parameter
    vector (back-propagation through the layers above)."""
    P = unpack(params)
    y, hs = forward(params, X, bf16=bf16, cache=True)
    t = np.asarray(target, np.float64)
    m = len(t)
    d = y - t
    loss = float(np.mean(d * d))
    dy = 2.0 * d / m
    G = {"w5": hs[4].T @ dy, "b5": np.array([dy.sum()])}
    dZ = np.outer(dy, P["w5"]) * (hs[4] > 0)
    if bf16:
        dZ = bf16_round(dZ)
    for l in range(4, 0, -1):
        G[f"W{l}"] = dZ.T @ hs[l - 1]
        G[f"b{l}"] = dZ.sum(axis=0)
        if l > 1:
            W = P[f"W{l}"]
            if bf16:
                W = bf16_round(W)
            dZ = (dZ @ W) * (hs[l - 1] > 0)
            if bf16:
                dZ = bf16_round(dZ)
    return loss, pack(G)

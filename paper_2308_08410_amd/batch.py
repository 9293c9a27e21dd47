"""Union meshes for batched solves: many tetrahedral meshes (and their per-vertex
and per-element arrays) concatenated into one, instance by instance.  Index
bookkeeping only; every computation runs in the library's kernels."""
from __future__ import annotations

import numpy as np


def union_mesh(xyzs, tetss):
    """Returns (xyz [sum n_v,3], tets [sum n_e,4] with shifted vertex ids,
    vertex offsets [n+1], element offsets [n+1])."""
    nv = np.array([len(x) for x in xyzs])
    ne = np.array([len(t) for t in tetss])
    voff = np.concatenate([[0], np.cumsum(nv)]).astype(np.int32)
    eoff = np.concatenate([[0], np.cumsum(ne)]).astype(np.int32)
    xyz = np.concatenate([np.asarray(x, np.float32) for x in xyzs], axis=0)
    tets = np.concatenate([np.asarray(t, np.int64) + voff[i] for i, t in enumerate(tetss)], axis=0)
    return xyz, tets.astype(np.int32), voff, eoff


def concat(arrays, dtype=np.float32):
    return np.concatenate([np.asarray(a, dtype) for a in arrays], axis=0)


def shift_roots(root_nodes, voff):
    """Root vertex ids of every instance moved into the union numbering."""
    return np.concatenate([np.asarray(r, np.int64) + voff[i] for i, r in enumerate(root_nodes)]).astype(np.int32)

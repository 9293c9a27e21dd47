"""Writes the oracle's reference values for the batched form and the inverse
problem at their full sizes (calls only gbp_inputs and oracle; the oracle runs on
every host core, which does not change its results):

* batched64_reference.npz -- the 64-instance batched workload (8 shells of
  seeded sizes in [10k, 200k] vertices): for four instances (on the smallest
  mesh, the largest and two others) the target ECG from the hidden parameters,
  and at the fit's start parameters (velocity scale 1, perturbed onsets) the
  activation times, misfit, dL/dT, dL/dvscale and dL/droot_t of one iteration;
* multistart1m_reference.npz -- the inverse problem on the 1M-vertex shell: the
  target ECG and the same quantities for fit start 0.

Vertex arrays are stored at a seeded sample of vertices (all of a mesh's
vertices when it has fewer), with the exact max-norm and L2 norm of the full
gradient arrays.  The velocity-scale gradient jumps where a vertex's two best
parents are within rounding of each other: the oracle's own gradient moves by
~1e-3 (relative) when its activation times are merely rounded to FP32.  So the
script also stores, per sampled vertex, the largest change of that gradient over
six such FP32-level perturbations of the oracle's times (rounding to FP32, and
relative noise of 1e-6 and 4e-6, seeded): the tie envelope.  Takes ~10-20
minutes on 8 cores.

    python tests/golden/make_forms_reference.py [batched|multistart]
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gbp_inputs as gi  # noqa: E402
import oracle as O  # noqa: E402

BATCHED_OUT = os.path.join(HERE, "batched64_reference.npz")
MULTISTART_OUT = os.path.join(HERE, "multistart1m_reference.npz")
BATCHED_INSTANCES = (0, 3, 7, 12)      # meshes 0 (smallest), 3, 7 (largest), 4
SAMPLE = 20_000


def input_hash(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def sample_ids(n, seed):
    if n <= SAMPLE:
        return np.arange(n, dtype=np.int32)
    r = np.random.Generator(np.random.PCG64(seed))
    return np.sort(r.choice(n, size=SAMPLE, replace=False)).astype(np.int32)


def one_iteration(p, vs_true, rt_true, rn, vs0, rt0, tag):
    """Oracle values of one Geodesic-BP iteration at the start parameters."""
    t = time.time()
    T_true, st1 = O.solve(p.xyz, p.tets, p.D, vs_true, rn, rt_true)
    target = O.ecg_forward(T_true, p.W, p.ap)
    T0, st0 = O.solve(p.xyz, p.tets, p.D, vs0, rn, rt0)
    ecg0 = O.ecg_forward(T0, p.W, p.ap)
    loss, G = O.ecg_loss(ecg0, target)
    gT = O.ecg_backward(T0, p.W, p.ap, G)
    res = O.adjoint(p.xyz, p.tets, p.D, vs0, rn, rt0, T0, gT)
    # the tie envelope: the gradient's change under FP32-level perturbations of T
    env = np.zeros(p.n_v)
    r = np.random.Generator(np.random.PCG64(77))
    perturbed = [T0.astype(np.float32).astype(np.float64)]
    for amp in (1e-6, 1e-6, 4e-6, 4e-6, 4e-6):
        perturbed.append(T0 * (1.0 + amp * r.uniform(-1.0, 1.0, size=len(T0))))
    for Tp in perturbed:
        e = O.ecg_forward(Tp, p.W, p.ap)
        _, Gp = O.ecg_loss(e, target)
        rp = O.adjoint(p.xyz, p.tets, p.D, vs0, rn, rt0, Tp, O.ecg_backward(Tp, p.W, p.ap, Gp))
        env = np.maximum(env, np.abs(rp["dvscale"] - res["dvscale"]))
    print(f"{tag}: n_v={p.n_v} sweeps {st1['sweeps']}/{st0['sweeps']} {time.time() - t:.1f}s, "
          f"tie envelope {env.max() / np.abs(res['dvscale']).max():.2e} of max", flush=True)
    return dict(target=target, T0=T0, loss=loss, gT=gT, dvscale=res["dvscale"], droot_t=res["droot_t"],
                dvscale_env=env)


def pack(prefix, r, ids, out):
    out[prefix + "ids"] = ids
    out[prefix + "target"] = r["target"].astype(np.float32)
    out[prefix + "T0"] = r["T0"][ids].astype(np.float32)
    out[prefix + "loss"] = np.float64(r["loss"])
    out[prefix + "droot_t"] = r["droot_t"]
    out[prefix + "dvscale_env"] = r["dvscale_env"][ids].astype(np.float32)
    for k in ("gT", "dvscale"):
        out[prefix + k] = r[k][ids].astype(np.float32)
        out[prefix + k + "_max"] = np.abs(r[k]).max()
        out[prefix + k + "_l2"] = np.linalg.norm(r[k])


def batched():
    wl = gi.batched_workload()
    out = {}
    for i in BATCHED_INSTANCES:
        p = wl.meshes[wl.mesh_of[i]]
        r = one_iteration(p, wl.vscale_true[i], wl.root_t_true[i], wl.root_node[i],
                          np.ones(p.n_v), wl.root_t_start[i], f"instance {i}")
        pack(f"i{i}_", r, sample_ids(p.n_v, 100 + i), out)
        out[f"i{i}_hash"] = input_hash(p.xyz, p.tets, p.D, wl.root_node[i], wl.root_t_true[i],
                                       wl.root_t_start[i], wl.vscale_true[i])
    out["instances"] = np.array(BATCHED_INSTANCES, np.int32)
    np.savez_compressed(BATCHED_OUT, **out)
    print(BATCHED_OUT, flush=True)


def multistart():
    p, vs_true, rt0 = gi.multistart_workload()
    r = one_iteration(p, vs_true, p.root_t, p.root_node, np.ones(p.n_v), rt0[0], "start 0")
    out = {}
    pack("s0_", r, sample_ids(p.n_v, 7), out)
    out["hash"] = input_hash(p.xyz, p.tets, p.D, p.root_node, p.root_t, vs_true, rt0[0])
    np.savez_compressed(MULTISTART_OUT, **out)
    print(MULTISTART_OUT, flush=True)


if __name__ == "__main__":
    O.set_threads(os.cpu_count() or 1)
    which = sys.argv[1:] or ["batched", "multistart"]
    if "batched" in which:
        batched()
    if "multistart" in which:
        multistart()

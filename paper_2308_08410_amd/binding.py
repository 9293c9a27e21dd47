"""ctypes binding of libgbp (include/gbp.h).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.  PyTorch supplies
device memory and the current stream.

The library must have been built (``python -m paper_2308_08410_amd.build``);
importing this module without it raises ImportError, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgbp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2308_08410_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

c_int, c_float, c_void_p = ctypes.c_int, ctypes.c_float, ctypes.c_void_p

ERRORS = {
    -1: "GBP_ERR_ARG", -2: "GBP_ERR_DEGENERATE_TET", -3: "GBP_ERR_NOT_SPD", -4: "GBP_ERR_NONFINITE",
    -5: "GBP_ERR_NOT_CONVERGED", -6: "GBP_ERR_HIP", -7: "GBP_ERR_NOMEM",
}


class GbpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Options(ctypes.Structure):
    _fields_ = [("eps_rel", c_float), ("max_rounds", c_int), ("reorder", c_int),
                ("reserved", c_int * 5)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", c_int), ("converged", c_int), ("face_solves", ctypes.c_int64),
                ("node_updates", ctypes.c_int64), ("unreached", c_int), ("reserved", c_int * 3)]

    def as_dict(self):
        return dict(rounds=self.rounds, converged=bool(self.converged), face_solves=self.face_solves,
                    node_updates=self.node_updates, unreached=self.unreached)


class AP(ctypes.Structure):
    _fields_ = [("K0", c_float), ("K1", c_float), ("tau", c_float), ("t0", c_float), ("dt", c_float),
                ("n_steps", c_int)]


def _sig(name, args, res=c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_plan_create = _sig("gbp_plan_create", [c_void_p, c_int, c_void_p, c_int, ctypes.POINTER(Options),
                                        ctypes.POINTER(c_void_p)])
_plan_destroy = _sig("gbp_plan_destroy", [c_void_p], None)
_plan_sizes = _sig("gbp_plan_sizes", [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(c_int)])
_forward = _sig("gbp_eikonal_forward", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                        c_void_p, c_void_p, ctypes.POINTER(Stats), c_void_p])
_backward = _sig("gbp_eikonal_backward", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                          c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p])
_parents = _sig("gbp_parent_map", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_void_p, c_void_p])
_forward_async = _sig("gbp_eikonal_forward_async", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                                    c_void_p, c_void_p, c_int, c_void_p])
_backward_async = _sig("gbp_eikonal_backward_async", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                                      c_int, c_void_p])
_ecg_fwd = _sig("gbp_ecg_forward", [c_void_p, c_int, c_void_p, c_int, ctypes.POINTER(AP), c_void_p,
                                    c_void_p])
_ecg_fwd_noalloc = _sig("gbp_ecg_forward_noalloc", [c_void_p, c_int, c_void_p, c_int, ctypes.POINTER(AP),
                                                      c_void_p, c_void_p])
_ecg_bwd = _sig("gbp_ecg_backward", [c_void_p, c_int, c_void_p, c_int, ctypes.POINTER(AP), c_void_p,
                                     c_void_p, c_void_p])
_ecg_loss = _sig("gbp_ecg_loss", [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p])
_adam = _sig("gbp_adam_step", [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_float, c_float, c_float,
                               c_float, c_int, c_float, c_float, c_void_p])
_bwd_info = _sig("gbp_backward_info", [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                       ctypes.POINTER(c_int)])
_prof_enable = _sig("gbp_profile_enable", [c_int])
_prof_reset = _sig("gbp_profile_reset", [], None)
_prof_read = _sig("gbp_profile_read", [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_double)])
_plan_status = _sig("gbp_plan_status", [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                        ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                        ctypes.POINTER(c_int), c_void_p])
_forward_work = _sig("gbp_plan_forward_work", [c_void_p, c_void_p, c_void_p, c_void_p])
_set_hold = _sig("gbp_plan_set_hold", [c_void_p, c_float, c_int, c_int])
_get_hold = _sig("gbp_plan_get_hold", [c_void_p, ctypes.POINTER(c_float), ctypes.POINTER(c_int),
                                       ctypes.POINTER(c_int)])
_set_warm_order = _sig("gbp_plan_set_warm_order", [c_void_p, c_int])
_get_warm_order = _sig("gbp_plan_get_warm_order", [c_void_p, ctypes.POINTER(c_int)])
_set_launch = _sig("gbp_plan_set_launch", [c_void_p, c_int, c_int, c_int, c_int])
_get_launch = _sig("gbp_plan_get_launch", [c_void_p] + [ctypes.POINTER(c_int)] * 4)
_set_split = _sig("gbp_plan_set_queue_split", [c_void_p, c_int])
_get_split = _sig("gbp_plan_get_queue_split", [c_void_p, ctypes.POINTER(c_int)])
_last_counts = _sig("gbp_plan_last_counts", [c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(c_int)])
_batch_create = _sig("gbp_batch_create", [c_void_p, c_int, c_int, ctypes.POINTER(c_void_p)])
_batch_destroy = _sig("gbp_batch_destroy", [c_void_p], None)
_ecg_fwd_b = _sig("gbp_ecg_forward_batched", [c_void_p, c_void_p, c_void_p, c_int, ctypes.POINTER(AP),
                                              c_void_p, c_void_p])
_ecg_bwd_b = _sig("gbp_ecg_backward_batched", [c_void_p, c_void_p, c_void_p, c_int, ctypes.POINTER(AP),
                                               c_void_p, c_void_p, c_void_p])
_ecg_loss_b = _sig("gbp_ecg_loss_batched", [c_void_p, c_void_p, c_int, c_int, c_void_p, c_void_p,
                                            c_void_p])
_step_create = _sig("gbp_step_create", [c_void_p, ctypes.POINTER(c_void_p)])
_step_launch = _sig("gbp_step_launch", [c_void_p, c_void_p])
_step_destroy = _sig("gbp_step_destroy", [c_void_p], None)
_step_gradients = _sig("gbp_step_gradients", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p])
_step_get_state = _sig("gbp_step_get_state", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                               ctypes.POINTER(c_int), c_void_p])
_step_set_state = _sig("gbp_step_set_state", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                               c_void_p])
_point_roots = _sig("gbp_point_roots", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                        c_void_p, c_void_p, c_void_p])
_point_roots_bwd = _sig("gbp_point_roots_backward", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                                     c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                                     c_void_p])
_locate = _sig("gbp_locate_points", [c_void_p, c_void_p, c_int, c_float, c_void_p, c_void_p])
_set_solver = _sig("gbp_plan_set_local_solver", [c_void_p, c_int, c_int, c_int])
_get_solver = _sig("gbp_plan_get_local_solver", [c_void_p] + [ctypes.POINTER(c_int)] * 3)
_set_reuse = _sig("gbp_plan_set_input_reuse", [c_void_p, c_int])
_set_stamp = _sig("gbp_plan_set_stamp_base", [c_void_p, c_int])
_set_fista_tol = _sig("gbp_plan_set_fista_tolerance", [c_void_p, c_float])
_get_fista_tol = _sig("gbp_plan_get_fista_tolerance", [c_void_p, ctypes.POINTER(c_float)])
_fista_iters = _sig("gbp_fista_iterations", [c_void_p, c_int, c_float, c_int, c_void_p, c_void_p])
_local_solve = _sig("gbp_local_solve", [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, c_int, c_void_p,
                                        c_void_p, c_void_p, c_void_p])
_lead_field = _sig("gbp_lead_field", [c_void_p, c_void_p, c_int, c_void_p, c_void_p])
_tri_create = _sig("gbp_tri_plan_create", [c_void_p, c_int, c_void_p, c_int, ctypes.POINTER(c_void_p)])
_tri_destroy = _sig("gbp_tri_plan_destroy", [c_void_p], None)
_tri_forward = _sig("gbp_tri_forward", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p,
                                        ctypes.POINTER(Stats), c_void_p])
_tri_backward = _sig("gbp_tri_backward", [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p,
                                          c_void_p, c_void_p, c_void_p, c_void_p, c_void_p])
_tri_backward_info = _sig("gbp_tri_backward_info", [c_void_p] + [ctypes.POINTER(c_int)] * 3)
_last_error = _sig("gbp_last_error", [], ctypes.c_char_p)
_version = _sig("gbp_version", [], ctypes.c_char_p)


def version() -> str:
    return _version().decode()


PROFILE_KERNELS = ("metric", "fim_sweep", "parent", "child_lists", "adj_level", "grad", "ecg_fwd",
                   "ecg_bwd", "aux")


def profile_enable(on=True):
    _check(_prof_enable(1 if on else 0))


def profile_reset():
    _prof_reset()


def profile_read():
    """{kernel family: (timed launches, total ms)} from the library's event timers."""
    out = {}
    for k in PROFILE_KERNELS:
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(_prof_read(k.encode(), ctypes.byref(n), ctypes.byref(ms)))
        out[k] = (int(n.value), float(ms.value))
    return out


def _check(rc):
    if rc != 0:
        raise GbpError(rc, _last_error().decode())


def _ptr(t, dtype, shape=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def make_ap(K0, K1, tau, t0, dt, n_steps) -> AP:
    return AP(float(K0), float(K1), float(tau), float(t0), float(dt), int(n_steps))


class Plan:
    """Per-mesh plan (gbp_plan).  xyz float32 [n_v,3], tets int32 [n_e,4] on the host."""

    def __init__(self, xyz, tets, eps_rel=0.0, max_rounds=0, reorder=True):
        xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32))
        tets = np.ascontiguousarray(np.asarray(tets, dtype=np.int32))
        if xyz.ndim != 2 or xyz.shape[1] != 3 or tets.ndim != 2 or tets.shape[1] != 4:
            raise ValueError("xyz must be [n_v,3] and tets [n_e,4]")
        opt = Options(float(eps_rel), int(max_rounds), 0 if reorder else -1)
        h = c_void_p()
        torch.cuda.current_device()
        _check(_plan_create(xyz.ctypes.data, len(xyz), tets.ctypes.data, len(tets), ctypes.byref(opt),
                            ctypes.byref(h)))
        self._h = h
        self.n_v, self.n_e = len(xyz), len(tets)
        self.device = torch.device("cuda", torch.cuda.current_device())

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _plan_destroy is not None:
            _plan_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def eikonal_forward(plan: Plan, D, vscale, root_node, root_t, T_init=None, out=None, stream=None):
    """Returns (T [n_v] float32, stats dict)."""
    n_v, n_e = plan.n_v, plan.n_e
    R = root_node.numel()
    if out is None:
        out = torch.empty(n_v, dtype=torch.float32, device=D.device)
    st = Stats()
    _check(_forward(plan.handle, _ptr(D, torch.float32, (n_e, 6), "D"),
                    _ptr(vscale, torch.float32, (n_v,), "vscale"),
                    _ptr(root_node, torch.int32, (R,), "root_node"),
                    _ptr(root_t, torch.float32, (R,), "root_t"), R,
                    _ptr(T_init, torch.float32, (n_v,), "T_init"),
                    _ptr(out, torch.float32, (n_v,), "T_out"), ctypes.byref(st), _stream(stream)))
    return out, st.as_dict()


def eikonal_backward(plan: Plan, D, vscale, root_node, root_t, T, dL_dT, want_D=True, want_vscale=True,
                     want_root_t=True, stream=None):
    """Returns (dL/dD [n_e,6] or None, dL/dvscale [n_v] or None, dL/droot_t [R] or None)."""
    n_v, n_e = plan.n_v, plan.n_e
    R = root_node.numel()
    dev = T.device
    dD = torch.empty((n_e, 6), dtype=torch.float32, device=dev) if want_D else None
    dvs = torch.empty(n_v, dtype=torch.float32, device=dev) if want_vscale else None
    dt = torch.empty(R, dtype=torch.float32, device=dev) if want_root_t else None
    _check(_backward(plan.handle, _ptr(D, torch.float32, (n_e, 6), "D"),
                     _ptr(vscale, torch.float32, (n_v,), "vscale"),
                     _ptr(root_node, torch.int32, (R,), "root_node"),
                     _ptr(root_t, torch.float32, (R,), "root_t"), R,
                     _ptr(T, torch.float32, (n_v,), "T"), _ptr(dL_dT, torch.float32, (n_v,), "dL_dT"),
                     _ptr(dD, torch.float32, (n_e, 6), "dL_dD"),
                     _ptr(dvs, torch.float32, (n_v,), "dL_dvscale"),
                     _ptr(dt, torch.float32, (R,), "dL_droot_t"), _stream(stream)))
    return dD, dvs, dt


def eikonal_forward_async(plan: Plan, D, vscale, root_node, root_t, round_budget, T_init=None, out=None,
                          stream=None):
    """gbp_eikonal_forward_async: enqueue `round_budget` relaxation rounds, no
    synchronisation; read convergence and input errors with plan_status."""
    n_v, n_e = plan.n_v, plan.n_e
    R = root_node.numel()
    if out is None:
        out = torch.empty(n_v, dtype=torch.float32, device=D.device)
    _check(_forward_async(plan.handle, _ptr(D, torch.float32, (n_e, 6), "D"),
                          _ptr(vscale, torch.float32, (n_v,), "vscale"),
                          _ptr(root_node, torch.int32, (R,), "root_node"),
                          _ptr(root_t, torch.float32, (R,), "root_t"), R,
                          _ptr(T_init, torch.float32, (n_v,), "T_init"),
                          _ptr(out, torch.float32, (n_v,), "T_out"), int(round_budget), _stream(stream)))
    return out


def eikonal_backward_async(plan: Plan, D, vscale, root_node, root_t, T, dL_dT, level_budget, gs_budget=32,
                           want_D=True, want_vscale=True, want_root_t=True, stream=None):
    """gbp_eikonal_backward_async: enqueue the adjoint with fixed budgets, no
    synchronisation.  Returns (dL/dD, dL/dvscale, dL/droot_t) tensors."""
    n_v, n_e = plan.n_v, plan.n_e
    R = root_node.numel()
    dev = T.device
    dD = torch.empty((n_e, 6), dtype=torch.float32, device=dev) if want_D else None
    dvs = torch.empty(n_v, dtype=torch.float32, device=dev) if want_vscale else None
    dt = torch.empty(R, dtype=torch.float32, device=dev) if want_root_t else None
    _check(_backward_async(plan.handle, _ptr(D, torch.float32, (n_e, 6), "D"),
                           _ptr(vscale, torch.float32, (n_v,), "vscale"),
                           _ptr(root_node, torch.int32, (R,), "root_node"),
                           _ptr(root_t, torch.float32, (R,), "root_t"), R,
                           _ptr(T, torch.float32, (n_v,), "T"), _ptr(dL_dT, torch.float32, (n_v,), "dL_dT"),
                           _ptr(dD, torch.float32, (n_e, 6), "dL_dD"),
                           _ptr(dvs, torch.float32, (n_v,), "dL_dvscale"),
                           _ptr(dt, torch.float32, (R,), "dL_droot_t"), int(level_budget), int(gs_budget),
                           _stream(stream)))
    return dD, dvs, dt


def backward_info(plan: Plan):
    """(levels, cyclic vertices, Gauss-Seidel sweeps) of the last backward on ``plan``."""
    a, b, c = c_int(), c_int(), c_int()
    _check(_bwd_info(plan.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return dict(levels=a.value, cyclic=b.value, gs_sweeps=c.value)


def parent_map(plan: Plan, D, vscale, root_node, root_t, T, stream=None):
    """Returns (par_tet [n_v], par_node [n_v,3], par_alpha [n_v,3], best [n_v])."""
    n_v, n_e = plan.n_v, plan.n_e
    R = root_node.numel()
    dev = T.device
    pt = torch.empty(n_v, dtype=torch.int32, device=dev)
    pn = torch.empty((n_v, 3), dtype=torch.int32, device=dev)
    pa = torch.empty((n_v, 3), dtype=torch.float32, device=dev)
    best = torch.empty(n_v, dtype=torch.float32, device=dev)
    _check(_parents(plan.handle, _ptr(D, torch.float32, (n_e, 6), "D"),
                    _ptr(vscale, torch.float32, (n_v,), "vscale"),
                    _ptr(root_node, torch.int32, (R,), "root_node"),
                    _ptr(root_t, torch.float32, (R,), "root_t"), R,
                    _ptr(T, torch.float32, (n_v,), "T"), pt.data_ptr(), pn.data_ptr(), pa.data_ptr(),
                    best.data_ptr(), _stream(stream)))
    return pt, pn, pa, best


class TriPlan:
    """Triangle-mesh plan (gbp_tri_plan, d = 2).  xy float32 [n_v,2], tris int32 [n_t,3] on the host."""

    def __init__(self, xy, tris):
        xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float32))
        tris = np.ascontiguousarray(np.asarray(tris, dtype=np.int32))
        if xy.ndim != 2 or xy.shape[1] != 2 or tris.ndim != 2 or tris.shape[1] != 3:
            raise ValueError("xy must be [n_v,2] and tris [n_t,3]")
        h = c_void_p()
        torch.cuda.current_device()
        _check(_tri_create(xy.ctypes.data, len(xy), tris.ctypes.data, len(tris), ctypes.byref(h)))
        self._h = h
        self.n_v, self.n_t = len(xy), len(tris)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _tri_destroy is not None:
            _tri_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def tri_forward(plan: TriPlan, D, vscale, root_node, root_t, out=None, stream=None):
    """Activation times on a triangle mesh: (T [n_v], stats)."""
    R = root_node.numel()
    if out is None:
        out = torch.empty(plan.n_v, dtype=torch.float32, device=D.device)
    st = Stats()
    _check(_tri_forward(plan.handle, _ptr(D, torch.float32, (plan.n_t, 3), "D"),
                        _ptr(vscale, torch.float32, (plan.n_v,), "vscale"),
                        _ptr(root_node, torch.int32, (R,), "root_node"), _ptr(root_t, torch.float32, (R,), "root_t"),
                        R, _ptr(out, torch.float32, (plan.n_v,), "T_out"), ctypes.byref(st), _stream(stream)))
    return out, st.as_dict()


def tri_backward(plan: TriPlan, D, vscale, root_node, root_t, T, dL_dT, want_D=True, want_vscale=True,
                 want_root_t=True, stream=None):
    """(dL/dD [n_t,3] or None, dL/dvscale [n_v] or None, dL/droot_t [R] or None) on a triangle mesh."""
    R = root_node.numel()
    dev = T.device
    dD = torch.empty((plan.n_t, 3), dtype=torch.float32, device=dev) if want_D else None
    dvs = torch.empty(plan.n_v, dtype=torch.float32, device=dev) if want_vscale else None
    dt = torch.empty(R, dtype=torch.float32, device=dev) if want_root_t else None
    _check(_tri_backward(plan.handle, _ptr(D, torch.float32, (plan.n_t, 3), "D"),
                         _ptr(vscale, torch.float32, (plan.n_v,), "vscale"),
                         _ptr(root_node, torch.int32, (R,), "root_node"), _ptr(root_t, torch.float32, (R,), "root_t"),
                         R, _ptr(T, torch.float32, (plan.n_v,), "T"), _ptr(dL_dT, torch.float32, (plan.n_v,), "dL_dT"),
                         _ptr(dD, torch.float32, (plan.n_t, 3), "dL_dD"),
                         _ptr(dvs, torch.float32, (plan.n_v,), "dL_dvscale"),
                         _ptr(dt, torch.float32, (R,), "dL_droot_t"), _stream(stream)))
    return dD, dvs, dt



def tri_backward_info(plan: TriPlan):
    """The last triangle backward: adjoint levels, vertices left to the Gauss-Seidel
    sweeps by parent-graph cycles, sweeps taken."""
    v = [c_int() for _ in range(3)]
    _check(_tri_backward_info(plan.handle, *[ctypes.byref(x) for x in v]))
    return dict(levels=v[0].value, cyclic=v[1].value, sweeps=v[2].value)

def point_roots(plan: Plan, D, vscale, root_tet, root_xyz, root_t, stream=None):
    """Vertex roots of roots at points inside elements (Sec. 2.3 Eq. (upwind_xi)).
    Returns (node int32 [4R] caller vertex ids, onset float32 [4R])."""
    R = root_tet.numel()
    dev = root_xyz.device
    node = torch.empty(4 * R, dtype=torch.int32, device=dev)
    onset = torch.empty(4 * R, dtype=torch.float32, device=dev)
    _check(_point_roots(plan.handle, _ptr(D, torch.float32, (plan.n_e, 6), "D"),
                        _ptr(vscale, torch.float32, (plan.n_v,), "vscale"),
                        _ptr(root_tet, torch.int32, (R,), "root_tet"),
                        _ptr(root_xyz, torch.float32, (R, 3), "root_xyz"),
                        _ptr(root_t, torch.float32, (R,), "root_t"), R,
                        _ptr(node, torch.int32, (4 * R,), "node_out"),
                        _ptr(onset, torch.float32, (4 * R,), "t_out"), _stream(stream)))
    return node, onset


def point_roots_backward(plan: Plan, D, vscale, root_tet, root_xyz, dL_donset, dL_dD=None, dL_dvscale=None,
                         want_t=True, want_xyz=True, stream=None):
    """Chain rule of ``point_roots``: returns (dL/droot_t [R] or None, dL/droot_xyz [R,3] or None)
    and ADDS the element-tensor and velocity-scale parts into dL_dD / dL_dvscale if given."""
    R = root_tet.numel()
    dev = root_xyz.device
    dt = torch.empty(R, dtype=torch.float32, device=dev) if want_t else None
    dx = torch.empty((R, 3), dtype=torch.float32, device=dev) if want_xyz else None
    _check(_point_roots_bwd(plan.handle, _ptr(D, torch.float32, (plan.n_e, 6), "D"),
                            _ptr(vscale, torch.float32, (plan.n_v,), "vscale"),
                            _ptr(root_tet, torch.int32, (R,), "root_tet"),
                            _ptr(root_xyz, torch.float32, (R, 3), "root_xyz"), R,
                            _ptr(dL_donset, torch.float32, (4 * R,), "dL_donset"),
                            _ptr(dt, torch.float32, (R,), "dL_droot_t"),
                            _ptr(dx, torch.float32, (R, 3), "dL_droot_xyz"),
                            _ptr(dL_dD, torch.float32, (plan.n_e, 6), "dL_dD"),
                            _ptr(dL_dvscale, torch.float32, (plan.n_v,), "dL_dvscale"), _stream(stream)))
    return dt, dx


def locate_points(plan: Plan, points, tol=1e-6, stream=None):
    """Caller element id holding each point (lowest id within barycentric tolerance) or -1."""
    n = points.shape[0]
    out = torch.empty(n, dtype=torch.int32, device=points.device)
    _check(_locate(plan.handle, _ptr(points, torch.float32, (n, 3), "points"), n, float(tol),
                   _ptr(out, torch.int32, (n,), "tet_out"), _stream(stream)))
    return out


def lead_field(plan: Plan, electrodes, out=None, stream=None):
    """Lead weights W = K Z [n_v, L] for point electrodes [L, 3] (Sec. 2.4)."""
    L = electrodes.shape[0]
    if out is None:
        out = torch.empty((plan.n_v, L), dtype=torch.float32, device=electrodes.device)
    _check(_lead_field(plan.handle, _ptr(electrodes, torch.float32, (L, 3), "electrodes"), L,
                       _ptr(out, torch.float32, (plan.n_v, L), "W"), _stream(stream)))
    return out


def ecg_forward(T, W, ap: AP, out=None, stream=None):
    n_v, L = W.shape
    if out is None:
        out = torch.empty((ap.n_steps, L), dtype=torch.float32, device=T.device)
    _check(_ecg_fwd(_ptr(T, torch.float32, (n_v,), "T"), n_v, _ptr(W, torch.float32, (n_v, L), "W"), L,
                    ctypes.byref(ap), _ptr(out, torch.float32, (ap.n_steps, L), "ecg"), _stream(stream)))
    return out


def ecg_forward_noalloc(T, W, ap: AP, out, stream=None):
    """gbp_ecg_forward_noalloc: the ECG into the caller's `out` [n_steps, L], the
    library allocating nothing (its scratch is a fixed array per GPU)."""
    n_v, L = W.shape
    _check(_ecg_fwd_noalloc(_ptr(T, torch.float32, (n_v,), "T"), n_v, _ptr(W, torch.float32, (n_v, L), "W"), L,
                            ctypes.byref(ap), _ptr(out, torch.float32, (ap.n_steps, L), "ecg"),
                            _stream(stream)))
    return out


def ecg_backward(T, W, ap: AP, dL_decg, out=None, stream=None):
    n_v, L = W.shape
    if out is None:
        out = torch.empty(n_v, dtype=torch.float32, device=T.device)
    _check(_ecg_bwd(_ptr(T, torch.float32, (n_v,), "T"), n_v, _ptr(W, torch.float32, (n_v, L), "W"), L,
                    ctypes.byref(ap), _ptr(dL_decg, torch.float32, (ap.n_steps, L), "dL_decg"),
                    _ptr(out, torch.float32, (n_v,), "dL_dT"), _stream(stream)))
    return out


def ecg_loss(ecg, target, grad=True, stream=None):
    n = ecg.numel()
    loss = torch.empty(1, dtype=torch.float32, device=ecg.device)
    g = torch.empty_like(ecg) if grad else None
    _check(_ecg_loss(_ptr(ecg, torch.float32, None, "ecg"), _ptr(target, torch.float32, ecg.shape, "target"),
                     n, loss.data_ptr(), g.data_ptr() if g is not None else None, _stream(stream)))
    return loss, g


def adam_step(param, grad, m, v, step, lr=0.5, beta1=0.9, beta2=0.999, eps=1e-8, lo=0.0, hi=0.0,
              stream=None):
    n = param.numel()
    _check(_adam(_ptr(param, torch.float32, None, "param"), _ptr(grad, torch.float32, param.shape, "grad"),
                 _ptr(m, torch.float32, param.shape, "m"), _ptr(v, torch.float32, param.shape, "v"), n,
                 lr, beta1, beta2, eps, int(step), lo, hi, _stream(stream)))


# ---------------------------------------------------------------- plan control
def plan_status(plan: Plan, stream=None):
    """Synchronises and returns the device-side status of the last call."""
    e, f, b, r, l = c_int(), c_int(), c_int(), c_int(), c_int()
    _check(_plan_status(plan.handle, ctypes.byref(e), ctypes.byref(f), ctypes.byref(b), ctypes.byref(r),
                        ctypes.byref(l), _stream(stream)))
    return dict(err=e.value, forward_converged=bool(f.value), backward_settled=bool(b.value),
                rounds=r.value, levels=l.value)


def forward_work(plan: Plan, stream=None):
    """Synchronises and returns the last forward's work (gbp_plan_forward_work):
    local problems evaluated and vertex value changes."""
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(_forward_work(plan.handle, ctypes.byref(a), ctypes.byref(b), _stream(stream)))
    return dict(face_solves=a.value, node_updates=b.value)


def set_hold(plan: Plan, delta: float, window: int = 0, open_below: int = 0):
    """The cold forward's hold-back (gbp_plan_set_hold): bucket width, buckets past
    the current one that propagate at once, and the queue length below which a
    round opens the next bucket; delta 0 turns it off."""
    _check(_set_hold(plan.handle, float(delta), int(window), int(open_below)))


def get_hold(plan: Plan):
    """(delta, window, open_below)."""
    d, w, o = c_float(), c_int(), c_int()
    _check(_get_hold(plan.handle, ctypes.byref(d), ctypes.byref(w), ctypes.byref(o)))
    return d.value, w.value, o.value


def set_warm_order(plan: Plan, on: bool):
    """gbp_plan_set_warm_order: with on, a forward's T_init only orders the
    hold-back of a cold solve instead of seeding the two-sided update."""
    _check(_set_warm_order(plan.handle, 1 if on else 0))


def get_warm_order(plan: Plan) -> bool:
    v = c_int()
    _check(_get_warm_order(plan.handle, ctypes.byref(v)))
    return bool(v.value)


def set_launch(plan: Plan, lanes=16, sweep_blocks=2048, level_blocks=2048, sync_batch=16):
    _check(_set_launch(plan.handle, lanes, sweep_blocks, level_blocks, sync_batch))


def get_launch(plan: Plan):
    v = [c_int() for _ in range(4)]
    _check(_get_launch(plan.handle, *[ctypes.byref(x) for x in v]))
    return dict(lanes=v[0].value, sweep_blocks=v[1].value, level_blocks=v[2].value, sync_batch=v[3].value)


def set_queue_split(plan: Plan, split=True):
    """Relaxation queue split into 8 XCD sub-queues (True) or one queue (False)."""
    _check(_set_split(plan.handle, 1 if split else 0))


def set_local_solver(plan: Plan, solver="exact", n_f=32, lipschitz="tight"):
    """Local solver of the forward: "exact" (predicated KKT) or "fista" (Alg. 1, n_f
    iterations, step constant from Eq. (lipschitz_est) with the "bound" or the
    "tight" lower bound of h)."""
    s = {"exact": 0, "fista": 1}[solver]
    m = {"bound": 0, "tight": 1}[lipschitz]
    _check(_set_solver(plan.handle, s, int(n_f), m))


def set_stamp_base(plan: Plan, stamp: int):
    """Queue stamp base of the forward (for tests of its restart past 2^30)."""
    _check(_set_stamp(plan.handle, int(stamp)))


def set_input_reuse(plan: Plan, on=True):
    """Allow backward / parent-map calls to keep the element metric, scales and
    onsets built from the same D, vscale, root_node, root_t tensors by the last
    call on this plan; the caller promises those tensors are unchanged since."""
    _check(_set_reuse(plan.handle, 1 if on else 0))


def set_fista_tolerance(plan: Plan, tau: float):
    """Per-face FISTA iterations from the rate Eq. (fista_convergence) for value
    tolerance tau (capped by the n_f of set_local_solver); 0 turns it off."""
    _check(_set_fista_tol(plan.handle, float(tau)))


def get_fista_tolerance(plan: Plan) -> float:
    v = c_float()
    _check(_get_fista_tol(plan.handle, ctypes.byref(v)))
    return v.value


def fista_iterations(lip, tau: float, n_max: int, out=None, stream=None):
    """Per-face FISTA iteration counts for step constants lip [n] (int32 [n])."""
    n = lip.numel()
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=lip.device)
    _check(_fista_iters(_ptr(lip, torch.float32, (n,), "lip"), n, float(tau), int(n_max),
                        _ptr(out, torch.int32, (n,), "n_f"), _stream(stream)))
    return out


def get_local_solver(plan: Plan):
    v = [c_int() for _ in range(3)]
    _check(_get_solver(plan.handle, *[ctypes.byref(x) for x in v]))
    return dict(solver=("exact", "fista")[v[0].value], n_f=v[1].value,
                lipschitz=("bound", "tight")[v[2].value])


def local_solve(Q6, Phi, solver="exact", n_f=32, lip=None, lipschitz="tight", want_alpha=True,
                want_lip=False, stream=None):
    """n independent local problems: returns (value [n], alpha [n,3] or None, lip [n] or None)."""
    n = Q6.shape[0]
    dev = Q6.device
    val = torch.empty(n, dtype=torch.float32, device=dev)
    al = torch.empty((n, 3), dtype=torch.float32, device=dev) if want_alpha else None
    lo = torch.empty(n, dtype=torch.float32, device=dev) if want_lip else None
    _check(_local_solve(_ptr(Q6, torch.float32, (n, 6), "Q6"), _ptr(Phi, torch.float32, (n, 3), "Phi"), n,
                        {"exact": 0, "fista": 1}[solver], int(n_f), _ptr(lip, torch.float32, (n,), "lip"),
                        {"bound": 0, "tight": 1}[lipschitz], _ptr(val, torch.float32, (n,), "value"),
                        _ptr(al, torch.float32, (n, 3), "alpha"), _ptr(lo, torch.float32, (n,), "lip_out"),
                        _stream(stream)))
    return val, al, lo


def get_queue_split(plan: Plan) -> bool:
    v = c_int()
    _check(_get_split(plan.handle, ctypes.byref(v)))
    return bool(v.value)


def last_counts(plan: Plan):
    r, l = c_int(), c_int()
    _check(_last_counts(plan.handle, ctypes.byref(r), ctypes.byref(l)))
    return dict(rounds=r.value, levels=l.value)


# ---------------------------------------------------------------- batches
class Batch:
    """Instance offsets of a union mesh (gbp_batch)."""

    def __init__(self, offsets, max_steps):
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32))
        h = c_void_p()
        _check(_batch_create(off.ctypes.data, len(off) - 1, int(max_steps), ctypes.byref(h)))
        self._h = h
        self.offsets = off
        self.n_inst = len(off) - 1

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _batch_destroy is not None:
            _batch_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def ecg_forward_batched(batch: Batch, T, W, ap: AP, out=None, stream=None):
    n_v, L = W.shape
    if out is None:
        out = torch.empty((batch.n_inst, ap.n_steps, L), dtype=torch.float32, device=T.device)
    _check(_ecg_fwd_b(batch.handle, _ptr(T, torch.float32, (n_v,), "T"), _ptr(W, torch.float32, (n_v, L), "W"),
                      L, ctypes.byref(ap), _ptr(out, torch.float32, (batch.n_inst, ap.n_steps, L), "ecg"),
                      _stream(stream)))
    return out


def ecg_backward_batched(batch: Batch, T, W, ap: AP, dL_decg, out=None, stream=None):
    n_v, L = W.shape
    if out is None:
        out = torch.empty(n_v, dtype=torch.float32, device=T.device)
    _check(_ecg_bwd_b(batch.handle, _ptr(T, torch.float32, (n_v,), "T"), _ptr(W, torch.float32, (n_v, L), "W"),
                      L, ctypes.byref(ap), _ptr(dL_decg, torch.float32, (batch.n_inst, ap.n_steps, L), "dL_decg"),
                      _ptr(out, torch.float32, (n_v,), "dL_dT"), _stream(stream)))
    return out


def ecg_loss_batched(ecg, target, grad=True, stream=None):
    n_inst = ecg.shape[0]
    n_per = ecg[0].numel()
    loss = torch.empty(n_inst, dtype=torch.float32, device=ecg.device)
    g = torch.empty_like(ecg) if grad else None
    _check(_ecg_loss_b(_ptr(ecg, torch.float32, None, "ecg"), _ptr(target, torch.float32, ecg.shape, "target"),
                       n_inst, n_per, loss.data_ptr(), g.data_ptr() if g is not None else None,
                       _stream(stream)))
    return loss, g


# ---------------------------------------------------------------- captured iteration
class StepDesc(ctypes.Structure):
    _fields_ = [("plan", c_void_p), ("batch", c_void_p), ("D", c_void_p), ("vscale", c_void_p),
                ("root_node", c_void_p), ("root_t", c_void_p), ("n_roots", c_int), ("W", c_void_p),
                ("L", c_int), ("ap", AP), ("target", c_void_p), ("T", c_void_p), ("ecg", c_void_p),
                ("loss", c_void_p), ("lr_vscale", c_float), ("lr_root_t", c_float),
                ("vscale_lo", c_float), ("vscale_hi", c_float), ("round_budget", c_int),
                ("level_budget", c_int), ("gs_budget", c_int), ("warm", c_int), ("reserved", c_int * 4)]


class Step:
    """One Geodesic-BP iteration captured in a HIP graph (gbp_step).  The tensors
    passed in are kept referenced for the lifetime of the step."""

    def __init__(self, plan: Plan, batch: Batch, D, vscale, root_node, root_t, W, ap: AP, target, T, ecg,
                 loss, round_budget, level_budget, gs_budget=32, warm=False, lr_vscale=0.01,
                 lr_root_t=0.5, vscale_lo=0.2, vscale_hi=5.0):
        n_v, L = W.shape
        R = root_node.numel()
        self._keep = (plan, batch, D, vscale, root_node, root_t, W, target, T, ecg, loss)
        d = StepDesc()
        d.plan, d.batch = plan.handle, batch.handle
        d.D = _ptr(D, torch.float32, (plan.n_e, 6), "D")
        d.vscale = _ptr(vscale, torch.float32, (n_v,), "vscale")
        d.root_node = _ptr(root_node, torch.int32, (R,), "root_node")
        d.root_t = _ptr(root_t, torch.float32, (R,), "root_t")
        d.n_roots = R
        d.W, d.L, d.ap = _ptr(W, torch.float32, (n_v, L), "W"), L, ap
        d.target = _ptr(target, torch.float32, (batch.n_inst, ap.n_steps, L), "target")
        d.T = _ptr(T, torch.float32, (n_v,), "T")
        d.ecg = _ptr(ecg, torch.float32, (batch.n_inst, ap.n_steps, L), "ecg")
        d.loss = _ptr(loss, torch.float32, (batch.n_inst,), "loss")
        d.lr_vscale, d.lr_root_t, d.vscale_lo, d.vscale_hi = lr_vscale, lr_root_t, vscale_lo, vscale_hi
        d.round_budget, d.level_budget, d.gs_budget = int(round_budget), int(level_budget), int(gs_budget)
        d.warm = 1 if warm else 0
        h = c_void_p()
        _check(_step_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._n_v, self._R, self._dev = n_v, R, T.device

    def launch(self, stream=None):
        _check(_step_launch(self._h, _stream(stream)))

    def gradients(self, stream=None):
        """(dL/dT, dL/dvscale, dL/droot_t) of the last replay, before its Adam
        updates (gbp_step_gradients)."""
        gT = torch.empty(self._n_v, dtype=torch.float32, device=self._dev)
        gv = torch.empty(self._n_v, dtype=torch.float32, device=self._dev)
        gr = torch.empty(max(self._R, 1), dtype=torch.float32, device=self._dev)
        _check(_step_gradients(self._h, gT.data_ptr(), gv.data_ptr(), gr.data_ptr(), _stream(stream)))
        return gT, gv, gr[: self._R]

    def get_state(self, stream=None):
        """The fit's optimiser state (gbp_step_get_state): dict of device tensors
        m_vscale, v_vscale, m_root_t, v_root_t and the int counter."""
        f = lambda n: torch.empty(n, dtype=torch.float32, device=self._dev)
        st = dict(m_vscale=f(self._n_v), v_vscale=f(self._n_v), m_root_t=f(max(self._R, 1)),
                  v_root_t=f(max(self._R, 1)))
        c = c_int()
        _check(_step_get_state(self._h, *[st[k].data_ptr() for k in ("m_vscale", "v_vscale", "m_root_t",
                                                                      "v_root_t")],
                               ctypes.byref(c), _stream(stream)))
        st["m_root_t"], st["v_root_t"] = st["m_root_t"][: self._R], st["v_root_t"][: self._R]
        st["counter"] = c.value
        return st

    def set_state(self, state, stream=None):
        """Restore a state from get_state (tensors or arrays of the same sizes)."""
        t = lambda k, n: torch.as_tensor(np.asarray(state[k].cpu() if torch.is_tensor(state[k]) else state[k],
                                                    np.float32), device=self._dev).reshape(n).contiguous()
        mv, vv = t("m_vscale", self._n_v), t("v_vscale", self._n_v)
        mr, vr = t("m_root_t", self._R), t("v_root_t", self._R)
        _check(_step_set_state(self._h, mv.data_ptr(), vv.data_ptr(), mr.data_ptr() if self._R else None,
                               vr.data_ptr() if self._R else None, int(state["counter"]), _stream(stream)))

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _step_destroy is not None:
            _step_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- learned warm start (MLP)
_mlp_create = _sig("gbp_mlp_create", [c_int, ctypes.c_uint64, ctypes.POINTER(c_void_p)])
_mlp_destroy = _sig("gbp_mlp_destroy", [c_void_p], None)
_mlp_nparams = _sig("gbp_mlp_num_params", [c_void_p])
_mlp_set = _sig("gbp_mlp_set_params", [c_void_p, c_void_p, c_void_p])
_mlp_get = _sig("gbp_mlp_get_params", [c_void_p, c_void_p, c_void_p, c_void_p])
_mlp_get_state = _sig("gbp_mlp_get_state", [c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_int), c_void_p])
_mlp_set_state = _sig("gbp_mlp_set_state", [c_void_p, c_void_p, c_void_p, c_int, c_void_p])
_mlp_features = _sig("gbp_mlp_features", [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p,
                                          c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                          c_void_p])
_mlp_forward = _sig("gbp_mlp_forward", [c_void_p, c_void_p, c_int, c_float, c_void_p, c_void_p])
_mlp_gradient = _sig("gbp_mlp_gradient", [c_void_p, c_void_p, c_int, c_void_p, c_void_p, c_void_p])
_mlp_train = _sig("gbp_mlp_train_step", [c_void_p, c_void_p, c_int, c_void_p, c_float, c_void_p,
                                         c_void_p])

MLP_IN = 16


class MLP:
    """The warm-start network (gbp_mlp): parameters live on the device."""

    def __init__(self, max_rows, seed=0):
        h = c_void_p()
        _check(_mlp_create(int(max_rows), int(seed), ctypes.byref(h)))
        self._h = h
        self.max_rows = int(max_rows)
        self.n_params = _mlp_nparams(h)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _mlp_destroy is not None:
            _mlp_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def get_params(self, grads=False, stream=None):
        p = np.empty(self.n_params, np.float32)
        g = np.empty(self.n_params, np.float32) if grads else None
        _check(_mlp_get(self._h, p.ctypes.data, g.ctypes.data if grads else None, _stream(stream)))
        return (p, g) if grads else p

    def set_params(self, params, stream=None):
        p = np.ascontiguousarray(np.asarray(params, np.float32))
        if p.shape != (self.n_params,):
            raise ValueError(f"params must have shape ({self.n_params},)")
        _check(_mlp_set(self._h, p.ctypes.data, _stream(stream)))

    def get_state(self, stream=None):
        """Adam's moments and step count (gbp_mlp_get_state): dict m, v, step."""
        m = np.empty(self.n_params, np.float32)
        v = np.empty(self.n_params, np.float32)
        k = c_int()
        _check(_mlp_get_state(self._h, m.ctypes.data, v.ctypes.data, ctypes.byref(k), _stream(stream)))
        return dict(m=m, v=v, step=k.value)

    def set_state(self, state, stream=None):
        m = np.ascontiguousarray(np.asarray(state["m"], np.float32))
        v = np.ascontiguousarray(np.asarray(state["v"], np.float32))
        if m.shape != (self.n_params,) or v.shape != (self.n_params,):
            raise ValueError(f"moments must have shape ({self.n_params},)")
        _check(_mlp_set_state(self._h, m.ctypes.data, v.ctypes.data, int(state["step"]), _stream(stream)))

    def forward(self, X, out_scale=1.0, out=None, stream=None):
        m = X.shape[0]
        if out is None:
            out = torch.empty(m, dtype=torch.float32, device=X.device)
        _check(_mlp_forward(self._h, _ptr(X, torch.int16, (m, MLP_IN), "X"), m, float(out_scale),
                            _ptr(out, torch.float32, (m,), "y"), _stream(stream)))
        return out

    def gradient(self, X, target, stream=None):
        m = X.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        _check(_mlp_gradient(self._h, _ptr(X, torch.int16, (m, MLP_IN), "X"), m,
                             _ptr(target, torch.float32, (m,), "target"), loss.data_ptr(), _stream(stream)))
        return loss

    def train_step(self, X, target, lr, loss=None, stream=None):
        m = X.shape[0]
        _check(_mlp_train(self._h, _ptr(X, torch.int16, (m, MLP_IN), "X"), m,
                          _ptr(target, torch.float32, (m,), "target"), float(lr),
                          _ptr(loss, torch.float32, (1,), "loss"), _stream(stream)))


def mlp_features(xyz, fibre, root_xyz, root_t, norm, vscale=None, rows=None, T=None, n_rows=None,
                 stream=None):
    """Feature rows (bf16 bit patterns in an int16 tensor [n_rows, 16]) and, with
    T, the training targets T[rows] / time_scale.  norm = (cx, cy, cz, len_scale,
    time_scale)."""
    n_v = xyz.shape[0]
    R = root_t.numel()
    n = rows.numel() if rows is not None else (n_rows if n_rows is not None else n_v)
    X = torch.empty((n, MLP_IN), dtype=torch.int16, device=xyz.device)
    tgt = torch.empty(n, dtype=torch.float32, device=xyz.device) if T is not None else None
    nrm = np.ascontiguousarray(np.asarray(norm, np.float32))
    if nrm.shape != (5,):
        raise ValueError("norm must hold 5 values")
    _check(_mlp_features(_ptr(xyz, torch.float32, (n_v, 3), "xyz"), _ptr(fibre, torch.float32, (n_v, 3), "fibre"),
                         _ptr(vscale, torch.float32, (n_v,), "vscale"), n_v,
                         _ptr(rows, torch.int32, (n,), "rows"),
                         n, _ptr(root_xyz, torch.float32, (R, 3), "root_xyz"),
                         _ptr(root_t, torch.float32, (R,), "root_t"), R, nrm.ctypes.data,
                         _ptr(T, torch.float32, (n_v,), "T"), X.data_ptr(),
                         tgt.data_ptr() if tgt is not None else None, _stream(stream)))
    return (X, tgt) if T is not None else X

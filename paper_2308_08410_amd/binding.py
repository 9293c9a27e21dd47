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
_ecg_fwd = _sig("gbp_ecg_forward", [c_void_p, c_int, c_void_p, c_int, ctypes.POINTER(AP), c_void_p,
                                    c_void_p])
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


def ecg_forward(T, W, ap: AP, out=None, stream=None):
    n_v, L = W.shape
    if out is None:
        out = torch.empty((ap.n_steps, L), dtype=torch.float32, device=T.device)
    _check(_ecg_fwd(_ptr(T, torch.float32, (n_v,), "T"), n_v, _ptr(W, torch.float32, (n_v, L), "W"), L,
                    ctypes.byref(ap), _ptr(out, torch.float32, (ap.n_steps, L), "ecg"), _stream(stream)))
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

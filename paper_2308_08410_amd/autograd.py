"""torch.autograd.Function wrappers around the library.

``EikonalFn`` replaces the autograd tape that the paper records through every
sweep of Alg. 2 (Sec. 2.3, Sec. 2.5): its forward keeps only the inputs and the
converged activation times; its backward recomputes the geodesic parents from
them (they are never stored) and solves the adjoint system along those parents.
``PointRootsFn`` turns roots at points inside elements into vertex roots
(Sec. 2.3 Eq. (upwind_xi)) and carries their gradient to the points.
``EcgFn`` and ``EcgLossFn`` wrap the lead-field ECG (Sec. 2.4) and the misfit of
Eq. (inverse_ecg).  All arithmetic runs in libgbp's HIP kernels on torch's
current stream.
"""
from __future__ import annotations

import torch

from . import binding as B


class EikonalFn(torch.autograd.Function):
    """T = EikonalFn.apply(plan, D, vscale, root_node, root_t[, T_init]).

    Differentiable w.r.t. D [n_e,6] (off-diagonal gradient entries doubled, the
    packed-symmetric convention of the C ABI), vscale [n_v] and root_t [R]."""

    @staticmethod
    def forward(ctx, plan, D, vscale, root_node, root_t, T_init=None):
        T, stats = B.eikonal_forward(plan, D, vscale, root_node, root_t, T_init=T_init)
        ctx.plan = plan
        ctx.stats = stats
        ctx.save_for_backward(D, vscale, root_node, root_t, T)
        return T

    @staticmethod
    def backward(ctx, gT):
        D, vscale, root_node, root_t, T = ctx.saved_tensors
        need = ctx.needs_input_grad
        dD, dvs, dt = B.eikonal_backward(ctx.plan, D, vscale, root_node, root_t, T, gT.contiguous(),
                                         want_D=need[1], want_vscale=need[2] and vscale is not None,
                                         want_root_t=need[4])
        return None, dD, dvs, None, dt, None


class TriEikonalFn(torch.autograd.Function):
    """T = TriEikonalFn.apply(plan, D, vscale, root_node, root_t) on a triangle mesh
    (d = 2, ``binding.TriPlan``); differentiable w.r.t. D [n_t,3] (off-diagonal
    entries doubled), vscale and root_t, parents recomputed in the backward."""

    @staticmethod
    def forward(ctx, plan, D, vscale, root_node, root_t):
        T, stats = B.tri_forward(plan, D, vscale, root_node, root_t)
        ctx.plan = plan
        ctx.stats = stats
        ctx.save_for_backward(D, vscale, root_node, root_t, T)
        return T

    @staticmethod
    def backward(ctx, gT):
        D, vscale, root_node, root_t, T = ctx.saved_tensors
        need = ctx.needs_input_grad
        dD, dvs, dt = B.tri_backward(ctx.plan, D, vscale, root_node, root_t, T, gT.contiguous(),
                                     want_D=need[1], want_vscale=need[2] and vscale is not None,
                                     want_root_t=need[4])
        return None, dD, dvs, None, dt


class PointRootsFn(torch.autograd.Function):
    """node, onset = PointRootsFn.apply(plan, D, vscale, root_tet, root_xyz, root_t).

    Roots at points inside elements (Sec. 2.3 Eq. (upwind_xi)) as vertex roots
    for ``EikonalFn``; differentiable w.r.t. D, vscale, root_xyz and root_t (the
    gradient w.r.t. the point is the one the paper derives from Eq. (upwind_xi))."""

    @staticmethod
    def forward(ctx, plan, D, vscale, root_tet, root_xyz, root_t):
        node, onset = B.point_roots(plan, D, vscale, root_tet, root_xyz, root_t)
        ctx.plan = plan
        ctx.save_for_backward(D, vscale, root_tet, root_xyz)
        ctx.mark_non_differentiable(node)
        return node, onset

    @staticmethod
    def backward(ctx, g_node, g_onset):
        D, vscale, root_tet, root_xyz = ctx.saved_tensors
        need = ctx.needs_input_grad
        plan = ctx.plan
        dD = torch.zeros((plan.n_e, 6), dtype=torch.float32, device=D.device) if need[1] else None
        dvs = (torch.zeros(plan.n_v, dtype=torch.float32, device=D.device)
               if need[2] and vscale is not None else None)
        if g_onset is None:
            g_onset = torch.zeros(4 * root_tet.numel(), dtype=torch.float32, device=D.device)
        dt, dx = B.point_roots_backward(plan, D, vscale, root_tet, root_xyz, g_onset.contiguous(), dL_dD=dD,
                                        dL_dvscale=dvs, want_t=need[5], want_xyz=need[4])
        return None, dD, dvs, None, dx, dt


class EcgFn(torch.autograd.Function):
    """ecg = EcgFn.apply(T, W, ap): [n_steps, L] lead signals; differentiable w.r.t. T."""

    @staticmethod
    def forward(ctx, T, W, ap):
        ecg = B.ecg_forward(T, W, ap)
        ctx.ap = ap
        ctx.save_for_backward(T, W)
        return ecg

    @staticmethod
    def backward(ctx, g):
        T, W = ctx.saved_tensors
        dT = B.ecg_backward(T, W, ctx.ap, g.contiguous()) if ctx.needs_input_grad[0] else None
        return dT, None, None


class EcgLossFn(torch.autograd.Function):
    """loss = EcgLossFn.apply(ecg, target): mean squared misfit (scalar tensor)."""

    @staticmethod
    def forward(ctx, ecg, target):
        loss, grad = B.ecg_loss(ecg.contiguous(), target.contiguous(), grad=True)
        ctx.save_for_backward(grad)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return grad * g, None


def eikonal(plan, D, vscale, root_node, root_t, T_init=None):
    return EikonalFn.apply(plan, D, vscale, root_node, root_t, T_init)


def tri_eikonal(plan, D, vscale, root_node, root_t):
    return TriEikonalFn.apply(plan, D, vscale, root_node, root_t)


def point_roots(plan, D, vscale, root_tet, root_xyz, root_t):
    return PointRootsFn.apply(plan, D, vscale, root_tet, root_xyz, root_t)


def ecg(T, W, ap):
    return EcgFn.apply(T, W, ap)


def ecg_loss(ecg_signal, target):
    return EcgLossFn.apply(ecg_signal, target)

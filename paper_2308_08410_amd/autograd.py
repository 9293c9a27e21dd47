"""torch.autograd.Function wrappers around the library.

``EikonalFn`` replaces the autograd tape that the paper records through every
sweep of Alg. 2 (Sec. 2.3, Sec. 2.5): its forward keeps only the inputs and the
converged activation times; its backward recomputes the geodesic parents from
them (they are never stored) and solves the adjoint system along those parents.
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


def ecg(T, W, ap):
    return EcgFn.apply(T, W, ap)


def ecg_loss(ecg_signal, target):
    return EcgLossFn.apply(ecg_signal, target)

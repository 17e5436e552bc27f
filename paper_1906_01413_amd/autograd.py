"""PyTorch differentiation of observation maps through the HIP TL/AD kernels.

``observe(x0, handle)`` returns the model's observed values y(x0) = {H_t M_{0->t} x0}
over the assimilation window (Sec. 2.1). Its backward pass (vector-Jacobian product) is
the exact discrete adjoint of the RK4 Lorenz-96 window, and its forward-mode derivative
(jvp) is the tangent-linear model; both run in the library on a trajectory kept only at
every c-th step (c = the handle's ckpt_stride), recomputing one segment at a time. With
these, the 4D-Var cost of eq. 2 and its gradient can be written as ordinary PyTorch code.
"""

from __future__ import annotations

import torch


class _Observe(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, handle):
        ck, obs = handle.ckpt_forward(x0.detach())
        ctx.handle = handle
        ctx.save_for_backward(ck)
        ctx.ck_fwd = ck
        return obs.clone()

    @staticmethod
    def backward(ctx, g_obs):
        (ck,) = ctx.saved_tensors
        gx = ctx.handle.ckpt_adjoint(ck, g_obs.detach().contiguous())
        return gx[:, 0].clone(), None

    @staticmethod
    def jvp(ctx, dx0, _):
        d = ctx.handle.ckpt_tangent(ctx.ck_fwd, dx0.detach().reshape(-1, 1))
        return d[:, 0].clone()


def observe(x0: torch.Tensor, handle) -> torch.Tensor:
    """Observed values of the window started at x0 (differentiable in x0, both modes)."""
    if handle.ckpt_stride <= 0:
        raise ValueError("observe() needs a handle created with ckpt_stride > 0")
    return _Observe.apply(x0, handle)


class _TracerObserve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, s, tracer):
        obs = tracer.forward(s.detach())
        ctx.tracer = tracer
        ctx.version = tracer.base_version
        ctx.save_for_backward(s.detach())
        ctx.s_fwd = s.detach()
        return obs.clone()

    @staticmethod
    def _rebase(ctx, s):
        # the handle linearises at the controls of its latest forward call
        if ctx.tracer.base_version != ctx.version:
            ctx.tracer.forward(s)
            ctx.version = ctx.tracer.base_version

    @staticmethod
    def backward(ctx, g_obs):
        (s,) = ctx.saved_tensors
        _TracerObserve._rebase(ctx, s)
        return ctx.tracer.adjoint(g_obs.detach().contiguous())[:, 0].clone(), None

    @staticmethod
    def jvp(ctx, ds, _):
        _TracerObserve._rebase(ctx, ctx.s_fwd)
        return ctx.tracer.tangent(ds.detach().reshape(-1, 1))[:, 0].clone()


def observe_tracer(s: torch.Tensor, tracer) -> torch.Tensor:
    """Observed concentrations of the tracer model for controls s (differentiable in s:
    backward = the model's adjoint, jvp = its tangent, at s)."""
    return _TracerObserve.apply(s, tracer)

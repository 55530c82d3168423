"""Adjoint form: c(x, pd, qd) as a torch.autograd.Function.

Forward evaluates every constraint row for the given point and load profile;
backward returns J(x)^T lambda (matrix-free, in the HIP kernels) and the load
adjoint d(lambda^T c)/d(pd, qd) = (-lambda_balP, -lambda_balQ): the load
enters the balance rows (Sec. II, eq. (1b)-(1c)) with coefficient -1.  All
tensors are FP64 on the model's device; a batched model evaluates all of its
instances (x, c concatenated; pd, qd concatenated [T*N] blocks).
"""
from __future__ import annotations

import torch

from .capi import Model


class OpfCons(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, pd, qd, model: Model):
        model.use_current_torch_stream()
        x = x.contiguous()
        model.set_load(pd.contiguous(), qd.contiguous())
        c = torch.empty(model.m, dtype=torch.float64, device=x.device)
        model.eval_cons(x, c)
        ctx.save_for_backward(x)
        ctx.model = model
        ctx.load_shape = (pd.shape, qd.shape)
        return c

    @staticmethod
    def backward(ctx, gc):
        (x,) = ctx.saved_tensors
        model: Model = ctx.model
        model.use_current_torch_stream()
        gc = gc.contiguous()
        gx = gpd = gqd = None
        if ctx.needs_input_grad[0]:
            gx = torch.empty(model.n, dtype=torch.float64, device=x.device)
            model.jtprod(x, gc, gx)
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            nload = sum(net.T * net.N for net in model.nets)
            gpd = torch.empty(nload, dtype=torch.float64, device=x.device)
            gqd = torch.empty(nload, dtype=torch.float64, device=x.device)
            model.load_adjoint(gc, gpd, gqd)
            gpd = gpd.reshape(ctx.load_shape[0])
            gqd = gqd.reshape(ctx.load_shape[1])
        return gx, gpd, gqd, None


def opf_cons(x, pd, qd, model: Model):
    """c(x, pd, qd) with the hand-written adjoint."""
    return OpfCons.apply(x, pd, qd, model)

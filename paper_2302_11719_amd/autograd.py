"""Autograd face of the hand-written adjoint rollout kernel.

SmppiRolloutCost.apply(V, ctx, db, model, cost, seed, nominal) returns the
per-sample modified trajectory costs S~ [sum K] (smppi_rollout); its backward
is smppi_rollout_backward with the cost objective, i.e. grad_V = sum_m
grad_S[m] dS~_m/dV (the collision indicator is piecewise constant and
contributes nothing).  Gradients flow to V only; x0 and the noise are inputs.

The forward pass snapshots the start states and iteration counters it used:
a plant step (smppi_execute, or a plan with execute set) advances the batch's
own x0 and counters in place, and the gradient must belong to the costs it
differentiates.
"""
from __future__ import annotations

import torch

from . import core

OBJ_COST = dict(w_S=1.0, w_sq=0.0, w_lin=0.0, n_lin=0)


class SmppiRolloutCost(torch.autograd.Function):
    @staticmethod
    def forward(fctx, V, ctx, db, model, cost, seed, nominal=False):
        Vd = V.detach().contiguous().clone()
        x0 = db.x0.detach().clone()
        iters = db.iter.detach().clone()
        S = core.rollout(ctx, db, model, cost, seed, nominal, V=Vd, x0=x0, iters=iters)
        fctx.save_for_backward(Vd, x0, iters)
        fctx.args = (ctx, db, model, cost, seed, nominal)
        return S

    @staticmethod
    def backward(fctx, grad_S):
        V, x0, iters = fctx.saved_tensors
        ctx, db, model, cost, seed, nominal = fctx.args
        gV = core.rollout_backward(ctx, db, model, cost, seed, grad_S.contiguous(), OBJ_COST, nominal, V=V,
                                   x0=x0, iters=iters)
        return gV, None, None, None, None, None, None

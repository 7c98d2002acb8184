"""Autograd face of the hand-written adjoint rollout kernel.

SmppiRolloutCost.apply(V, ctx, db, model, cost, seed, nominal) returns the
per-sample modified trajectory costs S~ [sum K] (smppi_rollout); its backward
is smppi_rollout_backward with the cost objective, i.e. grad_V = sum_m
grad_S[m] dS~_m/dV (the collision indicator is piecewise constant and
contributes nothing).  Gradients flow to V only; x0 and the noise are inputs.
"""
from __future__ import annotations

import torch

from . import core

OBJ_COST = dict(w_S=1.0, w_sq=0.0, w_lin=0.0, n_lin=0)


class SmppiRolloutCost(torch.autograd.Function):
    @staticmethod
    def forward(fctx, V, ctx, db, model, cost, seed, nominal=False):
        Vd = V.detach().contiguous()
        S = core.rollout(ctx, db, model, cost, seed, nominal, V=Vd)
        fctx.save_for_backward(Vd)
        fctx.args = (ctx, db, model, cost, seed, nominal)
        return S

    @staticmethod
    def backward(fctx, grad_S):
        (V,) = fctx.saved_tensors
        ctx, db, model, cost, seed, nominal = fctx.args
        gV = core.rollout_backward(ctx, db, model, cost, seed, grad_S.contiguous(), OBJ_COST, nominal, V=V)
        return gV, None, None, None, None, None, None

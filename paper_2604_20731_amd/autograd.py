"""Differentiation form: the robust CRVPINN loss as a torch autograd function
of the network parameters and the nodal log-permeability.

Forward: alpha from log K, the network pressure, the residual, the Gram
solve and LOSS = RES . G^-1 RES (eq. 21-28).  Backward: the adjoint field
g_u = 2 A^T q drives the network backward for dLOSS/dtheta, and
dLOSS/dlog K = g_alpha * alpha with g_alpha = 2 h^(d-2) sum_dir
grad+ u . grad+ q (derived from eq. 25 and 27).  Both gradients come out of
the one libcrv call that evaluates the loss; the returned tensors are
scaled by the incoming gradient.

The scenario supplies geometry, wells, saturation and precision; its
training state (Adam moments, step count) is left as it was, its theta and
log K are replaced by the arguments.
"""
from __future__ import annotations

import numpy as np
import torch

from . import crv


class CRVLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta: torch.Tensor, log_perm: torch.Tensor, scenario: crv.Scenario):
        scenario.set_theta(theta.detach().to("cpu", torch.float64).numpy())
        scenario.set_log_perm(log_perm.detach().to("cpu", torch.float64).numpy())
        loss, g, gl = scenario.loss_grad(with_logperm=True)
        ctx.save_for_backward(torch.from_numpy(g).to(theta.device, theta.dtype),
                              torch.from_numpy(gl.reshape(log_perm.shape)).to(
                                  log_perm.device, log_perm.dtype))
        return torch.tensor(loss, dtype=theta.dtype, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        g, gl = ctx.saved_tensors
        return grad_out * g, grad_out * gl, None


def crv_loss(theta: torch.Tensor, log_perm: torch.Tensor, scenario: crv.Scenario) -> torch.Tensor:
    """LOSS(theta, log K) of the scenario, differentiable in both arguments."""
    return CRVLoss.apply(theta, log_perm, scenario)

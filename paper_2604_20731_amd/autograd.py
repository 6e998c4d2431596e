"""Differentiation form: the robust CRVPINN loss as a torch autograd function
of the network parameters and the nodal log-permeability.

Forward: alpha from log K, the network pressure, the residual, the Gram
solve and LOSS = RES . G^-1 RES (eq. 21-28).  Backward: the adjoint field
g_u = 2 A^T q drives the network backward for dLOSS/dtheta, and
dLOSS/dlog K = g_alpha * alpha with g_alpha = 2 h^(d-2) sum_dir
grad+ u . grad+ q (derived from eq. 25 and 27).  Both gradients come out of
the one libcrv call that evaluates the loss; the returned tensors are
scaled by the incoming gradient.  CUDA tensors on a float32 context go
through the device-array calls (no host copy of theta, log K or the
gradients); CPU tensors and float64 contexts through the host-array calls.

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
        if theta.is_cuda and log_perm.is_cuda and scenario.cfg.precision != crv.PREC["fp64"]:
            # CUDA tensors on a float32 context: parameters in and gradients
            # out stay in device memory (crv_set_params_device,
            # crv_loss_grad_device), stream-ordered with no host wait
            scenario.set_params_device(
                theta.detach().to(torch.float32).contiguous().view(-1),
                log_perm.detach().to(torch.float32).contiguous().view(-1))
            loss, g, gl = scenario.loss_grad_device(with_logperm=True)
            ctx.save_for_backward(g.to(theta.dtype).view(theta.shape),
                                  gl.to(log_perm.dtype).view(log_perm.shape))
            return loss.to(theta.dtype)
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

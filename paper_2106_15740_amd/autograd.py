"""torch.autograd.Function over the library's forward + adjoint sweep.

Real inputs (gamma, beta: float64 of length p) and a real output E, so torch's
complex conventions never cross the boundary; the gradient comes from the
hand-written reverse sweep over the buckets.
"""
from __future__ import annotations

import torch

from .net import QaoaNet


class QaoaEnergy(torch.autograd.Function):
    """E(gamma, beta) = <gamma beta| C |gamma beta> with dE/dgamma, dE/dbeta."""

    @staticmethod
    def forward(ctx, gamma: torch.Tensor, beta: torch.Tensor, net: QaoaNet, mode: str = "batched"):
        net.set_params(gamma.detach().cpu().double().numpy(), beta.detach().cpu().double().numpy())
        e, dg, db = net.energy_grad(mode)
        # outputs and saved gradients live where the angles do
        ctx.save_for_backward(torch.from_numpy(dg).to(device=gamma.device, dtype=gamma.dtype),
                              torch.from_numpy(db).to(device=beta.device, dtype=beta.dtype))
        return torch.tensor(e, dtype=torch.float64, device=gamma.device)

    @staticmethod
    def backward(ctx, grad_e):
        dg, db = ctx.saved_tensors
        return grad_e.to(device=dg.device, dtype=dg.dtype) * dg, grad_e.to(device=db.device, dtype=db.dtype) * db, \
            None, None


def qaoa_energy(gamma: torch.Tensor, beta: torch.Tensor, net: QaoaNet, mode: str = "batched") -> torch.Tensor:
    return QaoaEnergy.apply(gamma, beta, net, mode)

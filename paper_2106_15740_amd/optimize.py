"""Classical outer loop of QAOA: choose (gamma, beta) that maximise the
expected cut <C> with a torch optimiser over the library's energy and adjoint
gradient (the use the paper motivates in Section II; the paper itself does not
optimise).  Every energy and gradient evaluation is one batched sweep of the
HIP kernels through QaoaEnergy.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

import torch

from .autograd import qaoa_energy
from .net import QaoaNet


@dataclass
class OptResult:
    gamma: List[float]
    beta: List[float]
    energy: float
    history: List[float] = field(default_factory=list)  # energy before each step


def maximize_cut(net: QaoaNet, gamma0: Sequence[float], beta0: Sequence[float], steps: int = 100,
                 lr: float = 0.05, optimizer: str = "adam", mode: str = "batched") -> OptResult:
    """Gradient ascent on E(gamma, beta) = <gamma beta|C|gamma beta> from
    (gamma0, beta0): `steps` updates of torch's Adam (or plain SGD) on -E."""
    if len(gamma0) != net.p or len(beta0) != net.p:
        raise ValueError(f"gamma0 and beta0 must have length p={net.p}")
    g = torch.tensor(list(gamma0), dtype=torch.float64, requires_grad=True)
    b = torch.tensor(list(beta0), dtype=torch.float64, requires_grad=True)
    if optimizer == "adam":
        opt = torch.optim.Adam([g, b], lr=lr)
    elif optimizer == "sgd":
        opt = torch.optim.SGD([g, b], lr=lr)
    else:
        raise ValueError("optimizer must be 'adam' or 'sgd'")
    hist = []
    for _ in range(int(steps)):
        opt.zero_grad()
        e = qaoa_energy(g, b, net, mode)
        hist.append(float(e.item()))
        (-e).backward()
        opt.step()
    with torch.no_grad():
        e = qaoa_energy(g, b, net, mode)
    return OptResult(gamma=g.detach().tolist(), beta=b.detach().tolist(), energy=float(e.item()), history=hist)

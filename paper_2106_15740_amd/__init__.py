"""MI355X (gfx950) QAOA-MaxCut energy by light-cone tensor-network contraction.

The method follows Lykov & Alexeev, "Importance of Diagonal Gates in Tensor
Network Simulations": each edge term <Z_j Z_k> is a light-cone network in which
the ZZ phase gates are rank-2 diagonal tensors that add no index (Section
IV.B), contracted by bucket elimination (Section III.B).  The contraction, its
adjoint and the reductions run in hand-written HIP kernels behind the C ABI of
include/qtn.h; this package is the Python binding of that library.
"""
from ._lib import QtnError, lib  # noqa: F401
from .net import Context, QaoaAmplitude, QaoaNet, copy_bandwidth  # noqa: F401


def __getattr__(name):
    if name in ("QaoaEnergy", "qaoa_energy"):
        from . import autograd

        return getattr(autograd, name)
    if name in ("maximize_cut", "OptResult"):
        from . import optimize

        return getattr(optimize, name)
    raise AttributeError(name)

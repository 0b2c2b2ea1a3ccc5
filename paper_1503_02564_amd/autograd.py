"""``torch.autograd.Function`` over the SWR solve: forward u0, V -> u(T) with
``swr_solve``; backward by the discrete adjoint through the same
decomposition (``swr_grad``), returning dJ/dV and dJ/du0.

Argument marshalling only: both directions run in the HIP library.  A
status other than SWR_OK (an interface solve that did not converge) raises
SwrError instead of returning the last iterate as a result.
"""
from __future__ import annotations

import torch

from . import swr


class SWRFunction(torch.autograd.Function):
    """uT = SWRFunction.apply(V, u0, problem)

    V: float64 CUDA tensor, [nx] (shared) or [B][nx] (``v_per_problem``);
    u0: complex128 CUDA tensor [B][nx]; problem: a ``swr.Problem`` with a
    static potential (its V is replaced by the argument).  Gradients follow
    PyTorch's convention for complex tensors (dJ/dRe + i dJ/dIm)."""

    @staticmethod
    def forward(ctx, V, u0, problem):
        Vc = V.detach().contiguous()
        u0c = u0.detach().contiguous()
        swr.swr_set_potential(problem.ctx, Vc)
        uT = torch.empty_like(u0c)
        st, info = swr.swr_solve(problem.ctx, u0c, uT)
        if st != swr.SWR_OK:
            # an unconverged interface solve would hand back its last iterate
            raise swr.SwrError(st, f"SWRFunction.forward (residual {info.residual:.3e})")
        ctx.save_for_backward(Vc, u0c)
        ctx.problem = problem
        return uT

    @staticmethod
    def backward(ctx, gbar):
        V, u0 = ctx.saved_tensors
        pb = ctx.problem
        swr.swr_set_potential(pb.ctx, V)
        dV = torch.empty((u0.shape[0], u0.shape[1]), dtype=torch.float64, device=u0.device)
        du0 = torch.empty_like(u0)
        st, info = swr.swr_grad(pb.ctx, u0, gbar.contiguous(), dV, du0)
        if st != swr.SWR_OK:
            raise swr.SwrError(st, f"SWRFunction.backward (adjoint residual {info.residual:.3e})")
        if V.dim() == 1:
            dV = dV.sum(0)
        return dV.reshape(V.shape), du0, None


def swr_forward(V, u0, problem):
    return SWRFunction.apply(V, u0, problem)

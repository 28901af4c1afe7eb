"""The pseudofermion action as a differentiable torch function.

S(phi) = sum_k chi_k^dagger (M[phi]^dagger M[phi])^{-1} chi_k (Eq. 21), with chi held fixed
(the Gibbs step of Methods D refreshes it separately).  forward runs the library's CG
solve and reduction; backward runs the library's hand-written gradient kernel
(dS/dphi = -2 Re Y^dagger (dM/dphi) x with Y = M x).  By default the CG solution is not
kept between forward and backward: backward solves again (memory policy "recompute");
policy "store" keeps x, one complex128 spinor per pseudofermion.
"""
import torch

from ._lib import HMC_FORCE_PF


class PseudofermionAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, chi, hmc, store_solution=False):
        x = torch.empty_like(chi) if store_solution else None
        S, st = hmc.pf_action(phi, chi, x=x)
        ctx.hmc = hmc
        ctx.cg_stats = st
        if store_solution:
            ctx.save_for_backward(phi, chi, x)
        else:
            ctx.save_for_backward(phi, chi)
        return torch.tensor(S, dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(ctx, grad_out):
        saved = ctx.saved_tensors
        hmc = ctx.hmc
        if len(saved) == 3:
            phi, _, x = saved
            F = hmc.force_from_solution(phi, x, flags=HMC_FORCE_PF)
        else:
            phi, chi = saved
            F, _, _ = hmc.force(phi, chi, flags=HMC_FORCE_PF)
        return grad_out * F, None, None, None


def pf_action(phi, chi, hmc, store_solution=False):
    """Differentiable S_PF(phi) for fixed pseudofermions chi (complex128 spinors)."""
    return PseudofermionAction.apply(phi, chi, hmc, store_solution)

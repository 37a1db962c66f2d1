"""torch.autograd.Function wrapper of the pseudo-fermion action (binding layer: the action
and its gradient are computed by the library's kernels).

The action is taken as a function of su(3) link momenta omega (sap momentum layout):
U(omega) = exp(i omega) U0, S(omega) = ||W1^{-1} phi1||^2 + ||R_hat^{-1} chi||^2 on U(omega)
(Sec. 1). The forward pass sets the context's gauge field to U(omega) and evaluates S; the
backward pass returns the library's force F^a = dS/dw^a along U -> exp(i w T^a) U(omega),
which is the gradient dS/d omega at omega = 0 (the molecular-dynamics force of Sec. 2).
At omega != 0 it is the derivative along the left-invariant directions at U(omega).
"""
import torch

from . import block_pf_force, schwarz_boundary_force, sap_update_links


class PseudoFermionAction(torch.autograd.Function):
    @staticmethod
    def forward(actx, omega, sctx, U0, phi1, chi, opts):
        sctx.set_gauge(U0)
        sap_update_links(sctx, omega, 1.0)
        F = sctx.new_momenta()
        S = 0.0
        if phi1 is not None:
            S += block_pf_force(sctx, F, 1.0, phi1, opts)
        if chi is not None:
            S += schwarz_boundary_force(sctx, F, 1.0, chi, opts)
        actx.save_for_backward(F)
        return torch.tensor(S, dtype=torch.float64, device=omega.device)

    @staticmethod
    def backward(actx, grad):
        (F,) = actx.saved_tensors
        return grad * F, None, None, None, None, None


def pseudo_fermion_action(omega, sctx, U0, phi1=None, chi=None, opts=None):
    """S_pf(U(omega)) with the gradient of ``PseudoFermionAction``; phi1 and chi are FP64
    fields in the sap layout (either may be None), U0 the canonical gauge field."""
    return PseudoFermionAction.apply(omega, sctx, U0, phi1, chi, opts)

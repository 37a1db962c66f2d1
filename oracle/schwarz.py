"""Schwarz boundary operator on the black-block boundaries (oracle, FP64).

Sec. 1 (Schwarz preconditioning, following Luescher): with the x0 blocks coloured
red/black, det^2(W1^{-1} M) is represented by a pseudo-fermion field living on the
boundaries of the black blocks only, and the field dimension is halved by a spin
projection (Luescher's Appendix B, used by the paper without change). The paper does
not print these formulas; the oracle writes out the reading below, whose determinant
identity det M = det W1 * det R_hat is pinned densely by the tests.

Notation (Omega = black blocks, Omega* = white blocks, P_X = restriction to X):
    D_Om     = P_Om W1 P_Om          D_Om*     = P_Om* W1 P_Om*
    D_dOm    = P_Om M P_Om*          D_dOm*    = P_Om* M P_Om
A black block's first slice (x0 = 0 mod l0) couples to the white slice before it only
through the spin components selected by (1 - gamma_0)/2, its last slice
(x0 = l0-1 mod l0) only through (1 + gamma_0)/2 (one crossing direction per site: the
decomposition is one-dimensional, so no block corners). Pi is that projector, zero
elsewhere, and
    R_hat       = Pi - Pi D_Om^{-1} D_dOm D_Om*^{-1} D_dOm* Pi        (on range Pi),
    R_hat^{-1}  = Pi - Pi M^{-1} D_dOm* Pi,
    S_R(chi)    = || R_hat^{-1} chi ||^2,   heat bath  chi = R_hat Pi g,  g ~ exp(-|g|^2).
The inverse follows from the 2x2 block inverse of M in the (Omega, Omega*) partition.

Iterated decomposition (Sec. 1, end: the factor det^2(W1 W2^{-1}) of the four-part
action): every function takes ``outer``, the block length of the operator that plays the
role of M (None: M itself). With outer = l0^(1) and l0 = l0^(2) the same formulas give
det W1 = det W2 * det R_hat_2; then a black sub-block slice next to a level-1 block
boundary has no crossing hop in W1, and Pi keeps only the components whose crossing hop
exists in the outer operator (one interface per level-1 block).
"""
import numpy as np

from .gamma import ONE4, GAMMA, spin_mul
from .lattice import coords, block_of_x0, site_mask, colour_x0_mask
from .dirac import apply_op
from . import solvers


def black_white_masks(L, l0):
    return (site_mask(L, colour_x0_mask(L, l0, "black")),
            site_mask(L, colour_x0_mask(L, l0, "white")))


def boundary_slices(L, l0, outer=None):
    """Boolean masks (shape L) of the first and last slice of every black block whose
    crossing hop (backward from the first, forward from the last slice) exists in the
    outer operator (M for outer None, else W_outer)."""
    x0 = coords(L)[0]
    black = (block_of_x0(x0, l0) % 2) == 1
    first = black & (x0 % l0 == 0)
    last = black & (x0 % l0 == l0 - 1)
    if outer is not None:
        first = first & (x0 % outer != 0)
        last = last & (x0 % outer != outer - 1)
    return first, last


def Pi(psi, L, l0, outer=None):
    """(1 - gamma_0)/2 on first slices of black blocks, (1 + gamma_0)/2 on their last
    slices (where the outer operator has the crossing hop), zero elsewhere."""
    first, last = boundary_slices(L, l0, outer)
    lo = spin_mul(0.5 * (ONE4 - GAMMA[0]), psi) * site_mask(L, first)
    hi = spin_mul(0.5 * (ONE4 + GAMMA[0]), psi) * site_mask(L, last)
    return lo + hi


class Solvers:
    """The inversions the pseudo-fermion forces need: W_l0 (block-diagonal) and its
    adjoint, and the outer operator (M, or W_outer) and its adjoint (named M_inv /
    Mdag_inv). Default: CGLS to ``tol``; tests may pass dense LU solvers instead."""

    def __init__(self, U, kappa, l0, tol=1e-12, W_inv=None, M_inv=None, Mdag_inv=None,
                 Wdag_inv=None, outer=None):
        self.W_inv = W_inv or (lambda v: solvers.solve_eo(U, v, kappa, l0, tol=tol)[0])
        self.Wdag_inv = Wdag_inv or (
            lambda v: solvers.solve(U, v, kappa, l0, tol=tol, adjoint=True)[0])
        self.M_inv = M_inv or (lambda v: solvers.solve_eo(U, v, kappa, outer, tol=tol)[0])
        if Mdag_inv is None:
            # the adjoint system is solved as its own system (CGLS with the roles swapped).
            Mdag_inv = lambda v: solvers.solve(U, v, kappa, outer, tol=tol, adjoint=True)[0]
        self.Mdag_inv = Mdag_inv


def D_dOm_star(U, psi, kappa, l0, outer=None):
    """P_Om* A P_Om psi with A = M (outer None) or W_outer."""
    L = U.shape[:4]
    blk, wht = black_white_masks(L, l0)
    return wht * apply_op(U, blk * psi, kappa, outer)


def D_dOm(U, psi, kappa, l0, outer=None):
    """P_Om A P_Om* psi."""
    L = U.shape[:4]
    blk, wht = black_white_masks(L, l0)
    return blk * apply_op(U, wht * psi, kappa, outer)


def apply_Rhat(U, chi, kappa, l0, S: Solvers, outer=None):
    """R_hat chi for chi in range Pi (block solves only)."""
    L = U.shape[:4]
    blk, wht = black_white_masks(L, l0)
    v = D_dOm_star(U, chi, kappa, l0, outer)   # on white sites
    w = wht * S.W_inv(v)                        # D_Om*^{-1}: W_l0 is block diagonal
    u = D_dOm(U, w, kappa, l0, outer)           # on black sites
    z = blk * S.W_inv(u)                        # D_Om^{-1}
    return Pi(chi, L, l0, outer) - Pi(z, L, l0, outer)


def apply_Rhat_inv(U, chi, kappa, l0, S: Solvers, outer=None):
    """R_hat^{-1} chi = chi - Pi A^{-1} D_dOm* chi (one solve with the outer operator A);
    also returns psi = A^{-1} D_dOm* chi."""
    L = U.shape[:4]
    psi = S.M_inv(D_dOm_star(U, chi, kappa, l0, outer))
    return Pi(chi, L, l0, outer) - Pi(psi, L, l0, outer), psi


def action(U, chi, kappa, l0, S: Solvers, outer=None):
    """S_R = ||R_hat^{-1} chi||^2."""
    eta, _ = apply_Rhat_inv(U, chi, kappa, l0, S, outer)
    return float(np.sum(np.abs(eta) ** 2))


def heat_bath(U, g, kappa, l0, S: Solvers, outer=None):
    """chi = R_hat Pi g for Gaussian g with density ~ exp(-|g|^2)."""
    L = U.shape[:4]
    return apply_Rhat(U, Pi(g, L, l0, outer), kappa, l0, S, outer)

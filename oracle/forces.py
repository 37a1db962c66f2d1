"""Gauge action and forces (oracle, FP64).

Force convention (the paper's T_P step, Sec. 2 eq. 3, reads delta_U S as the derivative
along the su(3) directions): with T^a = lambda^a / 2 (Gell-Mann) and
U_mu(x) -> exp(i w T^a) U_mu(x),
    F^a(x, mu) = d S / d w at w = 0,
and the momentum update is p^a <- p^a - dtau F^a.

* ``pair_force(U, a, b, kappa, l0)`` = 2 Re < a, (d_{x,mu,a} W) b > for W = M (l0 None)
  or W = W_l0 (links between x0 blocks are absent from W, so their entries are zero).
  From eq. 2, only two entries of W contain U_mu(x):
      (d W b)(x)        = -kappa (1 - gamma_mu) i T^a U_mu(x) b(x + mu),
      (d W b)(x + mu)   = +i kappa (1 + gamma_mu) U_mu(x)^dagger T^a b(x),
  with the x0 wrap phase -1 carried by b(x+mu) and a(x+mu).
* ``pf_force``: S = ||W^{-1} phi||^2, X = W^{-1} phi, Y = W^{-dagger} X,
  F = -2 Re <Y, (d W) X>.
* ``schwarz_force``: S_R = ||R_hat^{-1} chi||^2 with psi = M^{-1} D_dOm* chi,
  eta = Pi chi - Pi psi, xi = M^{-dagger} Pi eta:
      F = 2 Re <xi, (d M) psi> - 2 Re <P_Om* xi, (d M) chi>.
* ``gauge_action`` (Sec. 1): S_G = -beta/3 sum_x sum_{mu>nu} Re Tr U_mu(x) U_nu(x+mu)
  U_mu(x+nu)^dagger U_nu(x)^dagger; ``gauge_force`` = -beta/3 Re Tr(i T^a U_mu(x) A_mu(x))
  with A_mu the sum of the six staples closing the plaquettes that contain U_mu(x).
"""
import numpy as np

from .gamma import ONE4, GAMMA, spin_mul
from .lattice import shift_fwd, shift_bwd
from .dirac import colour_mul, dagger, hop_keep_masks
from . import schwarz as sz
from . import solvers

# Gell-Mann matrices.
_l = np.zeros((8, 3, 3), dtype=complex)
_l[0][0, 1] = _l[0][1, 0] = 1
_l[1][0, 1] = -1j; _l[1][1, 0] = 1j
_l[2][0, 0] = 1; _l[2][1, 1] = -1
_l[3][0, 2] = _l[3][2, 0] = 1
_l[4][0, 2] = -1j; _l[4][2, 0] = 1j
_l[5][1, 2] = _l[5][2, 1] = 1
_l[6][1, 2] = -1j; _l[6][2, 1] = 1j
_l[7][0, 0] = _l[7][1, 1] = 1 / np.sqrt(3); _l[7][2, 2] = -2 / np.sqrt(3)
T = _l / 2.0           # T^a, Tr(T^a T^b) = delta_ab / 2


def _inner_re(a, b):
    """Re sum over spin and colour of conj(a) b, per site (shape L)."""
    return np.sum((a.conj() * b).real, axis=(-2, -1))


def pair_force(U, a, b, kappa, l0=None):
    """F[x, mu, a] = 2 Re <a, (d_{x,mu,a} W) b>."""
    L = U.shape[:4]
    keep_f, _ = hop_keep_masks(L, l0)
    F = np.zeros(tuple(L) + (4, 8))
    for mu in range(4):
        Umu = U[:, :, :, :, mu]
        b_f = shift_fwd(b, mu, fermion=True)      # b(x + mu) with the wrap phase
        a_f = shift_fwd(a, mu, fermion=True)      # a(x + mu) with the wrap phase
        for c in range(8):
            t1 = -kappa * spin_mul(ONE4 - GAMMA[mu], 1j * colour_mul(T[c] @ Umu, b_f))
            t2 = 1j * kappa * spin_mul(ONE4 + GAMMA[mu], colour_mul(dagger(Umu) @ T[c], b))
            val = 2.0 * (_inner_re(a, t1) + _inner_re(a_f, t2))
            if keep_f[mu] is not None:
                val = val * keep_f[mu][..., 0, 0]
            F[:, :, :, :, mu, c] = val
    return F


def pf_force(U, phi, kappa, l0, tol=1e-12, W_inv=None, Wdag_inv=None):
    """Force of S = ||W_l0^{-1} phi||^2 (l0 None: W = M)."""
    W_inv = W_inv or (lambda v: solvers.solve_eo(U, v, kappa, l0, tol=tol)[0])
    Wdag_inv = Wdag_inv or (lambda v: solvers.solve(U, v, kappa, l0, tol=tol, adjoint=True)[0])
    X = W_inv(phi)
    Y = Wdag_inv(X)
    return -pair_force(U, Y, X, kappa, l0)


def pf_action(U, phi, kappa, l0, tol=1e-12, W_inv=None):
    W_inv = W_inv or (lambda v: solvers.solve_eo(U, v, kappa, l0, tol=tol)[0])
    X = W_inv(phi)
    return float(np.sum(np.abs(X) ** 2))


def schwarz_force(U, chi, kappa, l0, S: "sz.Solvers", outer=None):
    """Force of S_R = ||R_hat^{-1} chi||^2 (outer operator M, or W_outer)."""
    L = U.shape[:4]
    eta, psi = sz.apply_Rhat_inv(U, chi, kappa, l0, S, outer)
    xi = S.Mdag_inv(sz.Pi(eta, L, l0, outer))
    _, wht = sz.black_white_masks(L, l0)
    return pair_force(U, xi, psi, kappa, outer) - pair_force(U, wht * xi, chi, kappa, outer)


def plaquette_field(U):
    """Re Tr U_P for every site and plane mu > nu, summed over planes (shape L)."""
    tot = 0.0
    for mu in range(4):
        for nu in range(mu):
            Umu = U[:, :, :, :, mu]
            Unu = U[:, :, :, :, nu]
            P = Umu @ shift_fwd(Unu, mu, False) @ dagger(shift_fwd(Umu, nu, False)) @ dagger(Unu)
            tot = tot + np.trace(P, axis1=-2, axis2=-1).real
    return tot


def gauge_action(U, beta):
    return float(-beta / 3.0 * np.sum(plaquette_field(U)))


def mean_plaquette(U):
    """(1 / 6V) sum_{x, mu>nu} (1/3) Re Tr U_P."""
    V = np.prod(U.shape[:4])
    return float(np.sum(plaquette_field(U)) / (3.0 * 6.0 * V))


def staples(U, mu):
    A = 0.0
    Umu = U[:, :, :, :, mu]
    for nu in range(4):
        if nu == mu:
            continue
        Unu = U[:, :, :, :, nu]
        up = shift_fwd(Unu, mu, False) @ dagger(shift_fwd(Umu, nu, False)) @ dagger(Unu)
        # U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
        dn_at_xmnu = dagger(shift_fwd(Unu, mu, False)) @ dagger(Umu) @ Unu   # evaluated at y = x - nu
        A = A + up + shift_bwd(dn_at_xmnu, nu, False)
    return A


def gauge_force(U, beta):
    L = U.shape[:4]
    F = np.zeros(tuple(L) + (4, 8))
    for mu in range(4):
        UA = U[:, :, :, :, mu] @ staples(U, mu)
        for c in range(8):
            F[:, :, :, :, mu, c] = -beta / 3.0 * np.trace(1j * T[c] @ UA, axis1=-2, axis2=-1).real
    return F


def force_profile(F):
    """x0 profile of a force field F[x0, x1, x2, x3, mu, a] (Sec. 3, Fig. 1: the plot of the average
    force on the spatial links against x0): row 0 = mean over the sites of each slice and
    over mu = 1, 2, 3 of |F(x, mu)|, row 1 = the same for mu = 0, where |F| is the
    Euclidean norm of the eight components F^a."""
    n = np.sqrt(np.sum(F ** 2, axis=-1))                 # [L0, L1, L2, L3, 4]
    spatial = n[..., 1:].mean(axis=(1, 2, 3, 4))
    time = n[..., 0].mean(axis=(1, 2, 3))
    return np.stack([spatial, time])

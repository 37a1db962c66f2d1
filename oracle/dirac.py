"""Wilson-Dirac operator M, its x0-block restriction W and the even-odd Schur complement
(oracle, FP64).

Sec. 1, eq. 2:
    (M psi)(x) = psi(x) - kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                                        + (1 + gamma_mu) U_mu(x - mu)^dagger psi(x - mu) ].
The "1" is the unit in site, spin and colour.

Sec. 1 (Schwarz preconditioning, one-dimensional decomposition): W with blocks of length
l0 along x0 is M with every hop whose two end points lie in different blocks removed.
With l_mu = L_mu for mu = 1, 2, 3 only the x0 hops between slices l0-1 and 0 (mod l0)
are removed, including the wrap between x0 = L0-1 and x0 = 0.

Sec. 1 (W_{2,eo}): M = [[1, -kappa D_eo], [-kappa D_oe, 1]] in the (even, odd) site
partition, and M_hat = 1 - kappa^2 D_eo D_oe on even sites.

The adjoint is written out from the definition (gamma_mu -> -gamma_mu with U and U^dagger
attached to the same links), not through gamma_5; gamma_5-hermiticity is a test.
"""
import numpy as np

from .gamma import ONE4, GAMMA, spin_mul
from .lattice import shift_fwd, shift_bwd, coords, block_of_x0, parity, site_mask


def colour_mul(U: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U psi)_{s,a}(x) = sum_b U_ab(x) psi_{s,b}(x)."""
    return np.matmul(U[..., None, :, :], psi[..., :, :, None])[..., 0]


def dagger(U: np.ndarray) -> np.ndarray:
    return np.swapaxes(U.conj(), -1, -2)


def hop_keep_masks(L, l0):
    """Per direction, booleans over sites saying whether the forward hop x -> x+mu and the
    backward hop x -> x-mu stay inside one x0 block (l0 = None: no blocks, keep all)."""
    keep_f, keep_b = [], []
    x0 = coords(L)[0]
    L0 = L[0]
    for mu in range(4):
        if l0 is None or mu != 0:
            keep_f.append(None)
            keep_b.append(None)
            continue
        same_f = block_of_x0(x0, l0) == block_of_x0((x0 + 1) % L0, l0)
        same_b = block_of_x0(x0, l0) == block_of_x0((x0 - 1) % L0, l0)
        keep_f.append(site_mask(L, same_f))
        keep_b.append(site_mask(L, same_b))
    return keep_f, keep_b


def hop(U: np.ndarray, psi: np.ndarray, l0=None, adjoint: bool = False) -> np.ndarray:
    """D psi = sum_mu [(1 - s gamma_mu) U_mu(x) psi(x+mu) + (1 + s gamma_mu) U_mu(x-mu)^+ psi(x-mu)]
    with s = +1 (D) or s = -1 (D^dagger); hops between different x0 blocks of length l0
    are dropped when l0 is given."""
    L = U.shape[:4]
    keep_f, keep_b = hop_keep_masks(L, l0)
    s = -1.0 if adjoint else 1.0
    out = np.zeros(np.broadcast_shapes(psi.shape), dtype=complex)
    for mu in range(4):
        Umu = U[:, :, :, :, mu]
        fwd = spin_mul(ONE4 - s * GAMMA[mu], colour_mul(Umu, shift_fwd(psi, mu, fermion=True)))
        bwd = spin_mul(ONE4 + s * GAMMA[mu],
                       shift_bwd(colour_mul(dagger(Umu), psi), mu, fermion=True))
        if keep_f[mu] is not None:
            fwd = fwd * keep_f[mu]
            bwd = bwd * keep_b[mu]
        out += fwd + bwd
    return out


def apply_M(U, psi, kappa, adjoint=False):
    """M psi (eq. 2), or M^dagger psi."""
    return psi - kappa * hop(U, psi, None, adjoint)


def apply_W(U, psi, kappa, l0, adjoint=False):
    """W psi: M with the hops between x0 blocks of length l0 removed (or W^dagger psi)."""
    return psi - kappa * hop(U, psi, l0, adjoint)


def apply_op(U, psi, kappa, l0=None, adjoint=False):
    """M (l0 None) or W_l0, optionally adjoint."""
    return psi - kappa * hop(U, psi, l0, adjoint)


def parity_masks(L):
    p = parity(L)
    return site_mask(L, p == 0), site_mask(L, p == 1)


def apply_Mhat(U, psi_e, kappa, l0=None, adjoint=False):
    """Even-odd Schur complement on even sites:
    M_hat psi_e = psi_e - kappa^2 D_eo D_oe psi_e  (adjoint: psi_e - kappa^2 (D_eo D_oe)^+ psi_e).
    Input and output are full-lattice arrays that vanish on odd sites."""
    L = U.shape[:4]
    e, o = parity_masks(L)
    t = o * hop(U, e * psi_e, l0, adjoint)
    return e * psi_e - kappa * kappa * (e * hop(U, t, l0, adjoint))


def gamma5_field(psi):
    from .gamma import GAMMA5
    return spin_mul(GAMMA5, psi)


def dense_matrix(U, kappa, l0=None, adjoint=False) -> np.ndarray:
    """Dense matrix of M / W (3072 x 3072 on a 4^4 lattice); column j = op(e_j), with the
    unit vectors in canonical (site, spin, colour) order."""
    L = U.shape[:4]
    n = int(np.prod(L)) * 12
    eye = np.eye(n, dtype=complex).reshape((n,) + tuple(L) + (4, 3))
    cols = apply_op(U, eye, kappa, l0, adjoint)
    return cols.reshape(n, n).T

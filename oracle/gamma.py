"""Euclidean Dirac matrices for the oracle.

The paper (Sec. 1, eq. 2) uses "Euclidean gamma matrices" without fixing a representation.
The library's interchange format fixes the chiral basis written here in 2x2 blocks:

    gamma_0 = [[0, -1], [-1, 0]],   gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],
    gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3 = diag(1, 1, -1, -1).

Pins (tests/test_oracle_dirac.py::test_gamma_algebra): Clifford algebra {g_mu, g_nu} = 2 delta, hermiticity,
gamma_5 = diag(1,1,-1,-1), gamma_5 anticommuting with every gamma_mu.
"""
import numpy as np

_I2 = np.eye(2, dtype=complex)
_Z2 = np.zeros((2, 2), dtype=complex)
SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=complex),
    np.array([[0, -1j], [1j, 0]], dtype=complex),
    np.array([[1, 0], [0, -1]], dtype=complex),
)

GAMMA = (
    np.block([[_Z2, -_I2], [-_I2, _Z2]]),
    np.block([[_Z2, -1j * SIGMA[0]], [1j * SIGMA[0], _Z2]]),
    np.block([[_Z2, -1j * SIGMA[1]], [1j * SIGMA[1], _Z2]]),
    np.block([[_Z2, -1j * SIGMA[2]], [1j * SIGMA[2], _Z2]]),
)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ONE4 = np.eye(4, dtype=complex)

# The two spin structures of the hop in eq. 2.
ONE_MINUS = tuple(ONE4 - g for g in GAMMA)   # multiplies U_mu(x) psi(x + mu)
ONE_PLUS = tuple(ONE4 + g for g in GAMMA)    # multiplies U_mu(x - mu)^dagger psi(x - mu)


def spin_mul(S: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(S psi)_s = sum_t S_st psi_t on the spin index (axis -2) of a spinor field."""
    return np.matmul(S, psi)


def gamma5(psi: np.ndarray) -> np.ndarray:
    return spin_mul(GAMMA5, psi)

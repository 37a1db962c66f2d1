"""Pins of the oracle's Schwarz boundary operator: the exact determinant identity
det M = det W1 * det R_hat (dense, 4^4 and a 4-block lattice), its independence of the
colour assignment and of the halving, and R_hat^{-1} R_hat = 1 through the CG solvers."""
import numpy as np
import pytest

import synth
from oracle import dirac, lattice, schwarz, solvers


def lu_solvers(U, kappa, l0):
    return schwarz.Solvers(
        U, kappa, l0,
        W_inv=solvers.lu_solver(U, kappa, l0), M_inv=solvers.lu_solver(U, kappa, None),
        Mdag_inv=solvers.lu_solver(U, kappa, None, adjoint=True),
        Wdag_inv=solvers.lu_solver(U, kappa, l0, adjoint=True))


def _range_basis(P_apply, L):
    n = int(np.prod(L)) * 12
    eye = np.eye(n, dtype=complex).reshape((n,) + tuple(L) + (4, 3))
    P = P_apply(eye).reshape(n, n).T
    w, v = np.linalg.eigh(P)
    assert np.allclose(w[np.abs(w) > 1e-9], 1.0)          # Pi is an orthogonal projector
    return v[:, w > 0.5]


def _logdet(A):
    s, l = np.linalg.slogdet(A)
    return s, l


@pytest.mark.parametrize("L,l0,k,seed", [((4, 4, 4, 4), 2, 0.155, 1001),
                                         ((8, 2, 4, 2), 2, 0.16, 7),
                                         ((12, 2, 2, 2), 3, 0.17, 8)])
def test_det_M_equals_det_W1_times_det_Rhat(L, l0, k, seed):
    U = synth.gauge_field(L, 0.5, seed)
    S = lu_solvers(U, k, l0)
    B = _range_basis(lambda f: schwarz.Pi(f, L, l0), L)
    # dimension: 2 boundary slices per black block x V3 sites x 2 spins x 3 colours
    nblack = L[0] // l0 // 2
    assert B.shape[1] == nblack * 2 * (np.prod(L[1:])) * 6
    basis_fields = B.T.reshape((B.shape[1],) + tuple(L) + (4, 3))
    R = schwarz.apply_Rhat(U, basis_fields, k, l0, S)
    Rmat = B.conj().T @ R.reshape(B.shape[1], -1).T
    sM, lM = _logdet(dirac.dense_matrix(U, k))
    sW, lW = _logdet(dirac.dense_matrix(U, k, l0))
    sR, lR = _logdet(Rmat)
    assert abs(lM - (lW + lR)) <= 1e-10 * abs(lM) + 1e-10
    assert abs(sM - sW * sR) <= 1e-9
    # The unhalved boundary operator (Pi replaced by the full restriction to the black
    # boundary slices) has the same determinant: the halving is exact.
    first, last = schwarz.boundary_slices(L, l0)
    Pfull = lambda f: f * lattice.site_mask(L, first | last)
    Bf = _range_basis(Pfull, L)
    blk, wht = schwarz.black_white_masks(L, l0)
    F = Bf.T.reshape((Bf.shape[1],) + tuple(L) + (4, 3))
    v = schwarz.D_dOm_star(U, F, k, l0)
    w = wht * S.W_inv(v)
    z = blk * S.W_inv(schwarz.D_dOm(U, w, k, l0))
    Rf = Bf.conj().T @ (F - Pfull(z)).reshape(Bf.shape[1], -1).T
    sF, lF = _logdet(Rf)
    assert abs(lF - lR) <= 1e-10 * abs(lR) + 1e-10 and abs(sF - sR) <= 1e-9


def test_det_Rhat_independent_of_colour_choice():
    """Translating the gauge field by l0 slices swaps black and white blocks; det M and
    det W1 are unchanged by the translation, so det R_hat must be too."""
    L, l0, k = (8, 2, 2, 4), 2, 0.16
    U = synth.gauge_field(L, 0.5, 9)
    Ut = np.roll(U, -l0, axis=0)
    dets = []
    for V in (U, Ut):
        S = lu_solvers(V, k, l0)
        B = _range_basis(lambda f: schwarz.Pi(f, L, l0), L)
        R = schwarz.apply_Rhat(V, B.T.reshape((B.shape[1],) + L + (4, 3)), k, l0, S)
        dets.append(_logdet(B.conj().T @ R.reshape(B.shape[1], -1).T))
    assert abs(dets[0][1] - dets[1][1]) < 1e-10 * abs(dets[0][1])
    assert abs(dets[0][0] - dets[1][0]) < 1e-9


def test_heat_bath_action_equals_noise_norm_with_cg():
    """S_R(R_hat Pi g) = ||Pi g||^2: the full-solve inverse undoes the block-solve R_hat."""
    L, l0, k = (8, 4, 4, 4), 2, 0.155
    U = synth.gauge_field(L, 0.5, 1001)
    g = synth.noise_spinor(L, 4005)
    S = schwarz.Solvers(U, k, l0, tol=1e-13)
    chi = schwarz.heat_bath(U, g, k, l0, S)
    # chi lies in range Pi
    np.testing.assert_allclose(schwarz.Pi(chi, L, l0), chi, atol=1e-14)
    SR = schwarz.action(U, chi, k, l0, S)
    ref = float(np.sum(np.abs(schwarz.Pi(g, L, l0)) ** 2))
    assert abs(SR - ref) <= 1e-9 * ref

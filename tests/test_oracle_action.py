"""Pins of the four-part pseudo-fermion action and the five-level integrator (Sec. 1 end,
Sec. 2): the iterated Schwarz identity det W1 = det W2 det R_hat_2, the factorisation of
det M into the four parts (dense determinants), the heat baths (each S_j equals its
squared noise), every new force against finite differences, and the trajectory's
reversibility and dH ~ h^2."""
import numpy as np
import pytest

import synth
from oracle import action, dirac, hmc, schwarz, solvers
from test_oracle_schwarz import _range_basis, _logdet

L, L0_1, L0_2, K, RHO = (8, 2, 2, 2), 4, 2, 0.15, 0.2


def _lu_parts(U, k=K):
    sz4 = schwarz.Solvers(U, k, L0_1, W_inv=solvers.lu_solver(U, k, L0_1), M_inv=solvers.lu_solver(U, k, None),
                          Mdag_inv=solvers.lu_solver(U, k, None, adjoint=True),
                          Wdag_inv=solvers.lu_solver(U, k, L0_1, adjoint=True))
    sz3 = schwarz.Solvers(U, k, L0_2, W_inv=solvers.lu_solver(U, k, L0_2), M_inv=solvers.lu_solver(U, k, L0_1),
                          Mdag_inv=solvers.lu_solver(U, k, L0_1, adjoint=True),
                          Wdag_inv=solvers.lu_solver(U, k, L0_2, adjoint=True), outer=L0_1)
    return action.FourPart(U, k, L0_1, L0_2, RHO, tol=1e-13, sz4=sz4, sz3=sz3)


def _rhat_logdet(U, k, l0, S, outer, Lat):
    B = _range_basis(lambda f: schwarz.Pi(f, Lat, l0, outer), Lat)
    bf = B.T.reshape((B.shape[1],) + tuple(Lat) + (4, 3))
    R = schwarz.apply_Rhat(U, bf, k, l0, S, outer)
    return B.shape[1], _logdet(B.conj().T @ R.reshape(B.shape[1], -1).T)


@pytest.mark.parametrize("Lat,seed", [((8, 2, 2, 2), 11), ((8, 2, 2, 4), 12)])
def test_iterated_schwarz_determinant_identity(Lat, seed):
    """det W1 = det W2 * det R_hat_2 with R_hat_2 built from (W1, W2); its range is one
    interface (two spins x three colours x V3 sites) per level-1 block."""
    U = synth.gauge_field(Lat, 0.5, seed)
    S = schwarz.Solvers(U, K, L0_2, W_inv=solvers.lu_solver(U, K, L0_2), M_inv=solvers.lu_solver(U, K, L0_1),
                        outer=L0_1)
    dim, (sR, lR) = _rhat_logdet(U, K, L0_2, S, L0_1, Lat)
    assert dim == (Lat[0] // L0_1) * int(np.prod(Lat[1:])) * 6
    s1, l1 = _logdet(dirac.dense_matrix(U, K, L0_1))
    s2, l2 = _logdet(dirac.dense_matrix(U, K, L0_2))
    assert abs(l1 - (l2 + lR)) <= 1e-10 * abs(l1)
    assert abs(s1 - s2 * sR) <= 1e-9


def test_four_part_factorisation_of_det_M():
    """log det M = log det R_hat + log det R_hat_2 + log det W2eo (dense): with
    det W2eo = det(W2eo W3eo^-1) det W3eo the four parts reproduce det^2 M."""
    U = synth.gauge_field(L, 0.5, 13)
    A = _lu_parts(U)
    _, (s4, l4) = _rhat_logdet(U, K, L0_1, A.sz4, None, L)
    _, (s3, l3) = _rhat_logdet(U, K, L0_2, A.sz3, L0_1, L)
    n = int(np.prod(L)) * 12
    ev = A.e.reshape(-1)
    eye = np.eye(n, dtype=complex).reshape((n,) + L + (4, 3))
    W2 = A.W2eo(eye * A.e).reshape(n, n).T
    W3 = A.W3eo(eye * A.e).reshape(n, n).T
    idx = np.nonzero(np.broadcast_to(A.e, L + (4, 3)).reshape(-1))[0]
    s2, l2 = _logdet(W2[np.ix_(idx, idx)])
    s3w, l3w = _logdet(W3[np.ix_(idx, idx)])
    sM, lM = _logdet(dirac.dense_matrix(U, K))
    assert abs(lM - (l4 + l3 + l2)) <= 1e-10 * abs(lM)
    assert abs(sM - s4 * s3 * s2) <= 1e-9
    # the mass shift changes the determinant that S1 carries (S2 carries the ratio)
    assert abs(l3w - l2) > 1.0


def test_heat_baths_give_the_noise_norms():
    U = synth.gauge_field(L, 0.5, 31)
    A = _lu_parts(U)
    xi1, xi2 = synth.gaussian_spinor(L, 32) * A.e, synth.gaussian_spinor(L, 33) * A.e
    g3, g4 = synth.noise_spinor(L, 34), synth.noise_spinor(L, 35)
    n2 = lambda f: float(np.sum(np.abs(f) ** 2))
    assert abs(A.S1(A.heat_bath1(xi1)) - n2(xi1)) <= 1e-10 * n2(xi1)
    assert abs(A.S2(A.heat_bath2(xi2)) - n2(xi2)) <= 1e-10 * n2(xi2)
    p3 = n2(schwarz.Pi(g3, L, L0_2, L0_1))
    assert abs(A.S3(A.heat_bath3(g3)) - p3) <= 1e-10 * p3
    p4 = n2(schwarz.Pi(g4, L, L0_1))
    assert abs(A.S4(A.heat_bath4(g4)) - p4) <= 1e-10 * p4


def _fd(S, U, site, mu, a, h=1e-4):
    def Ut(t):
        p = np.zeros(tuple(U.shape[:4]) + (4, 8))
        p[site + (mu, a)] = 1.0
        return hmc.T_U(U, p, t)
    d = lambda h: (S(Ut(h)) - S(Ut(-h))) / (2 * h)
    return (4 * d(h / 2) - d(h)) / 3


def test_four_part_forces_match_finite_differences():
    """F1, F2 (even-odd W2 with the mass shift) and F3 (Schwarz term of W1 over W2)
    against central differences (Richardson); the links cut in W2 carry no S1/S2 force,
    the links between level-1 blocks no S3 force."""
    U = synth.gauge_field(L, 0.5, 31)
    A = _lu_parts(U)
    phi1 = A.heat_bath1(synth.gaussian_spinor(L, 32) * A.e)
    phi2 = A.heat_bath2(synth.gaussian_spinor(L, 33) * A.e)
    chi3 = A.heat_bath3(synth.noise_spinor(L, 34))
    F = {1: A.F1(phi1), 2: A.F2(phi2), 3: A.F3(chi3)}
    S = {1: lambda V: _lu_parts(V).S1(phi1), 2: lambda V: _lu_parts(V).S2(phi2),
         3: lambda V: _lu_parts(V).S3(chi3)}
    links = [((4, 0, 1, 0), 2, 6), ((5, 0, 0, 1), 1, 0), ((1, 1, 1, 0), 0, 3), ((2, 1, 0, 1), 3, 5),
             ((3, 1, 0, 1), 0, 1), ((6, 0, 1, 1), 0, 2)]
    for j in (1, 2, 3):
        for site, mu, a in links:
            fd = _fd(S[j], U, site, mu, a)
            assert abs(fd - F[j][site + (mu, a)]) <= 1e-7 * max(1.0, abs(fd)), (j, site, mu, a)
    x0 = np.arange(L[0])
    cut2 = (x0 % L0_2) == L0_2 - 1
    cut1 = (x0 % L0_1) == L0_1 - 1
    assert np.all(F[1][cut2, ..., 0, :] == 0) and np.all(F[2][cut2, ..., 0, :] == 0)
    assert np.all(F[3][cut1, ..., 0, :] == 0)
    assert np.any(F[3][cut2 & ~cut1, ..., 0, :] != 0)


def test_five_level_trajectory_reversible_and_dH_scales():
    """Gauge (SW), S1 (SW), S2, S3, S4 (leap-frog) nested as in Sec. 2: a trajectory run
    forward, momenta flipped and run again returns to the start; dH falls ~4x when every
    step size is halved."""
    U0 = synth.gauge_field(L, 0.5, 41)
    A = action.FourPart(U0, K, L0_1, L0_2, RHO, tol=1e-13)
    fields = (A.heat_bath1(synth.gaussian_spinor(L, 42) * A.e), A.heat_bath2(synth.gaussian_spinor(L, 43) * A.e),
              A.heat_bath3(synth.noise_spinor(L, 44)), A.heat_bath4(synth.noise_spinor(L, 45)))
    beta = 5.6
    make = lambda U: action.FourPart(U, K, L0_1, L0_2, RHO, tol=1e-13)
    p0 = synth.gaussian_momenta(L, 46)
    tau = 0.2
    lv = action.five_level(fields, K, beta, L0_1, L0_2, RHO, (2, 2, 1, 1, 2), make)
    U1, p1 = hmc.integrate(lv, U0, p0, tau)
    U2, p2 = hmc.integrate(lv, U1, -p1, tau)
    assert np.max(np.abs(U2 - U0)) <= 1e-10 and np.max(np.abs(-p2 - p0)) <= 1e-10
    dH = []
    for n4 in (2, 4):
        lv = action.five_level(fields, K, beta, L0_1, L0_2, RHO, (2, 2, 1, 1, n4), make)
        U1, p1 = hmc.integrate(lv, U0, p0, tau)
        dH.append(abs(hmc.hamiltonian(lv, U1, p1) - hmc.hamiltonian(lv, U0, p0)))
    assert 3.0 <= dH[0] / dH[1] <= 5.0, dH

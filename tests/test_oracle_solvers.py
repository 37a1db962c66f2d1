"""Pins of the oracle's BiCGstab, Schwarz alternating procedure and geometric series
(Sec. 3: geometric series for the block terms, BiCGstab with even-odd and Schwarz
preconditioning for the full-lattice term) against facts that do not come from the
oracle: Krylov finite termination, numpy's dense solve, the exact vanishing of the SAP
residual on the colour updated last, and the free-field spectrum, which fixes the
convergence rate of the geometric series in closed form."""
import numpy as np
import pytest

import synth
from oracle import dirac, lattice, solvers


def test_bicgstab_terminates_for_three_eigenvalues():
    """A = diag(d) with d taking three distinct complex values: the minimal polynomial has
    degree 3, so BiCGstab reaches the exact solution b / d within 3 iterations."""
    L = (2, 2, 2, 4)
    b = synth.gaussian_spinor(L, 7)
    lam = np.array([1.5 + 0.5j, 0.7 - 0.2j, 2.0 + 1.0j])
    d = lam[np.arange(b.size).reshape(b.shape) % 3]
    x, its, res = solvers.bicgstab(lambda v: d * v, b, tol=1e-13)
    assert its <= 3
    assert np.max(np.abs(x - b / d)) <= 1e-12 * np.max(np.abs(b / d))


def test_bicgstab_matches_dense_solve_with_and_without_preconditioner():
    rng = np.random.default_rng(3)
    L = (2, 2, 2, 2)
    n = 12 * 16
    A = np.eye(n) * 4 + (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) / np.sqrt(n)
    b = synth.gaussian_spinor(L, 8, nrhs=2)
    op = lambda v: (v.reshape(v.shape[0], n) @ A.T).reshape(v.shape)
    ref = np.linalg.solve(A, b.reshape(2, n).T).T.reshape(b.shape)
    Kd = 1.0 / np.diag(A)
    K = lambda v: (v.reshape(v.shape[0], n) * Kd).reshape(v.shape)
    for prec in (None, K):
        x, its, res = solvers.bicgstab(op, b, tol=1e-13, K=prec)
        assert np.all(np.asarray(res) <= 1e-13)
        assert np.max(np.abs(x - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_eo_bicgstab_matches_dense_lu():
    L, k = (4, 4, 4, 4), 0.155
    U = synth.gauge_field(L, 0.5, 1001)
    b = synth.gaussian_spinor(L, 2001)
    for l0 in (None, 2):
        A = dirac.dense_matrix(U, k, l0)
        ref = np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)
        x, its, res = solvers.solve_eo_bicgstab(U, b, k, l0, tol=1e-12)
        assert res <= 1e-12
        assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= np.linalg.cond(A) * 1e-12


def test_sap_residual_vanishes_on_the_last_colour():
    """After a Schwarz cycle (black blocks, then white blocks, exact block solves) the
    residual r - M x is zero on the white blocks: every hop leaving a white block ends on
    a black site, so M and W_l0 agree on the white sites for a field supported on them."""
    L, l0, k = (8, 2, 2, 4), 2, 0.15
    U = synth.gauge_field(L, 0.5, 11)
    r = synth.gaussian_spinor(L, 12)
    x = solvers.sap_precond(U, r, k, l0, ncy=1, block_tol=1e-14)
    res = r - dirac.apply_M(U, x, k)
    white = lattice.site_mask(L, lattice.colour_x0_mask(L, l0, "white"))
    black = lattice.site_mask(L, lattice.colour_x0_mask(L, l0, "black"))
    assert np.max(np.abs(res * white)) <= 1e-12 * np.max(np.abs(r))
    assert np.max(np.abs(res * black)) > 1e-3 * np.max(np.abs(r))


def test_sap_cycles_converge_to_the_inverse_and_precondition_bicgstab():
    L, l0, k = (8, 2, 2, 4), 2, 0.15
    U = synth.gauge_field(L, 0.5, 13)
    r = synth.gaussian_spinor(L, 14)
    ref = np.linalg.solve(dirac.dense_matrix(U, k), r.reshape(-1)).reshape(r.shape)
    errs = [np.linalg.norm(solvers.sap_precond(U, r, k, l0, n, 1e-14) - ref) / np.linalg.norm(ref)
            for n in (1, 2, 4, 8)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3 * errs[0], errs
    x, its, res = solvers.solve_sap_bicgstab(U, r, k, l0, ncy=2, tol=1e-12, block_tol=1e-14)
    assert res <= 1e-12
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-10
    _, its_plain, _ = solvers.bicgstab(lambda v: dirac.apply_M(U, v, k), r, tol=1e-12)
    assert its < its_plain


def _free_field(L):
    U = np.zeros(tuple(L) + (4, 3, 3), dtype=complex)
    U[...] = np.eye(3)
    return U


def _free_spectral_radius(L, kappa):
    """kappa^2 max_p |lambda(p)|^2 of D_eo D_oe on the free field: D acts on a plane wave
    as a - i sum_mu gamma_mu b_mu with a = sum 2 cos p_mu, b_mu = 2 sin p_mu (a normal
    matrix with eigenvalues a +/- i|b|); p_0 = (2 n + 1) pi / L0 (antiperiodic),
    p_k = 2 pi n / L_k; D_eo D_oe has the squares of these eigenvalues."""
    ps = [(2 * np.arange(L[0]) + 1) * np.pi / L[0]] + [2 * np.pi * np.arange(n) / n for n in L[1:]]
    P = np.meshgrid(*ps, indexing="ij")
    a = sum(2 * np.cos(p) for p in P)
    b2 = sum(4 * np.sin(p) ** 2 for p in P)
    return kappa ** 2 * np.max(a ** 2 + b2)


def test_geometric_series_rate_is_the_free_field_spectral_radius():
    """On the free field the residual of the series after N terms falls by the spectral
    radius rho = kappa^2 max|lambda(D)|^2 per term (closed form from the free Wilson
    spectrum): rho < 1 converges, rho > 1 diverges."""
    L = (4, 4, 4, 4)
    U = _free_field(L)
    b = synth.gaussian_spinor(L, 21)
    for k in (0.12, 0.13):
        rho = _free_spectral_radius(L, k)
        assert rho < 1.0
        r60 = solvers.geometric_series(U, b, k, tol=0.0, maxiter=60)[2]
        r70 = solvers.geometric_series(U, b, k, tol=0.0, maxiter=70)[2]
        assert abs(r70 / r60 - rho ** 10) <= 2e-3 * rho ** 10, (k, r70 / r60, rho ** 10)
    k = 0.14
    rho = _free_spectral_radius(L, k)
    assert rho > 1.0
    r30 = solvers.geometric_series(U, b, k, tol=0.0, maxiter=30)[2]
    r40 = solvers.geometric_series(U, b, k, tol=0.0, maxiter=40)[2]
    assert r40 > r30 > 1.0
    assert abs(r40 / r30 - rho ** 10) <= 2e-2 * rho ** 10


def test_geometric_series_matches_dense_lu_on_blocks():
    L, k = (4, 4, 4, 4), 0.155
    U = synth.gauge_field(L, 0.5, 1001)
    b = synth.gaussian_spinor(L, 2001)
    A = dirac.dense_matrix(U, k, 2)
    ref = np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)
    x, n, res = solvers.geometric_series(U, b, k, 2, tol=1e-12)
    assert res <= 1e-12 and n > 1
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= np.linalg.cond(A) * 1e-12


def test_sap_with_series_block_solves_is_linear_and_converges():
    """Schwarz cycles whose block systems take N terms of the even-odd geometric series:
    (i) the preconditioner is a linear map (K(a u + v) = a K(u) + K(v) to rounding), which
    an adaptive block solve is not; (ii) as N grows the block solves approach the exact
    ones (the series converges at kappa = 0.12), so K approaches the exact-block cycles;
    (iii) BiCGstab right-preconditioned by it reaches the dense solution."""
    L, l0, k = (8, 2, 2, 4), 2, 0.12
    U = synth.gauge_field(L, 0.5, 15)
    u = synth.gaussian_spinor(L, 16)
    v = synth.gaussian_spinor(L, 17)
    a = 0.7 - 1.3j
    K = lambda w, n: solvers.sap_precond(U, w, k, l0, 2, block_terms=n)
    lhs, rhs = K(a * u + v, 6), a * K(u, 6) + K(v, 6)
    assert np.max(np.abs(lhs - rhs)) <= 1e-13 * np.max(np.abs(rhs))
    exact = solvers.sap_precond(U, u, k, l0, 2, block_tol=1e-14)
    errs = [np.linalg.norm(K(u, n) - exact) / np.linalg.norm(exact) for n in (2, 8, 32, 128)]
    assert all(b < a_ for a_, b in zip(errs, errs[1:])), errs
    assert errs[-1] <= 1e-10, errs
    ref = np.linalg.solve(dirac.dense_matrix(U, k), u.reshape(-1)).reshape(u.shape)
    x, its, res = solvers.solve_sap_bicgstab(U, u, k, l0, ncy=2, tol=1e-12, block_terms=6)
    assert res <= 1e-12
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) <= 1e-10


def _dense_eo_shifted(U, k, l0, rho, adjoint):
    """Dense (M_hat + rho) on the even sites, from the oracle's dense M_hat-free operators:
    built column by column from the plain hop of eq. 2 on unit vectors (no series code)."""
    L = U.shape[:4]
    e, o = dirac.parity_masks(L)
    n = int(np.prod(L)) * 12
    ev = np.nonzero(np.broadcast_to(e, tuple(L) + (4, 3)).reshape(-1))[0]
    cols = []
    for i in ev:
        v = np.zeros(n, dtype=complex)
        v[i] = 1.0
        v = v.reshape(tuple(L) + (4, 3))
        w = dirac.apply_Mhat(U, v, k, l0, adjoint) + rho * v
        cols.append(w.reshape(-1)[ev])
    return np.array(cols).T, ev


@pytest.mark.parametrize("l0,adjoint", [(None, False), (2, False), (2, True)])
def test_shifted_geometric_series_matches_dense_solve(l0, adjoint):
    """(M_hat + rho) x = b on the even sites (rho = 0.3, the W3eo = W2eo + rho of the mass
    preconditioning, and rho = 0) against numpy's dense solve; a dropped 1/(1 + rho) in
    t_0 or in the ratio of the terms fails it."""
    L, k = (4, 2, 2, 4), 0.13
    U = synth.gauge_field(L, 0.5, 31)
    e, _ = dirac.parity_masks(L)
    b = e * synth.gaussian_spinor(L, 32)
    for rho in (0.3, 0.0):
        A, ev = _dense_eo_shifted(U, k, l0, rho, adjoint)
        ref = np.linalg.solve(A, b.reshape(-1)[ev])
        x, n, res = solvers.geometric_series_eo(U, b, k, l0, rho, tol=1e-13, adjoint=adjoint)
        assert res <= 1e-13 and n > 2
        assert np.all(x.reshape(-1)[np.setdiff1d(np.arange(b.size), ev)] == 0)
        assert np.linalg.norm(x.reshape(-1)[ev] - ref) <= 1e-11 * np.linalg.norm(ref), (rho, l0)


def test_shifted_geometric_series_rate_is_free_radius_over_one_plus_rho():
    """Free field: the residual falls per term by the spectral radius of the unshifted
    series divided by 1 + rho (closed form of the free Wilson spectrum); at kappa = 0.14,
    where the unshifted series diverges, rho = 0.2 makes it converge."""
    L = (4, 4, 4, 4)
    U = _free_field(L)
    e, _ = dirac.parity_masks(L)
    b = e * synth.gaussian_spinor(L, 33)
    for k, rho in ((0.12, 0.1), (0.14, 0.2)):
        rate = _free_spectral_radius(L, k) / (1.0 + rho)
        assert rate < 1.0
        r60 = solvers.geometric_series_eo(U, b, k, None, rho, tol=0.0, maxiter=60)[2]
        r70 = solvers.geometric_series_eo(U, b, k, None, rho, tol=0.0, maxiter=70)[2]
        assert abs(r70 / r60 - rate ** 10) <= 2e-3 * rate ** 10, (k, rho, r70 / r60, rate ** 10)

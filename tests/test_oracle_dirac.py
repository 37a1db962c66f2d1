"""Pins of the oracle's gamma matrices, M, W and even-odd operator against facts that do
not depend on the oracle's own code: the Clifford algebra, gamma5-hermiticity, gauge
covariance, the free-field plane-wave closed form and spectrum, the exact equivalence of W
with M on a field whose block-crossing links are zero, and dense linear algebra on 4^4."""
import itertools

import numpy as np
import pytest

import synth
from oracle import dirac, gamma, lattice, solvers

L4 = (4, 4, 4, 4)


def _rand_su3_field(L, seed):
    return synth.gauge_field(L, 0.7, seed)


def _vdot(a, b):
    return np.vdot(a.reshape(-1), b.reshape(-1))


def test_gamma_algebra():
    g = gamma.GAMMA
    for m, n in itertools.product(range(4), range(4)):
        np.testing.assert_allclose(g[m] @ g[n] + g[n] @ g[m], 2.0 * (m == n) * np.eye(4), atol=0)
    for m in range(4):
        np.testing.assert_allclose(g[m], g[m].conj().T, atol=0)
        np.testing.assert_allclose(gamma.GAMMA5 @ g[m] + g[m] @ gamma.GAMMA5, 0, atol=0)
    np.testing.assert_allclose(gamma.GAMMA5, np.diag([1, 1, -1, -1]), atol=1e-15)


def test_kappa_zero_is_identity():
    U = _rand_su3_field(L4, 11)
    psi = synth.gaussian_spinor(L4, 12)
    assert np.array_equal(dirac.apply_M(U, psi, 0.0), psi)
    assert np.array_equal(dirac.apply_W(U, psi, 0.0, 2), psi)


@pytest.mark.parametrize("l0", [None, 2])
def test_adjoint_and_gamma5_hermiticity(l0):
    L = (4, 4, 2, 6) if l0 is None else (8, 2, 4, 2)
    U = _rand_su3_field(L, 13)
    chi = synth.gaussian_spinor(L, 14)
    psi = synth.gaussian_spinor(L, 15)
    k = 0.17
    Mpsi = dirac.apply_op(U, psi, k, l0)
    Mdchi = dirac.apply_op(U, chi, k, l0, adjoint=True)
    lhs, rhs = _vdot(chi, Mpsi), _vdot(Mdchi, psi)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    g5Mg5 = dirac.gamma5_field(dirac.apply_op(U, dirac.gamma5_field(chi), k, l0))
    np.testing.assert_allclose(g5Mg5, Mdchi, rtol=0, atol=1e-13)


def test_gauge_covariance():
    L = (4, 2, 4, 6)
    U = _rand_su3_field(L, 16)
    g = _rand_su3_field(L, 17)[:, :, :, :, 0]          # one SU(3) matrix per site
    psi = synth.gaussian_spinor(L, 18)
    Ug = np.empty_like(U)
    for mu in range(4):
        g_fwd = lattice.shift_fwd(g, mu, fermion=False)
        Ug[:, :, :, :, mu] = g @ U[:, :, :, :, mu] @ dirac.dagger(g_fwd)
    gpsi = dirac.colour_mul(g, psi)
    for l0 in (None, 2):
        lhs = dirac.apply_op(Ug, gpsi, 0.13, l0)
        rhs = dirac.colour_mul(g, dirac.apply_op(U, psi, 0.13, l0))
        np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-13)


def test_free_field_plane_wave():
    """U = 1: M e^{ipx} u = e^{ipx} [1 - 2k sum cos p + 2ik sum gamma_mu sin p_mu] u with
    p_0 = pi (2 n_0 + 1) / L_0 (antiperiodic) and p_k = 2 pi n_k / L_k."""
    L = (6, 4, 2, 8)
    U = np.zeros(L + (4, 3, 3), complex)
    U[..., :, :] = np.eye(3)
    k = 0.15
    rng = np.random.default_rng(3)
    x = np.meshgrid(*[np.arange(n) for n in L], indexing="ij")
    for n in [(0, 0, 0, 0), (1, 2, 1, 3), (5, 3, 0, 7), (2, 1, 1, 4)]:
        p = [np.pi * (2 * n[0] + 1) / L[0]] + [2 * np.pi * n[i] / L[i] for i in (1, 2, 3)]
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * sum(p[m] * x[m] for m in range(4)))
        psi = phase[..., None, None] * u
        K = (1 - 2 * k * sum(np.cos(pm) for pm in p)) * np.eye(4) \
            + 2j * k * sum(gamma.GAMMA[m] * np.sin(p[m]) for m in range(4))
        expect = phase[..., None, None] * (K @ u)
        np.testing.assert_allclose(dirac.apply_M(U, psi, k), expect, rtol=0, atol=1e-13)


def test_free_field_dense_spectrum():
    """Eigenvalues of the free M on 4^4: 1 - 2k sum cos p +- 2ik sqrt(sum sin^2 p), each
    6-fold (2 spin x 3 colour)."""
    L = L4
    U = np.zeros(L + (4, 3, 3), complex)
    U[..., :, :] = np.eye(3)
    k = 0.155
    ev = np.linalg.eigvals(dirac.dense_matrix(U, k))
    expect = []
    for n in itertools.product(*[range(n) for n in L]):
        p = [np.pi * (2 * n[0] + 1) / L[0]] + [2 * np.pi * n[i] / L[i] for i in (1, 2, 3)]
        re = 1 - 2 * k * sum(np.cos(pm) for pm in p)
        im = 2 * k * np.sqrt(sum(np.sin(pm) ** 2 for pm in p))
        expect += [re + 1j * im] * 6 + [re - 1j * im] * 6
    expect = np.array(expect)
    key = lambda z: np.lexsort((np.round(z.imag, 9), np.round(z.real, 9)))
    np.testing.assert_allclose(ev[key(ev)], expect[key(expect)], rtol=0, atol=1e-11)


@pytest.mark.parametrize("l0", [2, 3, 4])
def test_W_equals_M_with_crossing_links_zeroed(l0):
    L = (12, 2, 4, 2)
    U = _rand_su3_field(L, 19)
    psi = synth.gaussian_spinor(L, 20, nrhs=2)
    Uz = U.copy()
    x0 = np.arange(L[0])
    Uz[(x0 % l0) == l0 - 1, :, :, :, 0] = 0.0
    np.testing.assert_array_equal(dirac.apply_W(U, psi, 0.16, l0), dirac.apply_M(Uz, psi, 0.16))


def test_W_keeps_fields_on_their_block():
    L = (8, 4, 2, 4)
    U = _rand_su3_field(L, 21)
    psi = synth.gaussian_spinor(L, 22)
    for b in range(4):
        m = lattice.site_mask(L, lattice.single_block_mask(L, 2, b))
        out = dirac.apply_W(U, m * psi, 0.2, 2)
        assert np.all(out[~np.broadcast_to(m, out.shape)] == 0)


def test_even_odd_determinant_and_solve_against_dense():
    """det M = det M_hat (Schur complement with a unit diagonal block), and the even-odd
    solve reproduces the dense LU solution of M x = b."""
    L = L4
    U = synth.gauge_field(L, 0.5, 1001)
    k = 0.155
    A = dirac.dense_matrix(U, k)
    e = (lattice.parity(L) == 0)
    ev = np.repeat(e.reshape(-1), 12)
    Ahat = A[np.ix_(ev, ev)] - A[np.ix_(ev, ~ev)] @ A[np.ix_(~ev, ev)]   # diag blocks are 1
    s1, l1 = np.linalg.slogdet(A)
    s2, l2 = np.linalg.slogdet(Ahat)
    assert abs(l1 - l2) < 1e-10 and abs(s1 - s2) < 1e-10
    # The Schur complement is M_hat: compare with the oracle's M_hat on a random even field.
    v = synth.gaussian_spinor(L, 23) * lattice.site_mask(L, e)
    mv = dirac.apply_Mhat(U, v, k)
    np.testing.assert_allclose(mv.reshape(-1)[ev], Ahat @ v.reshape(-1)[ev], atol=1e-13)
    b = synth.gaussian_spinor(L, 2001)
    x_lu = np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)
    x_eo, _, res = solvers.solve_eo(U, b, k, tol=1e-12)
    x_cg, _, res2 = solvers.solve(U, b, k, tol=1e-12)
    cond = np.linalg.cond(A)
    assert res <= 1e-12 and res2 <= 1e-12
    for x in (x_eo, x_cg):
        assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) <= cond * 1e-12


def test_block_solve_and_adjoint_solve_against_dense():
    L = L4
    U = synth.gauge_field(L, 0.5, 1001)
    k = 0.155
    b = synth.gaussian_spinor(L, 2001, nrhs=2)
    for l0, adj in [(2, False), (2, True), (None, True)]:
        A = dirac.dense_matrix(U, k, l0, adj)
        x_lu = np.linalg.solve(A, b.reshape(2, -1).T).T.reshape(b.shape)
        x, _, res = solvers.solve(U, b, k, l0, tol=1e-12, adjoint=adj)
        assert np.all(res <= 1e-12)
        assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) <= np.linalg.cond(A) * 1e-12


def test_block_cg_needs_fewer_iterations_than_full():
    """Sec. 1 claim: the block operator is better conditioned than M. It holds for smooth
    fields (checked here at eps = 0.2, kappa = 0.125); on the rough, uncorrelated synthetic
    fields at kappa = 0.1575 the block system needs more iterations than the full one."""
    L = (16, 4, 4, 4)
    U = synth.gauge_field(L, 0.2, 31)
    b = synth.gaussian_spinor(L, 32)
    _, it_full, _ = solvers.solve_eo(U, b, 0.125, None, tol=1e-10)
    _, it_blk, _ = solvers.solve_eo(U, b, 0.125, 4, tol=1e-10)
    assert it_blk < it_full

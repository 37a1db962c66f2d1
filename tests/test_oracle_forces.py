"""Pins of the oracle's forces by central finite differences of the actions along
U_mu(x) -> exp(i w T^a) U_mu(x) (single link components, dense LU solves on small
lattices) and along a random su(3) direction on a larger lattice (CG solves)."""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import forces, schwarz, solvers, hmc

# Richardson-extrapolated central difference: (4 D(h/2) - D(h)) / 3 has error O(h^4);
# h = 1e-3 keeps the rounding of actions of size ~1e3 below 1e-10.
EPS = 1e-3


def lu_solvers(U, kappa, l0):
    return schwarz.Solvers(
        U, kappa, l0,
        W_inv=solvers.lu_solver(U, kappa, l0), M_inv=solvers.lu_solver(U, kappa, None),
        Mdag_inv=solvers.lu_solver(U, kappa, None, adjoint=True),
        Wdag_inv=solvers.lu_solver(U, kappa, l0, adjoint=True))


def _kick(U, site, mu, a, w):
    """U with U_mu(x) -> exp(i w T^a) U_mu(x), exponential from scipy."""
    V = U.copy()
    V[site + (mu,)] = scipy.linalg.expm(1j * w * forces.T[a]) @ U[site + (mu,)]
    return V


def _fd(action, U, site, mu, a):
    d = lambda h: (action(_kick(U, site, mu, a, h)) - action(_kick(U, site, mu, a, -h))) / (2 * h)
    return (4.0 * d(EPS / 2) - d(EPS)) / 3.0


LINKS = [((0, 1, 0, 1), 0, 0), ((3, 0, 1, 0), 0, 4), ((1, 1, 1, 1), 2, 7), ((2, 0, 1, 1), 3, 2),
         ((1, 0, 0, 1), 0, 5), ((0, 0, 0, 0), 1, 3)]


def test_gauge_force_matches_finite_differences():
    L = (4, 2, 2, 4)
    U = synth.gauge_field(L, 0.5, 41)
    F = forces.gauge_force(U, 5.6)
    for site, mu, a in LINKS:
        fd = _fd(lambda V: forces.gauge_action(V, 5.6), U, site, mu, a)
        assert abs(fd - F[site + (mu, a)]) <= 1e-8 * max(1.0, abs(fd))


@pytest.mark.parametrize("l0", [None, 2])
def test_pseudofermion_force_matches_finite_differences(l0):
    L = (4, 2, 2, 4)
    k = 0.16
    U = synth.gauge_field(L, 0.5, 42)
    phi = synth.gaussian_spinor(L, 43)
    act = lambda V: forces.pf_action(V, phi, k, l0, W_inv=solvers.lu_solver(V, k, l0))
    F = forces.pf_force(U, phi, k, l0, W_inv=solvers.lu_solver(U, k, l0),
                        Wdag_inv=solvers.lu_solver(U, k, l0, adjoint=True))
    for site, mu, a in LINKS:
        fd = _fd(act, U, site, mu, a)
        assert abs(fd - F[site + (mu, a)]) <= 1e-8 * max(1.0, abs(fd)), (site, mu, a)


def test_W1_force_vanishes_on_block_crossing_links():
    L, l0, k = (8, 2, 2, 2), 2, 0.16
    U = synth.gauge_field(L, 0.5, 44)
    phi = synth.gaussian_spinor(L, 45)
    F = forces.pf_force(U, phi, k, l0, W_inv=solvers.lu_solver(U, k, l0),
                        Wdag_inv=solvers.lu_solver(U, k, l0, adjoint=True))
    x0 = np.arange(L[0])
    assert np.all(F[(x0 % l0) == l0 - 1, :, :, :, 0] == 0)
    assert np.any(F[(x0 % l0) != l0 - 1, :, :, :, 0] != 0)


def test_schwarz_force_matches_finite_differences():
    L, l0, k = (8, 2, 2, 2), 2, 0.16
    U = synth.gauge_field(L, 0.5, 46)
    g = synth.noise_spinor(L, 47)
    chi = schwarz.heat_bath(U, g, k, l0, lu_solvers(U, k, l0))
    act = lambda V: schwarz.action(V, chi, k, l0, lu_solvers(V, k, l0))
    F = forces.schwarz_force(U, chi, k, l0, lu_solvers(U, k, l0))
    links = [((3, 1, 0, 1), 0, 1), ((4, 0, 1, 0), 0, 6), ((3, 0, 0, 0), 1, 2),
             ((7, 1, 1, 0), 0, 3), ((5, 0, 1, 1), 2, 0), ((1, 1, 0, 0), 3, 7),
             ((2, 0, 0, 1), 0, 4)]
    for site, mu, a in links:
        fd = _fd(act, U, site, mu, a)
        assert abs(fd - F[site + (mu, a)]) <= 1e-8 * max(1.0, abs(fd)), (site, mu, a, fd)


def test_directional_derivative_with_cg_solves():
    """d/dt S(exp(i t Omega) U) at t = 0 equals sum F^a omega^a for a random su(3) field
    Omega; S = S_G + ||W1^{-1} phi||^2 + S_R on an 8x4^3 lattice with CG solves."""
    L, l0, k, beta = (8, 4, 4, 4), 2, 0.155, 5.6
    U = synth.gauge_field(L, 0.5, 48)
    phi = synth.gaussian_spinor(L, 49)
    omega = synth.gaussian_momenta(L, 50)
    Sv = lambda V: schwarz.Solvers(V, k, l0, tol=1e-13)
    chi = schwarz.heat_bath(U, synth.noise_spinor(L, 51), k, l0, Sv(U))

    def action(V):
        S = Sv(V)
        return forces.gauge_action(V, beta) + forces.pf_action(V, phi, k, l0, W_inv=S.W_inv) \
            + schwarz.action(V, chi, k, l0, S)

    S = Sv(U)
    F = forces.gauge_force(U, beta) + forces.pf_force(U, phi, k, l0, W_inv=S.W_inv,
                                                       Wdag_inv=S.Wdag_inv) \
        + forces.schwarz_force(U, chi, k, l0, S)
    d = lambda h: (action(hmc.T_U(U, omega, h)) - action(hmc.T_U(U, omega, -h))) / (2 * h)
    fd = (4.0 * d(5e-4) - d(1e-3)) / 3.0
    an = float(np.sum(F * omega))
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_force_profile_closed_form():
    """force_profile is the slice mean of the norms |F(x, mu)|: per-slice constant fields
    of known norm, and a slice whose sites alternate between norms 1 and 3 (mean 2, where
    the norm of the mean or the root mean square would give other values)."""
    L = (4, 2, 2, 4)
    rng = np.random.default_rng(5)
    r = rng.uniform(0.5, 2.0, size=(L[0], 4))
    d = rng.normal(size=(L[0], 4, 8))
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    F = np.broadcast_to((r[..., None] * d)[:, None, None, None], L + (4, 8)).copy()
    F[2] = 0.0
    e = np.zeros(8)
    e[3] = 1.0
    sites = np.indices(L[1:]).sum(axis=0) % 2
    F[2, ..., 2, :] = np.where(sites[..., None] == 0, 1.0, 3.0) * e
    P = forces.force_profile(F)
    exp_sp = r[:, 1:].mean(axis=1)
    exp_sp[2] = 2.0 / 3.0
    exp_t = r[:, 0].copy()
    exp_t[2] = 0.0
    assert np.allclose(P[0], exp_sp, rtol=1e-14, atol=0)
    assert np.allclose(P[1], exp_t, rtol=1e-14, atol=0)


def test_schwarz_force_profile_decays_from_block_boundaries():
    """Sec. 4 (plot of the average force on the spatial links against x0): the force of the
    Schwarz term det^2(M W1^{-1}) is largest at the boundaries between the blocks and
    smallest in the middle of a block. Two blocks of l0 = L0/2 as in the paper's first
    decomposition, on a rough field at kappa = 0.13 (short correlation length, so the decay
    is clean): the spatial profile falls strictly from each block boundary to the block's
    middle, by more than a factor 100."""
    L, l0, k = (16, 4, 4, 4), 8, 0.13
    U = synth.gauge_field(L, 0.5, 61)
    S = schwarz.Solvers(U, k, l0, tol=1e-11)
    chi = schwarz.heat_bath(U, synth.noise_spinor(L, 62), k, l0, S)
    sp = forces.force_profile(forces.schwarz_force(U, chi, k, l0, S))[0]
    for b0 in range(0, L[0], l0):
        first, last, mid = b0, b0 + l0 - 1, b0 + l0 // 2
        down = sp[first:mid]                  # boundary -> middle from the first slice
        up = sp[mid - 1:last + 1]              # middle -> boundary at the last slice
        assert np.all(np.diff(down) < 0), sp
        assert np.all(np.diff(up[::-1][:l0 // 2]) < 0), sp
        assert min(sp[first], sp[last]) > 100 * min(sp[mid - 1], sp[mid]), sp

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
    """Sec. 3, Fig. 1 (plot of the average force on the spatial links against x0): the force of the
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


# ---- pins of the gauge action and the mean plaquette (Sec. 1, Wilson plaquette action) ----

def _random_su3(n, rng):
    """n Haar-ish SU(3) matrices from the QR decomposition of complex Gaussian matrices,
    phases fixed so that det = 1 (independent of the oracle and of synth)."""
    Z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    Q, R = np.linalg.qr(Z)
    d = np.diagonal(R, axis1=-2, axis2=-1)
    Q = Q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(Q)
    return Q / (det ** (1.0 / 3.0))[:, None, None]


def test_gauge_action_is_gauge_invariant():
    """S_G[U^g] = S_G[U] with U_mu(x) -> g(x) U_mu(x) g(x + mu)^dagger for a random SU(3)
    g per site: a plaquette with a misplaced dagger or a wrong shift is not invariant."""
    L = (4, 4, 2, 6)
    U = synth.gauge_field(L, 0.6, 51)
    rng = np.random.default_rng(52)
    g = _random_su3(int(np.prod(L)), rng).reshape(tuple(L) + (3, 3))
    assert np.max(np.abs(g @ np.swapaxes(g.conj(), -1, -2) - np.eye(3))) < 1e-13
    Ug = np.empty_like(U)
    for mu in range(4):
        g_next = np.roll(g, -1, axis=mu)                   # g(x + mu), periodic links
        Ug[..., mu, :, :] = g @ U[..., mu, :, :] @ np.swapaxes(g_next.conj(), -1, -2)
    s0, s1 = forces.gauge_action(U, 5.6), forces.gauge_action(Ug, 5.6)
    assert abs(s1 - s0) <= 1e-12 * abs(s0)
    assert abs(forces.mean_plaquette(Ug) - forces.mean_plaquette(U)) <= 1e-13


def test_unit_links_give_plaquette_one_and_action_minus_6_beta_V():
    """U = 1: every Re Tr U_P = 3, so <P> = 1 and S_G = -(beta/3) * 6V * 3 = -6 beta V."""
    L = (4, 2, 6, 2)
    V = int(np.prod(L))
    U = np.broadcast_to(np.eye(3, dtype=complex), tuple(L) + (4, 3, 3)).copy()
    assert forces.mean_plaquette(U) == pytest.approx(1.0, abs=1e-15)
    assert forces.gauge_action(U, 5.6) == pytest.approx(-6.0 * 5.6 * V, rel=1e-15)


def test_constant_abelian_flux_closed_form():
    """A constant U(1) flux through the (1, 2) planes embedded in SU(3):
    U_2(x) = diag(e^{iBx1}, e^{-iBx1}, 1), every other link 1, B = 2 pi n / L1 (periodic).
    Each (1, 2) plaquette is diag(e^{+-iB}, e^{-+iB}, 1), Re Tr = 1 + 2 cos B, and the
    other five planes give 3, so <P> = (15 + 1 + 2 cos B) / 18 and
    S_G = -(beta/3) V (16 + 2 cos B)."""
    L = (2, 6, 4, 2)
    V = int(np.prod(L))
    U = np.broadcast_to(np.eye(3, dtype=complex), tuple(L) + (4, 3, 3)).copy()
    B = 2.0 * np.pi * 1 / L[1]
    x1 = np.arange(L[1])[None, :, None, None]
    ph = np.exp(1j * B * x1) * np.ones(L)
    U[..., 2, 0, 0] = ph
    U[..., 2, 1, 1] = ph.conj()
    assert forces.mean_plaquette(U) == pytest.approx((16.0 + 2.0 * np.cos(B)) / 18.0, abs=1e-14)
    assert forces.gauge_action(U, 5.6) == pytest.approx(-5.6 / 3.0 * V * (16.0 + 2.0 * np.cos(B)), rel=1e-14)


def test_synthetic_mean_plaquette_is_c_to_the_fourth():
    """For independent links whose distribution is invariant under conjugation and
    under H -> -H, E[U] = c 1 with c = E[(1/3) Re Tr exp(i eps H)], and the expected
    mean plaquette is c^4 (each plaquette is a product of four independent links or their
    adjoints). c is estimated from 200 000 independently drawn H (eigenvalues of H only,
    no plaquette code); the oracle's <P> on an 8^4 field must lie within 5 standard
    errors of c^4 (the standard error from the spread of the per-site plaquettes)."""
    eps = 0.35
    rng = np.random.default_rng(53)
    A = rng.standard_normal((200000, 3, 3)) + 1j * rng.standard_normal((200000, 3, 3))
    H = 0.5 * (A + np.swapaxes(A.conj(), -1, -2))
    H = H - (np.trace(H, axis1=-2, axis2=-1).real / 3.0)[:, None, None] * np.eye(3)
    c = float(np.mean(np.cos(eps * np.linalg.eigvalsh(H)).sum(axis=-1)) / 3.0)
    L = (8, 8, 8, 8)
    U = synth.gauge_field(L, eps, 54)
    per_site = forces.plaquette_field(U) / 18.0            # six planes, (1/3) Re Tr each
    P = forces.mean_plaquette(U)
    assert P == pytest.approx(float(per_site.mean()), abs=1e-14)
    se = float(per_site.std()) / np.sqrt(per_site.size)
    assert abs(P - c ** 4) <= 5.0 * se, (P, c ** 4, se)
    assert 0.50 < c ** 4 < 0.52                            # the 0.509 of the workload recipe

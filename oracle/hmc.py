"""Molecular dynamics and the HMC trajectory (oracle, FP64).

Sec. 2, eq. 3: T_U(dt): U -> exp(i dt P) U and T_{P,j}(dt): P -> P - dt F_j, with
P = sum_a p^a T^a Hermitian traceless and F_j the force of action part S_j
(``forces`` module convention).
Sec. 2, eq. 4: leap-frog  T_LF,0(dt) = T_P,0(dt/2) T_U(dt) T_P,0(dt/2).
Sec. 2, eq. swimp: Sexton-Weingarten
    T_SW,0(dt) = T_P,0(l dt) T_U(dt/2) T_P,0((1-2l) dt) T_U(dt/2) T_P,0(l dt), l = 1/6.
Sec. 2, eqs. iterateLF / iterateSW: level j replaces T_U by n_{j-1} steps (SW: two runs of
n_{j-1}/2 steps) of level j-1 with dt_{j-1} = dt_j / n_{j-1}; a trajectory of length tau
is n_J steps of the top level J.
Metropolis (Sec. 3, P_acc): accept with probability min(1, exp(-dH)),
H = 1/2 sum p^2 + sum_j S_j.
"""
import numpy as np

from .forces import T

LAMBDA_SW = 1.0 / 6.0


def su3_algebra(p):
    """P = sum_a p^a T^a, shape [..., 3, 3]."""
    return np.einsum("...a,aij->...ij", p, T)


def exp_iP(p, dt):
    """exp(i dt P) via the eigen-decomposition of the Hermitian matrix P."""
    P = su3_algebra(p)
    w, v = np.linalg.eigh(P)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * dt * w), v.conj())


def T_U(U, p, dt):
    return exp_iP(p, dt) @ U


def kinetic(p):
    return 0.5 * float(np.sum(p * p))


class Level:
    """One action part S_j integrated on its own time scale: ``force(U)``, ``action(U)``,
    scheme 'LF' or 'SW', and n = number of its steps inside one step of the level above
    (for the top level: steps per trajectory)."""

    def __init__(self, force, action, scheme, n):
        self.force, self.action, self.scheme, self.n = force, action, scheme, n


def _inner(levels, j, U, p, dt):
    """What sits between the two half kicks of a leap-frog level j: T_U(dt) for j = 0,
    else n_{j-1} steps of level j-1 of length dt / n_{j-1}."""
    if j == 0:
        return T_U(U, p, dt), p
    nlow = levels[j - 1].n
    for _ in range(nlow):
        U, p = step(levels, j - 1, U, p, dt / nlow)
    return U, p


def step(levels, j, U, p, dt):
    lev = levels[j]
    if lev.scheme == "LF":
        p = p - 0.5 * dt * lev.force(U)
        U, p = _inner(levels, j, U, p, dt)
        p = p - 0.5 * dt * lev.force(U)
    elif lev.scheme == "SW":
        lam = LAMBDA_SW
        p = p - lam * dt * lev.force(U)
        if j == 0:
            U = T_U(U, p, 0.5 * dt)
        else:
            U, p = _half(levels, j, U, p, dt)
        p = p - (1 - 2 * lam) * dt * lev.force(U)
        if j == 0:
            U = T_U(U, p, 0.5 * dt)
        else:
            U, p = _half(levels, j, U, p, dt)
        p = p - lam * dt * lev.force(U)
    else:
        raise ValueError(lev.scheme)
    return U, p


def _half(levels, j, U, p, dt):
    """[T_X,j-1(dt_{j-1})]^{n_{j-1}/2} with dt_{j-1} = dt / n_{j-1}."""
    nlow = levels[j - 1].n
    if nlow % 2:
        raise ValueError("an SW level needs an even step count below it")
    for _ in range(nlow // 2):
        U, p = step(levels, j - 1, U, p, dt / nlow)
    return U, p


def integrate(levels, U, p, tau):
    """n_J steps of the top level, dt_J = tau / n_J."""
    J = len(levels) - 1
    dt = tau / levels[J].n
    for _ in range(levels[J].n):
        U, p = step(levels, J, U, p, dt)
    return U, p


def hamiltonian(levels, U, p):
    return kinetic(p) + sum(lev.action(U) for lev in levels)


def trajectory(levels, U, p0, tau, u_metropolis):
    """One HMC trajectory from (U, p0): returns (U_out, accepted, dH, H0, H1)."""
    H0 = hamiltonian(levels, U, p0)
    U1, p1 = integrate(levels, U, p0, tau)
    H1 = hamiltonian(levels, U1, p1)
    dH = H1 - H0
    acc = u_metropolis < np.exp(-dH)
    return (U1 if acc else U), bool(acc), dH, H0, H1


def schwarz_two_level(phi1, chi, kappa, beta, l0, n_outer, n_inner, make_solvers,
                      scheme_outer="SW", scheme_inner="SW"):
    """Two time scales: level 0 = Wilson gauge action S_G (n_inner steps per outer step),
    level 1 = S_pf = ||W1^{-1} phi1||^2 + ||R_hat^{-1} chi||^2 (n_outer steps per
    trajectory). This is the two-factor form M = (M W1^{-1}) W1 of the factorised
    pseudo-fermion action (Sec. 1, eq. factorpf): det M^2 = det W1^2 det R_hat^2.
    ``make_solvers(U)`` returns a ``schwarz.Solvers`` for the current links."""
    from . import forces, schwarz

    def pf_force(U):
        S = make_solvers(U)
        f1 = forces.pf_force(U, phi1, kappa, l0, W_inv=S.W_inv,
                             Wdag_inv=getattr(S, "Wdag_inv", None))
        return f1 + forces.schwarz_force(U, chi, kappa, l0, S)

    def pf_action(U):
        S = make_solvers(U)
        return forces.pf_action(U, phi1, kappa, l0, W_inv=S.W_inv) \
            + schwarz.action(U, chi, kappa, l0, S)

    return [
        Level(lambda U: forces.gauge_force(U, beta), lambda U: forces.gauge_action(U, beta),
              scheme_inner, n_inner),
        Level(pf_force, pf_action, scheme_outer, n_outer),
    ]

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
x0-dependent step size (Sec. 2): every link moves with dt * s_mu(x0) in both T_U and T_P
(s = 0: the link stays fixed); schemes A, B, C are the paper's periodic tables, separate
for space-like and time-like links. After a trajectory the configuration may be
translated in x0 (Sec. 2, ergodicity).
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


def T_U(U, p, dt, scale=None):
    """U <- exp(i dt s P) U; ``scale`` (shape [L0, 4]) gives s_mu(x0), default 1."""
    if scale is not None:
        p = p * scale[:, None, None, None, :, None]
    return exp_iP(p, dt) @ U


def kick(p, F, dt, scale=None):
    """p <- p - dt s F."""
    if scale is not None:
        F = F * scale[:, None, None, None, :, None]
    return p - dt * F


# Sec. 2, schemes (A) L0 = 24, (B) and (C) L0 = 32: s(x0) for space-like and time-like
# links over one period; scheme A's spatial x0 = 5 entry read as 0.2 (printed: 2).
STEP_SCHEMES = {
    "A": ([0.2, 0.5, 1, 1, 0.5, 0.2], [0.2, 0.5, 1, 0.5, 0.2, 0]),
    "B": ([0, 0.5, 1, 1, 1, 1, 0.5, 0], [0, 0.5, 1, 1, 1, 0.5, 0, 0]),
    "C": ([0, 0.25, 0.5, 1, 1, 1, 1, 0.25, 0.25, 1, 1, 1, 1, 0.5, 0.25, 0],
          [0, 0, 0.25, 0.5, 1, 1, 0.25, 0, 0.25, 1, 1, 1, 0.5, 0.25, 0, 0]),
}


def step_profile(scheme, L0):
    """s_mu(x0) as an array [L0, 4] (mu = 0 time-like, 1..3 space-like), the scheme's
    table repeated with its period."""
    sp, tm = STEP_SCHEMES[scheme]
    per = len(sp)
    if L0 % per:
        raise ValueError("L0 must be a multiple of the scheme's period")
    s = np.zeros((L0, 4))
    for x0 in range(L0):
        s[x0, 0] = tm[x0 % per]
        s[x0, 1:] = sp[x0 % per]
    return s


def time_shift(U, n):
    """The configuration translated by n slices in x0: U'(x0, ...) = U(x0 + n, ...)."""
    return np.roll(U, -n, axis=0)


def kinetic(p):
    return 0.5 * float(np.sum(p * p))


class Level:
    """One action part S_j integrated on its own time scale: ``force(U)``, ``action(U)``,
    scheme 'LF' or 'SW', and n = number of its steps inside one step of the level above
    (for the top level: steps per trajectory)."""

    def __init__(self, force, action, scheme, n):
        self.force, self.action, self.scheme, self.n = force, action, scheme, n


def _inner(levels, j, U, p, dt, sc):
    """What sits between the two half kicks of a leap-frog level j: T_U(dt) for j = 0,
    else n_{j-1} steps of level j-1 of length dt / n_{j-1}."""
    if j == 0:
        return T_U(U, p, dt, sc), p
    nlow = levels[j - 1].n
    for _ in range(nlow):
        U, p = step(levels, j - 1, U, p, dt / nlow, sc)
    return U, p


def step(levels, j, U, p, dt, sc=None):
    lev = levels[j]
    if lev.scheme == "LF":
        p = kick(p, lev.force(U), 0.5 * dt, sc)
        U, p = _inner(levels, j, U, p, dt, sc)
        p = kick(p, lev.force(U), 0.5 * dt, sc)
    elif lev.scheme == "SW":
        lam = LAMBDA_SW
        p = kick(p, lev.force(U), lam * dt, sc)
        if j == 0:
            U = T_U(U, p, 0.5 * dt, sc)
        else:
            U, p = _half(levels, j, U, p, dt, sc)
        p = kick(p, lev.force(U), (1 - 2 * lam) * dt, sc)
        if j == 0:
            U = T_U(U, p, 0.5 * dt, sc)
        else:
            U, p = _half(levels, j, U, p, dt, sc)
        p = kick(p, lev.force(U), lam * dt, sc)
    else:
        raise ValueError(lev.scheme)
    return U, p


def _half(levels, j, U, p, dt, sc):
    """[T_X,j-1(dt_{j-1})]^{n_{j-1}/2} with dt_{j-1} = dt / n_{j-1}."""
    nlow = levels[j - 1].n
    if nlow % 2:
        raise ValueError("an SW level needs an even step count below it")
    for _ in range(nlow // 2):
        U, p = step(levels, j - 1, U, p, dt / nlow, sc)
    return U, p


def integrate(levels, U, p, tau, scale=None):
    """n_J steps of the top level, dt_J = tau / n_J; ``scale`` = s_mu(x0) [L0, 4]."""
    J = len(levels) - 1
    dt = tau / levels[J].n
    for _ in range(levels[J].n):
        U, p = step(levels, J, U, p, dt, scale)
    return U, p


def hamiltonian(levels, U, p):
    return kinetic(p) + sum(lev.action(U) for lev in levels)


def trajectory(levels, U, p0, tau, u_metropolis, scale=None, shift=0):
    """One HMC trajectory from (U, p0): returns (U_out, accepted, dH, H0, H1); U_out is
    translated by ``shift`` slices in x0 after the accept / reject step."""
    H0 = hamiltonian(levels, U, p0)
    U1, p1 = integrate(levels, U, p0, tau, scale)
    H1 = hamiltonian(levels, U1, p1)
    dH = H1 - H0
    acc = u_metropolis < np.exp(-dH)
    Uo = U1 if acc else U
    return (time_shift(Uo, shift) if shift else Uo), bool(acc), dH, H0, H1


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

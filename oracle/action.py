"""The paper's four-part pseudo-fermion action and its five-level integration (oracle,
FP64; test infrastructure only).

Sec. 1, end: with W_i the Wilson operator restricted to x0 blocks of length l0^(i)
(l0^(2) = l0^(1) / 2), W_{2,eo} the even-odd reduced W_2 and W_{3,eo} = W_{2,eo} + rho
(mass preconditioning), the two-flavour determinant factorises as
    det^2 M = det^2(M W1^-1) det^2(W1 W2^-1) det^2(W_{2,eo} W_{3,eo}^-1) det^2(W_{3,eo}),
and the parts S4, S3, S2, S1 represent these factors (note the reversed labels); S0 is
the gauge action. Pseudo-fermion representations used here:
    S4 = ||R_hat^-1 chi4||^2        Schwarz term of (M, W1): chi4 on black level-1 block
                                    boundaries (oracle.schwarz, outer = M)
    S3 = ||R_hat_2^-1 chi3||^2      the same with (W1, W2): chi3 on the interface inside
                                    every level-1 block (oracle.schwarz, outer = l0^(1))
    S2 = ||W2eo^-1 W3eo phi2||^2 = ||phi2 + rho W2eo^-1 phi2||^2
    S1 = ||W3eo^-1 phi1||^2         phi1, phi2 on the even sites
with heat baths chi4 = R_hat Pi g4, chi3 = R_hat_2 Pi_2 g3, phi2 = W3eo^-1 W2eo xi2,
phi1 = W3eo xi1, so that S_j equals the squared noise at the heat bath.

Forces (dW_eo = -k^2 P_e (dD P_o D + D P_o dD) P_e, and 2 Re <a, dD b> = -pair_force/k):
    S1: X = W3eo^-1 phi1, Z = W3eo^-dag X,
        F = -2 Re <Z, dW_eo X> = -k [pf(Z, P_o D X) + pf(P_o D^dag Z, X)]
    S2: Y = W2eo^-1 phi2, X = phi2 + rho Y, Z = W2eo^-dag X,
        F = -2 rho Re <Z, dW_eo Y> = -rho k [pf(Z, P_o D Y) + pf(P_o D^dag Z, Y)]
with D the hop restricted to the level-2 blocks and pf = oracle.forces.pair_force.

Integration (Sec. 2): level j integrates S_j; leap-frog for j = 2, 3, 4 and the
Sexton-Weingarten step for j = 0, 1; n_j steps of level j inside one step of level j + 1
(n_4 per trajectory), as in Table 1.
"""
import numpy as np

from .dirac import apply_Mhat, hop, parity_masks
from . import forces, hmc, schwarz, solvers


class FourPart:
    """Operators, solves, actions, forces and heat baths of S1 .. S4 on one gauge field.
    l0 = l0^(1), l0s = l0^(2); tol for the CGLS solves (dense LU may be passed for the
    Schwarz parts through ``sz4`` / ``sz3``)."""

    def __init__(self, U, kappa, l0, l0s, rho, tol=1e-12, sz4=None, sz3=None):
        self.U, self.k, self.l0, self.l0s, self.rho, self.tol = U, kappa, l0, l0s, rho, tol
        L = U.shape[:4]
        self.e, self.o = parity_masks(L)
        self.sz4 = sz4 or schwarz.Solvers(U, kappa, l0, tol=tol)
        self.sz3 = sz3 or schwarz.Solvers(U, kappa, l0s, tol=tol, outer=l0)

    # even-odd operators on the level-2 blocks
    def W2eo(self, v, adjoint=False):
        return apply_Mhat(self.U, v, self.k, self.l0s, adjoint)

    def W3eo(self, v, adjoint=False):
        return self.W2eo(v, adjoint) + self.rho * (self.e * v)

    def _solve(self, op, b):
        x, _, res = solvers.cgls(lambda v: op(v, False), lambda v: op(v, True), b, tol=self.tol)
        return x

    def _solve_dag(self, op, b):
        x, _, res = solvers.cgls(lambda v: op(v, True), lambda v: op(v, False), b, tol=self.tol)
        return x

    def _eo_pair(self, Z, X):
        """2 Re <Z, dW_eo X> as a force field (the two pair terms)."""
        D = lambda v, adj=False: hop(self.U, v, self.l0s, adj)
        a = forces.pair_force(self.U, Z, self.o * D(X), self.k, self.l0s)
        b = forces.pair_force(self.U, self.o * D(Z, True), X, self.k, self.l0s)
        return self.k * (a + b)

    # S1 = ||W3eo^-1 phi1||^2
    def S1(self, phi1):
        return float(np.sum(np.abs(self._solve(self.W3eo, phi1)) ** 2))

    def F1(self, phi1):
        X = self._solve(self.W3eo, phi1)
        Z = self._solve_dag(self.W3eo, X)
        return -self._eo_pair(Z, X)

    def heat_bath1(self, xi1):
        return self.W3eo(self.e * xi1)

    # S2 = ||phi2 + rho W2eo^-1 phi2||^2
    def S2(self, phi2):
        X = phi2 + self.rho * self._solve(self.W2eo, phi2)
        return float(np.sum(np.abs(X) ** 2))

    def F2(self, phi2):
        Y = self._solve(self.W2eo, phi2)
        X = phi2 + self.rho * Y
        Z = self._solve_dag(self.W2eo, X)
        return -self.rho * self._eo_pair(Z, Y)

    def heat_bath2(self, xi2):
        return self._solve(self.W3eo, self.W2eo(self.e * xi2))

    # S3: Schwarz term of (W1, W2); S4: Schwarz term of (M, W1)
    def S3(self, chi3):
        return schwarz.action(self.U, chi3, self.k, self.l0s, self.sz3, outer=self.l0)

    def F3(self, chi3):
        return forces.schwarz_force(self.U, chi3, self.k, self.l0s, self.sz3, outer=self.l0)

    def heat_bath3(self, g3):
        L = self.U.shape[:4]
        return schwarz.heat_bath(self.U, g3, self.k, self.l0s, self.sz3, outer=self.l0)

    def S4(self, chi4):
        return schwarz.action(self.U, chi4, self.k, self.l0, self.sz4)

    def F4(self, chi4):
        return forces.schwarz_force(self.U, chi4, self.k, self.l0, self.sz4)

    def heat_bath4(self, g4):
        return schwarz.heat_bath(self.U, g4, self.k, self.l0, self.sz4)


def five_level(fields, kappa, beta, l0, l0s, rho, n, make=None):
    """Levels 0 .. 4 of the paper's integrator for pseudo-fermion fields
    fields = (phi1, phi2, chi3, chi4): gauge action (SW), S1 (SW), S2, S3, S4 (LF);
    n = (n0, n1, n2, n3, n4). make(U) -> FourPart (default CGLS solves)."""
    phi1, phi2, chi3, chi4 = fields
    make = make or (lambda U: FourPart(U, kappa, l0, l0s, rho))
    return [
        hmc.Level(lambda U: forces.gauge_force(U, beta), lambda U: forces.gauge_action(U, beta), "SW", n[0]),
        hmc.Level(lambda U: make(U).F1(phi1), lambda U: make(U).S1(phi1), "SW", n[1]),
        hmc.Level(lambda U: make(U).F2(phi2), lambda U: make(U).S2(phi2), "LF", n[2]),
        hmc.Level(lambda U: make(U).F3(chi3), lambda U: make(U).S3(chi3), "LF", n[3]),
        hmc.Level(lambda U: make(U).F4(chi4), lambda U: make(U).S4(chi4), "LF", n[4]),
    ]

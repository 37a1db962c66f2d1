"""Krylov solvers of the oracle (FP64).

The paper solves its action parts with the geometric series and with BiCGstab (Sec. 3:
geometric series for the block terms, BiCGstab with even-odd and Schwarz preconditioning
for the full-lattice term) but fixes neither a stopping rule nor a precision. Every
solver here starts from x = 0 and stops on ||b - A x|| / ||b|| <= tol with the residual
recomputed from A at the end (restarting from the current x if the recomputed one is not
yet below tol).

* ``cgls``: the textbook CG on the normal equations A^dagger A x = A^dagger b in its CGLS
  form (Hestenes-Stiefel; the residual s = b - A x of the original system is carried).
* ``bicgstab``: van der Vorst's BiCGstab (1992) with shadow residual r0 and an optional
  right preconditioner K (A K y = b, x = K y).
* ``sap_precond``: the Schwarz alternating procedure on the x0 blocks (black blocks,
  then white blocks, ncy cycles; block systems solved with ``solve_eo``), the Schwarz
  preconditioner of the full-lattice solve.
* ``geometric_series``: W x = b in the even-odd form, x_e = sum_n (k^2 D_eo D_oe)^n b_hat,
  stopped when the last term is below tol ||b|| (the residual of the partial sum is the
  next term).
* ``geometric_series_eo``: the same series for the even-site system (M_hat + rho) x = b of
  the mass-preconditioned action parts (Sec. 1, end: W3eo = W2eo + rho), whose terms carry
  the factor 1 / (1 + rho) each.

Leading batch axes are independent systems with their own scalars.
"""
import numpy as np

from .dirac import apply_op, apply_Mhat, parity_masks, hop


def _norm2(f: np.ndarray) -> np.ndarray:
    """Per-system ||f||^2 with the batch axes kept (keepdims over the 6 field axes)."""
    return np.sum(np.abs(f) ** 2, axis=tuple(range(f.ndim - 6, f.ndim)), keepdims=True)


def cgls(A, Adag, b, tol=1e-12, maxiter=20000, max_restarts=5):
    """Solve A x = b. Returns (x, iterations, true relative residual per system)."""
    bn = np.sqrt(_norm2(b))
    bn_safe = np.where(bn == 0, 1.0, bn)
    x = np.zeros_like(b)
    its = 0
    for _ in range(max_restarts + 1):
        s = b - A(x)
        r = Adag(s)
        p = r.copy()
        gam = _norm2(r)
        for _ in range(maxiter):
            done = np.sqrt(_norm2(s)) <= tol * bn_safe
            if np.all(done):
                break
            q = A(p)
            qq = _norm2(q)
            alpha = np.where(done | (qq == 0), 0.0, gam / np.where(qq == 0, 1.0, qq))
            x = x + alpha * p
            s = s - alpha * q
            r = Adag(s)
            gnew = _norm2(r)
            beta = np.where(done | (gam == 0), 0.0, gnew / np.where(gam == 0, 1.0, gam))
            p = r + beta * p
            gam = gnew
            its += 1
        res = np.sqrt(_norm2(b - A(x))) / bn_safe
        if np.all(res <= tol):
            break
    return x, its, res.reshape(res.shape[:-6]) if res.ndim > 6 else float(res.reshape(()))


def solve(U, b, kappa, l0=None, tol=1e-12, adjoint=False, maxiter=20000):
    """x with op x = b for op = M (l0 None) or W_l0 (op^dagger with ``adjoint``), CGLS on
    the full lattice."""
    A = lambda v: apply_op(U, v, kappa, l0, adjoint)
    Ad = lambda v: apply_op(U, v, kappa, l0, not adjoint)
    return cgls(A, Ad, b, tol=tol, maxiter=maxiter)


def solve_eo(U, b, kappa, l0=None, tol=1e-12, maxiter=20000):
    """Even-odd reduced solve (Sec. 1, W_eo): M_hat x_e = b_e + kappa D_eo b_o by CGLS on
    M_hat, then x_o = b_o + kappa D_oe x_e. Stops on the relative residual of the full
    system op x = b."""
    L = U.shape[:4]
    e, o = parity_masks(L)
    bhat = e * (b + kappa * hop(U, o * b, l0))
    A = lambda v: apply_Mhat(U, v, kappa, l0, False)
    Ad = lambda v: apply_Mhat(U, v, kappa, l0, True)
    bn = np.sqrt(_norm2(b))
    tol_hat = tol
    for _ in range(4):
        xe, its, _ = cgls(A, Ad, bhat, tol=tol_hat, maxiter=maxiter)
        x = xe + o * (b + kappa * hop(U, xe, l0))
        res = np.sqrt(_norm2(b - apply_op(U, x, kappa, l0))) / np.where(bn == 0, 1.0, bn)
        if np.all(res <= tol):
            break
        tol_hat *= 0.1
    res = res.reshape(res.shape[:-6]) if res.ndim > 6 else float(res.reshape(()))
    return x, its, res


def lu_solver(U, kappa, l0=None, adjoint=False):
    """Dense LU solve on tiny lattices (numpy.linalg.solve on the dense matrix)."""
    from .dirac import dense_matrix
    cache = []

    def f(b):
        if not cache:                       # build the matrix on first use
            cache.append(dense_matrix(U, kappa, l0, adjoint))
        Mat = cache[0]
        shp = b.shape
        n = Mat.shape[0]
        B = b.reshape(-1, n).T
        X = np.linalg.solve(Mat, B)
        return X.T.reshape(shp)
    return f


def _dot(a, b):
    """Per-system <a, b> = sum conj(a) b (keepdims over the 6 field axes)."""
    return np.sum(np.conj(a) * b, axis=tuple(range(a.ndim - 6, a.ndim)), keepdims=True)


def bicgstab(A, b, tol=1e-12, maxiter=20000, K=None, max_restarts=5):
    """Solve A x = b by BiCGstab (van der Vorst 1992), right-preconditioned by K if given.
    Returns (x, iterations, true relative residual per system). Systems that reach tol
    are frozen (alpha = omega = 0) while the others continue."""
    K = (lambda v: v) if K is None else K
    bn = np.sqrt(_norm2(b))
    bn_safe = np.where(bn == 0, 1.0, bn)
    x = np.zeros_like(b)
    its = 0
    for _ in range(max_restarts + 1):
        r = b - A(x)
        r0 = r.copy()
        rho = np.ones(_dot(r, r).shape, dtype=complex)
        alpha = np.ones_like(rho)
        omega = np.ones_like(rho)
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        for _ in range(maxiter):
            act = np.sqrt(_norm2(r)) > tol * bn_safe
            if not np.any(act):
                break
            rho_new = _dot(r0, r)
            beta = np.where(act, (rho_new / np.where(act, rho, 1.0)) * (alpha / np.where(act, omega, 1.0)), 0.0)
            p = r + beta * (p - omega * v)
            ph = K(p)
            v = A(ph)
            den = _dot(r0, v)
            alpha = np.where(act, rho_new / np.where(act, den, 1.0), 0.0)
            s = r - alpha * v
            sh = K(s)
            t = A(sh)
            tt = _dot(t, t)
            omega = np.where(act & (tt != 0), _dot(t, s) / np.where(tt == 0, 1.0, tt), 0.0)
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            rho = np.where(act, rho_new, rho)
            its += 1
        res = np.sqrt(_norm2(b - A(x))) / bn_safe
        if np.all(res <= tol):
            break
    return x, its, res.reshape(res.shape[:-6]) if res.ndim > 6 else float(res.reshape(()))


def solve_eo_bicgstab(U, b, kappa, l0=None, tol=1e-12, maxiter=20000):
    """Even-odd reduced solve of op x = b (op = M, or W_l0 for l0 given) with BiCGstab on
    M_hat x_e = b_e + kappa D_eo b_o, then x_o = b_o + kappa D_oe x_e."""
    L = U.shape[:4]
    e, o = parity_masks(L)
    bhat = e * (b + kappa * hop(U, o * b, l0))
    A = lambda v: apply_Mhat(U, v, kappa, l0, False)
    bn = np.sqrt(_norm2(b))
    tol_hat = tol
    for _ in range(4):
        xe, its, _ = bicgstab(A, bhat, tol=tol_hat, maxiter=maxiter)
        x = xe + o * (b + kappa * hop(U, xe, l0))
        res = np.sqrt(_norm2(b - apply_op(U, x, kappa, l0))) / np.where(bn == 0, 1.0, bn)
        if np.all(res <= tol):
            break
        tol_hat *= 0.1
    res = res.reshape(res.shape[:-6]) if res.ndim > 6 else float(res.reshape(()))
    return x, its, res


def sap_precond(U, r, kappa, l0, ncy, block_tol=1e-12, block_terms=0):
    """ncy cycles of the multiplicative Schwarz alternating procedure for M x = r on the x0
    blocks of length l0: for the black blocks, then the white blocks, add the solution of
    the block system W_l0 y = (r - M x) restricted to the blocks of that colour (W_l0 is
    block diagonal, so y stays on those blocks). Block systems: ``solve_eo`` to
    block_tol, or, with block_terms = N > 0, the first N terms of their even-odd geometric
    series (``geometric_series`` with no stopping test), which makes every cycle a fixed
    linear map of r."""
    from .lattice import site_mask, colour_x0_mask
    L = U.shape[:4]
    x = np.zeros_like(r)
    for _ in range(ncy):
        for colour in ("black", "white"):
            m = site_mask(L, colour_x0_mask(L, l0, colour))
            rho = (r - apply_op(U, x, kappa)) * m
            if block_terms > 0:
                y, _, _ = geometric_series(U, rho, kappa, l0, tol=0.0, maxiter=block_terms)
            else:
                y, _, _ = solve_eo(U, rho, kappa, l0, tol=block_tol)
            x = x + y
    return x


def solve_sap_bicgstab(U, b, kappa, l0, ncy=1, tol=1e-12, block_tol=1e-12, maxiter=2000, block_terms=0):
    """M x = b by BiCGstab on the full lattice, right-preconditioned by ncy Schwarz
    cycles (``sap_precond``) whose block systems are solved in the even-odd form."""
    A = lambda v: apply_op(U, v, kappa)
    K = lambda v: sap_precond(U, v, kappa, l0, ncy, block_tol, block_terms)
    return bicgstab(A, b, tol=tol, maxiter=maxiter, K=K)


def geometric_series(U, b, kappa, l0=None, tol=1e-12, maxiter=100000):
    """op x = b (op = M, or W_l0) by the geometric (Neumann) series of the even-odd
    reduced system: M_hat = 1 - kappa^2 D_eo D_oe, so
        x_e = sum_{n >= 0} t_n,  t_0 = b_hat = b_e + kappa D_eo b_o,
        t_{n+1} = kappa^2 D_eo D_oe t_n,
    then x_o = b_o + kappa D_oe x_e. After summing t_0 .. t_N the residual of op x = b is
    t_{N+1} on the even sites and zero on the odd ones, so the sum stops at the first
    term with ||t_{N+1}|| <= tol ||b|| (per system). Returns (x, terms added, true
    relative residual); the series diverges when the spectral radius of
    kappa^2 D_eo D_oe exceeds one, reported as a residual above tol after maxiter."""
    L = U.shape[:4]
    e, o = parity_masks(L)
    t = e * (b + kappa * hop(U, o * b, l0))
    bn = np.sqrt(_norm2(b))
    xe = np.zeros_like(b)
    n = 0
    for _ in range(maxiter):
        xe = xe + t
        n += 1
        t = kappa * kappa * (e * hop(U, o * hop(U, t, l0), l0))
        if np.all(np.sqrt(_norm2(t)) <= tol * bn) or not np.all(np.isfinite(t)):
            break
    x = xe + o * (b + kappa * hop(U, xe, l0))
    res = np.sqrt(_norm2(b - apply_op(U, x, kappa, l0))) / np.where(bn == 0, 1.0, bn)
    res = res.reshape(res.shape[:-6]) if res.ndim > 6 else float(res.reshape(()))
    return x, n, res


def geometric_series_eo(U, b, kappa, l0=None, rho=0.0, tol=1e-12, maxiter=100000, adjoint=False):
    """(M_hat + rho) x = b for b on the even sites, M_hat = 1 - kappa^2 P_e D P_o D P_e the
    even-odd operator of M (l0 None) or of W_l0 (Sec. 1; rho > 0 is W3eo = W2eo + rho of
    the mass preconditioning), or its adjoint (the hops D^dagger). Since
    M_hat + rho = (1 + rho) (1 - kappa^2 P_e D P_o D P_e / (1 + rho)), the series is
        x = sum_{n >= 0} t_n,  t_0 = b / (1 + rho),
        t_{n+1} = kappa^2 / (1 + rho) P_e D P_o D t_n,
    and the residual of the sum t_0 .. t_N is (1 + rho) t_{N+1}: the sum stops at the first
    term with ||(1 + rho) t_{N+1}|| <= tol ||b|| (per system). The series converges where
    the spectral radius of kappa^2 D_eo D_oe is below 1 + rho. Returns (x, terms added,
    true relative residual)."""
    L = U.shape[:4]
    e, o = parity_masks(L)
    c = 1.0 + rho
    D = lambda v: hop(U, v, l0, adjoint)
    t = e * b / c
    bn = np.sqrt(_norm2(b))
    x = np.zeros_like(b)
    n = 0
    for _ in range(maxiter):
        x = x + t
        n += 1
        t = kappa * kappa / c * (e * D(o * D(t)))
        if np.all(c * np.sqrt(_norm2(t)) <= tol * bn) or not np.all(np.isfinite(t)):
            break
    r = e * b - (c * x - kappa * kappa * (e * D(o * D(x))))
    res = np.sqrt(_norm2(r)) / np.where(bn == 0, 1.0, bn)
    res = res.reshape(res.shape[:-6]) if res.ndim > 6 else float(res.reshape(()))
    return x, n, res

"""Krylov solvers of the oracle (FP64).

The paper solves its action parts with the geometric series and with BiCGstab (Sec. 3)
but fixes neither a stopping rule nor a precision. The oracle uses the textbook CG on the
normal equations A^dagger A x = A^dagger b in its CGLS form (Hestenes-Stiefel; the
residual s = b - A x of the original system is carried along), from x = 0, and stops on
||b - A x|| / ||b|| <= tol with the residual recomputed from A at the end (and restarted
from the current x if the recomputed one is not yet below tol).

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

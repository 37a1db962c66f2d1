"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and shapes them into fields in the canonical
interchange layout; it holds none of the Dirac-operator, solver, force or integrator
arithmetic. Both the FP64 oracle and the HIP path read the same bytes it produces.

Canonical layout (little-endian, complex128 unless stated otherwise); the site index
is lexicographic with x0 slowest, i = ((x0*L1 + x1)*L2 + x2)*L3 + x3:

* gauge field      U[x0,x1,x2,x3, mu, row, col]      complex128, SU(3) per link
* spinor field     psi[(rhs,) x0,x1,x2,x3, spin, colour]  complex128 (4 spin x 3 colour)
* momentum/force   p[x0,x1,x2,x3, mu, a]            float64, a = 0..7 (basis T^a = lambda^a/2)

Workload recipe (the paper's thermalised beta=5.6 ensembles are not available, so these
stand in for them): every link is U = exp(i*eps*H) with H = (A + A^dagger)/2 - Tr(.)/3,
Re A and Im A independent N(0,1) (so E Tr H^2 = 8); links are independent, so the mean
plaquette is c(eps)^4 with c = E[Tr cos(eps*H)]/3 (about 0.51 at eps = 0.35).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "CONFIGS", "gauge_field", "gaussian_spinor", "gaussian_momenta", "noise_spinor",
    "uniform", "lattice_volume",
]


# Named workloads: lattice (L0, L1, L2, L3), link roughness eps, hopping parameter kappa,
# block length l0 of the first x0 decomposition and the seeds of every random draw.
CONFIGS = {
    "tiny_4x4x4x4": dict(L=(4, 4, 4, 4), eps=0.5, kappa=0.155, l0=2, l0_sub=1,
                         seed_gauge=1001, seed_src=2001),
    "plain_16x16x16x32": dict(L=(32, 16, 16, 16), eps=0.35, kappa=0.1575, l0=4, l0_sub=2,
                              seed_gauge=1002, seed_src=2002),
    "precision_16x16x16x32": dict(L=(32, 16, 16, 16), eps=0.35, kappa=0.1575, l0=4, l0_sub=2,
                                  seed_gauge=1002, seed_src=2003),
    "hmc_16x16x16x32": dict(L=(32, 16, 16, 16), eps=0.35, kappa=0.1575, beta=5.6, l0=4,
                            l0_sub=2, seed_gauge=1002, seed_src=2004, seed_mom=3004,
                            seed_noise1=4004, seed_noise2=4005, seed_metropolis=5004),
    "batched_24x24x24x48": dict(L=(48, 24, 24, 24), eps=0.35, kappa=0.158, l0=4, l0_sub=2,
                                nrhs=12, seed_gauge=1005, seed_src=2005),
}


def lattice_volume(L) -> int:
    return int(np.prod(L))


def _exp_i_hermitian(H: np.ndarray, eps: float) -> np.ndarray:
    """exp(i*eps*H) for a stack of Hermitian 3x3 matrices, via eigen-decomposition."""
    w, v = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", v, ph, v.conj())


def gauge_field(L, eps: float, seed: int) -> np.ndarray:
    """Random SU(3) links U = exp(i*eps*H), canonical layout [x0,x1,x2,x3,mu,3,3].

    Draw order: one PCG64 stream; real parts of A for all (site, mu, row, col) first,
    then the imaginary parts.
    """
    rng = np.random.default_rng(seed)
    shape = tuple(L) + (4, 3, 3)
    A = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    H = 0.5 * (A + np.swapaxes(A.conj(), -1, -2))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    H = H - tr[..., None, None] * np.eye(3)
    return np.ascontiguousarray(_exp_i_hermitian(H, eps))


def gaussian_spinor(L, seed: int, nrhs: int | None = None, scale: float = 1.0) -> np.ndarray:
    """Complex Gaussian spinor source(s), Re and Im ~ N(0, scale^2).

    Shape [x0,x1,x2,x3,4,3] or [nrhs,x0,x1,x2,x3,4,3].
    """
    rng = np.random.default_rng(seed)
    shape = (tuple(L) if nrhs is None else (nrhs,) + tuple(L)) + (4, 3)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def noise_spinor(L, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Pseudo-fermion heat-bath noise with density proportional to exp(-|xi|^2):
    Re and Im ~ N(0, 1/2)."""
    return gaussian_spinor(L, seed, nrhs=nrhs, scale=np.sqrt(0.5))


def gaussian_momenta(L, seed: int) -> np.ndarray:
    """su(3) momenta p^a(x, mu) ~ N(0, 1), canonical layout [x0,x1,x2,x3,mu,8]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(tuple(L) + (4, 8))


def uniform(seed: int) -> float:
    """One uniform number in [0, 1) for the Metropolis decision."""
    return float(np.random.default_rng(seed).random())

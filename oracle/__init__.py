"""Plain FP64 CPU oracle for the Schwarz-preconditioned two-flavour HMC hot path
(M. Hasenbusch, "HMC algorithm for two-flavour lattice QCD: Schwarz-preconditioning with a
one-dimensional domain decomposition", Lattice 2007, arXiv:0710.0066).

TEST INFRASTRUCTURE ONLY. This package is imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py`` and by nothing
else. It shares no code, table or helper with the HIP product path in
``paper_0710_0066_amd``; the only module both sides read is ``synth`` (seeded inputs).

Everything is written on full-lattice numpy arrays in the canonical layout
(``U[x0,x1,x2,x3,mu,3,3]``, ``psi[..., x0,x1,x2,x3, spin, colour]``,
``F[x0,x1,x2,x3,mu,a]``), float64 / complex128, with plain shifts (``np.roll``) and
explicit 4x4 gamma matrices: no half-spinor trick, no even-odd storage, no blocking.

Modules and what they follow:

* ``gamma``    Euclidean gamma matrices (chiral basis; the paper does not fix one).
* ``lattice``  shifts with the fermion boundary phase, parity, x0 blocks and colours.
* ``dirac``    the Wilson-Dirac operator M (Sec. 1, eq. 2), its block restriction W
               (Sec. 1, blocks of l0 along x0), even-odd Schur complement (Sec. 1, W_eo).
* ``solvers``  CGLS (CG on the normal equations) and the even-odd solve.
* ``schwarz``  the boundary operator R on black-block boundaries and its action
               (Sec. 1: det^2(W1^{-1} M) via a field on black-block boundaries,
               halved by spin projection).
* ``forces``   gauge action (Sec. 1, S_G) and all forces as derivatives along
               U -> exp(i w T^a) U.
* ``hmc``      T_U, T_P, leap-frog and Sexton-Weingarten steps and their nesting
               (Sec. 2, eqs. 3-4, swimp, iterateLF, iterateSW), Metropolis.

Parity status: every function here is pinned by ``tests/test_oracle_*.py`` against
closed forms, invariants, dense linear algebra or finite differences (none is
"parity unpinned").
"""

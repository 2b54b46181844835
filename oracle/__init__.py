"""Plain FP64 CPU oracle for the pseudo-inverse-preconditioned Wiener-filter /
constrained-realization solver of Seljebotn et al. (arXiv:1710.00621).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code,
tables or constants with the HIP library; both sides receive the same input
arrays from the seeded generators in ``paper_1710_00621_amd.inputs``.

The oracle is deliberately slow and literal: numpy in float64, loops over m
and ell, a naive DFT on every ring (no FFT, no alias folding), and library
primitives (matmul, SVD, Cholesky) used only as single steps.

Modules
-------
geometry   ring grids (HEALPix RING, Gauss-Legendre) and quadrature weights
legendre   normalised associated Legendre functions by the three-term
           recurrence with an exponent-carrying start (no underflow)
sht        synthesis Y and its literal transpose Y^T, ring by ring
dense      dense Y / A builders for tiny band-limits
model      the linear system A = S^-1 + P^T N^-1 P of Sect. 2.3 (eq:A)
precond    alpha (App. A.1), U and U^+ (Sect. 3.3), M_PI and M_diag (Sect. 5)
pcg        preconditioned conjugate gradients (Sect. 2.3)
philox     Philox4x64-10 counter-based generator + Box-Muller normals
rhs        right-hand side of the constrained-realization system (Sect. 2.3)
"""

"""Plain FP64 CPU oracle for the boundary-element solve (test infrastructure).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU
baseline of the benchmark may import this package. It shares no code with
the GPU library (``paper_1905_01341_amd``); the two meet only in the seeded
input generator, which holds none of the method's arithmetic.

The oracle computes the plain definition of what the GPU path approximates:
the discrete BEM system of Section 3.1 (eq3_1/eq3_2) with the nodal
quadrature of Section 3.2 (ns1) and the singular diagonals of Section 3.3
(s3, s5), summed directly over all O(N^2) pairs, then solved by textbook
restarted GMRES (Section 3.8; Saad and Schultz 1986) or by dense LU.

Pins (tests/test_oracle_*.py): closed forms on spheres (Gauss's identity,
single-layer eigenvalues, exact Neumann data of a point-source exterior
field), refinement convergence, scaling/rigid-motion invariance, dense LU vs
GMRES, and hand-computed geometry of a regular octahedron.
"""
from .core import (  # noqa: F401
    build, geometry, sums, diagonals, rhs, offdiag_mvp, dense_offdiag,
    system_dense, matvec_L, gmres, bubble_block_inverse, solve, num_threads,
)

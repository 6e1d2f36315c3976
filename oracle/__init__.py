"""Plain FP64 CPU oracle for one Chebyshev-filtered subspace iteration (CheFSI) step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark may use it.  It shares no code with the GPU library; the two meet
only at the seeded synthetic inputs, which carry none of the method's
arithmetic.

What it computes (Sharma et al., "GPU acceleration of local and semilocal
density functional calculations in the SPARC electronic structure code",
arXiv:2302.09708):

* ``fd``          -- central finite-difference weights for d^2/dx^2 of order
                     n0 = 2r (Section 2.1, the Laplacian stencil of order n0);
* ``hamiltonian`` -- matrix-free H = -1/2 Lap_FD + Veff + sum_J chi_J Gamma_J
                     chi_J^T (Section 2.1, the three bullet points on applying H);
* ``chefsi``      -- Algorithm 1: Chebyshev filtering, projection, subspace
                     diagonalisation and rotation (Sections 2.1-2.4), plus the
                     spectral bounds the filter needs (readings listed below).

Everything is float64 NumPy/SciPy, written for clarity, not speed.

Readings of points the paper leaves open (each one is also listed with its
reason in the design notes):

* the filter is applied in the scaled three-term form of Zhou et al. (the
  CheFSI reference the paper builds on), which returns the paper's
  p_m((H - cI)/e) X divided by the scalar p_m((lambda_lo - c)/e); Ritz pairs
  are identical in exact arithmetic and the unscaled form is kept as a check;
* "degree m" = m applications of H inside the filter (one more gives
  Y~ = H X~ for the projection);
* the KB quadrature weight dV = hx*hy*hz multiplies chi_J^T x;
* Dirichlet directions hold nodes 0..N-1 with zero ghost values outside;
* the generalized eigenproblem is solved as LAPACK dsygvd does (type 1:
  H Z = M Z D, Z^T M Z = I, eigenvalues ascending); Hs and Ms are symmetrised
  by averaging with their transposes first.

Parity status: every function is pinned by the CPU tests (closed-form
free-particle spectra, separable-potential and rank-one reductions, Chebyshev
plane-wave gains, dense brute force on tiny grids, FD identities).  The
multi-iteration trajectory as a whole is pinned only through its converged
limit (the exact lowest eigenvalues); intermediate iterates are "parity
unpinned" beyond the invariants checked every step.
"""
from . import fd, hamiltonian, chefsi  # noqa: F401

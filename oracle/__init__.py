"""Plain FP64 CPU oracle of the correction-function KFBI method (Zhou & Ying,
arXiv 2309.05965).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the HIP library is checked against.  Only the test-suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product path never does, and it shares no code with the HIP
library.

Modules and their pins (tests/test_oracle_*.py, run with -m "not gpu")
  levelset     level-set functions H and their gradients (Sec. 5.1; the
               product3d family is the domain of the 3D Dirichlet example of
               Sec. 6.2.2, molecule3d the molecular surface of Sec. 6.2.3,
               grid a level set known only at the nodes, Sec. 7); the grid
               family is pinned by exact reproduction of polynomials, the
               sampled sphere's analytic geometry and the sampled star's
               solution (tests/test_oracle_sampled.py); the others
               by the closed-form normals and curvatures of the sample tests
               and the exact intersections of the geometry tests
  geometry     node regions, surface points, collocation stencils, density
               extension, irregular nodes, closest-centre map, interpolation
               blocks, correction entries (Secs. 5.1, 5.2, 5.3, 5.5); pinned
               by the paper's printed N_b, brute-force closest centres,
               extension exactness on polynomials, and (two interfaces) the
               polynomial patch test of the whole simple solve
  collocation  local Cauchy problem by square collocation (Secs. 5.3.1, 5.4);
               pinned by exact reproduction of polynomials
  fd           compact finite-difference operators and the DST box solve
               (Sec. 5.2, eqs. 9p-cds / 27p-cds; Alg. 1 Step 3.3); pinned by
               the printed stencil coefficients, exactness on quintics, sine
               eigenmodes and sparse-LU solves
  kfbi         simple interface solve, BIE operator, GMRES, full solve
               (Secs. 3.2, 4, 5.5, Alg. 1); pinned by patch tests (one and
               two interfaces), A = I/2 for equal coefficients, a dense
               brute-force BIE, GMRES against a dense solve and the 2nd/4th
               order convergence rates
  bvp          interior Dirichlet and Neumann problems (eqs. bie-D, bie-N;
               Secs. 3.1, 4, 5.5): one-sided values of the corrected
               interpolation, the density as the jump [u] (Dirichlet) or
               [d_n u] (Neumann), the zero-mean shift of Sec. 6.2.1; pinned
               by exact polynomial traces, the double-layer potential of a
               constant density (exactly the indicator of Omega), the
               paper's printed Table 2d-poi-o4 (iterations and errors at
               paper level), the Neumann convergence rate, and the Neumann
               operator as the interface operator with beta_out = 0
  twodensity   two-density interface BIE (eq. bie-ifp-1) for different
               kappa_i / sigma_i on the two sides, as two simple solves per
               product (one per Green's function); pinned by the exact
               densities of piecewise-polynomial solutions (one and two
               interfaces, 2D and 3D) satisfying the discrete system to
               rounding, and the 2nd/4th-order convergence of a
               Poisson / modified-Helmholtz problem
  mg           two-grid multigrid box solver (a textbook method, not in the
               paper; its converged result is A_h^-1 F); pinned by the
               transfer identities, the Jacobi weight against the Fourier
               symbol, the per-cycle contraction and the converged result
               against the exact sine-transform solve within its bound
  learned      learned initial density (features, spherical harmonics,
               MLP with bf16 rounding, linear head, Adam); pinned by closed
               forms, quadrature orthonormality, exact band-limited
               transfers and coefficient recovery, bf16 tie cases, finite
               differences of every gradient and the published Adam update

Every reading of the paper that the oracle takes where the paper is silent
is stated beside the code that takes it; each function cites the passage it
follows.  Every function above is pinned by one of those tests.
"""

"""Plain FP64 CPU oracle for the structure-preserving geometric multigrid method
for isogeometric divergence-conforming discretizations of the generalized Stokes
and Oseen problems (Coley, Benzaken, Evans, arXiv:1705.09282).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` use it.  It shares no code with the HIP library; the only
module both sides import is the seeded input generator ``workloads``, which
holds none of the method's arithmetic.

Every function states the passage of the paper it follows.  The oracle is
deliberately plain: dense per-direction B-spline tables, d-dimensional Gauss
quadrature for every integral, scipy sparse products for the Galerkin triple
product, brute-force support containment for the subdomains, and numpy batched
inverses for the local saddle-point problems.

Pins (``-m "not gpu"`` tests in ``tests/test_oracle_*.py``), one or more per
module, each against a fact the paper or the mathematics fixes:

* ``bspline``: partition of unity, derivatives against finite differences,
  cardinal values.
* ``spaces``: the DOF columns printed in the paper's Tables 1, 2 and 4; Euler
  characteristics of the discrete complexes.
* ``assemble``: polynomial-exact integrals; B 1 = 0; O(h^{k+1}) velocity error
  of the solution.
* ``refine``: two-scale rows of the refinement matrix; Galerkin identity;
  refinement commutes with the curl (velocity and potential prolongation).
* ``patches``: interior subdomain dimensions of the paper's subsection on
  Schwarz smoothers; local exactness; colour disjointness.
* ``complex``: curl of a polynomial potential against its exact coefficients
  (polar forms); divergence-free images.
* ``diagnostics``: ||div u|| and ||u|| of polynomial fields against closed
  forms; the direct solve against the V-cycle limit.
* ``multigrid``: V-cycles against the direct solve; the divergence-free
  invariant; h-independent factors; the additive damping reading against the
  paper's protocol and its Table 2 (eta = 0.5 diverges, eta0 is the best
  stable sweep value); multiplicative Schwarz against the product formula of
  equation MSM, the sequential sweep, and Table 1; Chebyshev dampings against
  numpy's Chebyshev series.
* ``mlp``: gradients against finite differences; Adam on a quadratic.
* ``timestep``: the convective load of polynomial fields against the mass
  matrix times exact spline coefficients; the linear part of the
  Crank-Nicolson / Adams-Bashforth load against an independent assembly;
  the advection by a discrete polynomial field against the analytic field;
  a field advecting itself against the convective load; the Guermond load's
  linear part against an independent mass matrix.
* ``geometry``: the Bezier arc against the unit circle, J and its
  derivatives against finite differences of the map, the identity map
  against the unit-domain assembly, the Piola divergence identity, the whole
  operator on the annulus and cylinder section against an independent
  assembly in cylindrical coordinates, B^T u = 0 for divergence-free
  starts, and the mapped divergence norm against the unit-domain norm
  (identity map) and the physical-gradient quadrature.

None of these functions is "parity unpinned".
"""

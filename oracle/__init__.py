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

Parity status: every function is pinned by a ``-m "not gpu"`` test against a
fact the paper or the mathematics fixes (see ``tests/test_oracle_*.py``); none
is "parity unpinned".
"""

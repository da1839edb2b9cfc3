"""Knot-insertion refinement and intergrid transfer (oracle).

Follows the paper's subsection on B-spline refinement (a coarse function is a
linear combination of the refined functions, N_i = sum_j T_ij N~_j) and the
subsection on nested complexes and intergrid transfer (P^v, P^q built from T in
tensor-product fashion, block prolongation P = diag(P^v, P^q), restriction
R = P^T, Galerkin coarse matrices K_l = R_{l+1} K_{l+1} P_l).

The paper leaves the construction of T to the literature.  The oracle takes
the plain definition: since the coarse space is contained in the refined one,
T is the unique matrix with  Phi_coarse(x) = Phi_fine(x) T^T  at any set of
points that is unisolvent for the refined space; the Greville abscissae of the
refined knot vector are such a set (Schoenberg-Whitney).  A dense solve gives T.
"""
import numpy as np
import scipy.sparse as sp

from .bspline import open_knots, basis
from .assemble import _kron_all


def greville(knots, degree):
    n = len(knots) - degree - 1
    if degree == 0:
        return 0.5 * (knots[:-1] + knots[1:])[:n]
    return np.array([knots[i + 1:i + degree + 1].mean() for i in range(n)])


def refinement_matrix(n_coarse_elem, degree):
    """T (n_coarse x n_fine) for inserting every element midpoint once:
    coarse N_i = sum_j T_ij fine N_j."""
    kc = open_knots(n_coarse_elem, degree)
    kf = open_knots(2 * n_coarse_elem, degree)
    x = greville(kf, degree)
    Bf = basis(kf, degree, x)
    Bc = basis(kc, degree, x)
    Tt = np.linalg.solve(Bf, Bc)  # Bf @ T^T = Bc
    T = Tt.T
    T[np.abs(T) < 1e-14] = 0.0
    return T


def block_prolongation(block_c, block_f, n_coarse_elem):
    """P for one tensor-product block: kept fine rows x kept coarse columns,
    P = kron over directions of T_dir^T (direction 0 fastest)."""
    mats = []
    for j, q in enumerate(block_c.degrees):
        T = refinement_matrix(n_coarse_elem, q)
        Pj = T.T[block_f.lo[j]:block_f.hi[j], block_c.lo[j]:block_c.hi[j]]
        mats.append(sp.csr_matrix(Pj))
    return _kron_all(mats)


def prolongation(disc_c, disc_f):
    """Block prolongation P = diag(P^v_0, ..., P^v_{d-1}, P^q)."""
    blocks = [block_prolongation(bc, bf, disc_c.N) for bc, bf in zip(disc_c.blocks, disc_f.blocks)]
    return sp.block_diag(blocks, format="csr")


def potential_prolongation(disc_c, disc_f):
    blocks = [block_prolongation(bc, bf, disc_c.N) for bc, bf in zip(disc_c.pot, disc_f.pot)]
    return sp.block_diag(blocks, format="csr")


def galerkin(K_fine, P):
    """K_coarse = R K_fine P with R = P^T."""
    Kc = sp.csr_matrix(P.T @ K_fine @ P)
    Kc.sort_indices()
    return Kc

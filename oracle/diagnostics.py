"""Diagnostics for the oracle: divergence norm, L2 errors, direct solve.

* ||div u_h||_{L2} is the quantity of the paper's lemma (b(v_h, q_h) = 0 for
  all q_h implies div v_h = 0 pointwise) and of its divergence-preservation
  argument; it is computed here by Gauss quadrature of (div u_h)^2.
* The exact discrete solution U* = K^{-1} F with zero-mean pressure is the
  plain definition of what the solver approaches; it is computed by a sparse
  direct solve of the bordered system (global multiplier of the paper's
  footnote on the pressure basis).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import quadrature, tensor_eval, tensor_weights, tensor_points, pressure_integrals


def div_values(disc, U, pts):
    out = 0.0
    for c, blk in enumerate(disc.vel):
        u = U[disc.offsets[c]:disc.offsets[c + 1]]
        out = out + tensor_eval(disc, blk, pts, deriv_dir=c) @ u
    return out


def div_norm(disc, U):
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    dv = div_values(disc, U, pts)
    return float(np.sqrt(np.sum(w * dv * dv)))


def velocity_values(disc, U, pts):
    return np.stack([tensor_eval(disc, blk, pts) @ U[disc.offsets[c]:disc.offsets[c + 1]]
                     for c, blk in enumerate(disc.vel)], axis=1)


def l2_norm_velocity(disc, U):
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    v = velocity_values(disc, U, pts)
    return float(np.sqrt(np.sum(w[:, None] * v * v)))


def l2_error_velocity(disc, U, u_exact):
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    X = tensor_points(pts)
    e = velocity_values(disc, U, pts) - u_exact(X)
    return float(np.sqrt(np.sum(w[:, None] * e * e)))


def direct_solve(disc, K, F):
    """Solve [[K, e], [e^T, 0]] [U; mu] = [F; 0], e = [0; w]: zero-mean pressure."""
    w = pressure_integrals(disc)
    e = np.concatenate([np.zeros(disc.n_v), w])
    n = disc.n
    Kb = sp.bmat([[K, sp.csr_matrix(e[:, None])], [sp.csr_matrix(e[None, :]), None]], format="csc")
    sol = spla.spsolve(Kb, np.concatenate([F, [0.0]]))
    return sol[:n]

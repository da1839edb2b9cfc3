"""Discrete Stokes complex maps (oracle).

The paper's 2D complex maps streamfunctions to velocities by the rotated
gradient (grad-perp) and its 3D complex maps vector potentials to velocities
by the curl.  The oracle takes the plain definition: the velocity coefficients
of curl(psi_h) are those of its L2 projection onto the velocity space, which
is exact because curl maps the potential space into the velocity space.
2D sign convention: u = (d_y psi, -d_x psi).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import quadrature, tensor_eval, tensor_weights


def curl_values(disc, psi, pts):
    """Values of curl(psi_h) at the tensor grid ``pts``: (npts, d)."""
    d = disc.d
    parts = [psi[disc.pot_offsets[o]:disc.pot_offsets[o + 1]] for o in range(len(disc.pot))]
    if d == 2:
        pb = disc.pot[0]
        dx = tensor_eval(disc, pb, pts, deriv_dir=0) @ parts[0]
        dy = tensor_eval(disc, pb, pts, deriv_dir=1) @ parts[0]
        return np.stack([dy, -dx], axis=1)
    g = [[tensor_eval(disc, disc.pot[o], pts, deriv_dir=j) @ parts[o] for j in range(3)] for o in range(3)]
    # curl psi = (d_y psi_z - d_z psi_y, d_z psi_x - d_x psi_z, d_x psi_y - d_y psi_x)
    return np.stack([g[2][1] - g[1][2], g[0][2] - g[2][0], g[1][0] - g[0][1]], axis=1)


def curl(disc, psi):
    """Velocity coefficients of curl(psi_h) (L2 projection, exact)."""
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    cv = curl_values(disc, psi, pts)
    out = []
    for c, blk in enumerate(disc.vel):
        Phi = tensor_eval(disc, blk, pts)
        M = sp.csc_matrix(Phi.T @ sp.diags(w) @ Phi)
        out.append(spla.spsolve(M, Phi.T @ (w * cv[:, c])))
    return np.concatenate(out)


def random_divfree_start(disc, psi_coeffs, p_coeffs):
    """U_0 = [curl psi_0; p_0] from given random coefficients: the random
    divergence-free initial guess of the numerical-results section."""
    return np.concatenate([curl(disc, psi_coeffs), p_coeffs])

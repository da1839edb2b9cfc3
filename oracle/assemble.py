"""Assembly of the saddle-point system K U = F (oracle).

Follows the paper's weak formulation of the generalized Stokes and Oseen
problems, the weak (Nitsche) enforcement of no-slip with strong
no-penetration, and the block matrix system K = [[A, -B], [B^T, 0]] with
[A]_ij = a_h(N_i, N_j), [B]_ij = b(N_i, N^q_j), [F]_i = l(N_i).

Every integral is taken by d-dimensional Gauss-Legendre quadrature with k+3
points per direction per element (k+3 points integrate every bilinear form of
the paper exactly on the unit square/cube for constant sigma, nu and an
advection field that is linear or a velocity of the discrete space); boundary
integrals use the same rule on each face.  Basis values at the quadrature
points form sparse matrices Phi (points x functions) built from the per
direction tables by the tensor-product definition of multivariate B-splines,
so that each bilinear form is Phi_test^T diag(weights * coefficient) Phi_trial.
"""
import numpy as np
import scipy.sparse as sp

from .bspline import basis, basis_deriv, gauss_rule
from .spaces import Discretization


def _tables(disc, block, pts, deriv_dir=None):
    """Per-direction 1D tables (points x kept functions) for ``block``."""
    out = []
    for j in range(disc.d):
        q = block.degrees[j]
        kn = disc.knots(q)
        f = basis_deriv if deriv_dir == j else basis
        out.append(sp.csr_matrix(f(kn, q, pts[j])[:, block.lo[j]:block.hi[j]]))
    return out


def _kron_all(mats):
    """Tensor product with direction 0 fastest: kron(M_{d-1}, ..., kron(M_1, M_0))."""
    res = mats[0]
    for m in mats[1:]:
        res = sp.kron(m, res, format="csr")
    return sp.csr_matrix(res)


def tensor_eval(disc, block, pts, deriv_dir=None):
    """Sparse matrix of block basis values (or d/dx_dir) at the tensor grid of
    per-direction points ``pts`` (list of d arrays), rows x fastest."""
    return _kron_all(_tables(disc, block, pts, deriv_dir))


def tensor_weights(wts):
    res = wts[0]
    for w in wts[1:]:
        res = np.kron(w, res)
    return res


def tensor_points(pts):
    """Coordinates (npts, d) of the tensor grid, x fastest."""
    grids = np.meshgrid(*pts[::-1], indexing="ij")
    return np.stack([g.ravel() for g in grids[::-1]], axis=1)


def quadrature(disc, npts=None):
    npts = disc.k + 3 if npts is None else npts
    x, w = gauss_rule(disc.N, npts)
    return [x] * disc.d, [w] * disc.d


def assemble(disc, nu, sigma, advection=None, C_I=None, h=None):
    """Assemble K = [[A, -B], [B^T, 0]] on ``disc``.

    advection: None (generalized Stokes) or a callable mapping points (n, d)
    to the advection field a (n, d) (generalized Oseen).
    C_I: Nitsche penalty constant, default 4k (the paper's 4(p-1), p = k+1).
    h:   wall-normal element size, default 1/N.
    Returns dict with csr matrices K, A, B.
    """
    d, k = disc.d, disc.k
    C_I = 4.0 * k if C_I is None else C_I
    h = 1.0 / disc.N if h is None else h
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    X = tensor_points(pts)
    a_field = None if advection is None else advection(X)
    Phi_q = tensor_eval(disc, disc.pre, pts)

    A_blocks, B_blocks = [], []
    for c, blk in enumerate(disc.vel):
        Phi = tensor_eval(disc, blk, pts)
        dPhi = [tensor_eval(disc, blk, pts, deriv_dir=j) for j in range(d)]
        W = sp.diags(w)
        # sigma (v, u) + nu (grad v : grad u), component c only
        A = sigma * (Phi.T @ W @ Phi)
        for j in range(d):
            A = A + nu * (dPhi[j].T @ W @ dPhi[j])
        # advection (v, a . grad u)
        if a_field is not None:
            for j in range(d):
                A = A + Phi.T @ sp.diags(w * a_field[:, j]) @ dPhi[j]
        # Nitsche terms on every face: -nu (v, d_n u) - nu (d_n v, u) + C_I nu / h (v, u)
        A = A + _nitsche(disc, blk, nu, C_I, h)
        A_blocks.append(sp.csr_matrix(A))
        # b(v, q) = (div v, q): only d_c of component c
        B_blocks.append(sp.csr_matrix(dPhi[c].T @ W @ Phi_q))

    A = sp.block_diag(A_blocks, format="csr")
    B = sp.vstack(B_blocks, format="csr")
    K = sp.bmat([[A, -B], [B.T, None]], format="csr")
    K.sort_indices()
    return {"K": K, "A": A, "B": B}


def _nitsche(disc, blk, nu, C_I, h):
    d = disc.d
    pts, wts = quadrature(disc)
    n = blk.size
    out = sp.csr_matrix((n, n))
    for e in range(d):
        for side, normal in ((0.0, -1.0), (1.0, 1.0)):
            fp = list(pts)
            fw = list(wts)
            fp[e] = np.array([side])
            fw[e] = np.array([1.0])
            wf = sp.diags(tensor_weights(fw))
            Phi = tensor_eval(disc, blk, fp)
            dn = normal * tensor_eval(disc, blk, fp, deriv_dir=e)
            out = out - nu * (Phi.T @ wf @ dn) - nu * (dn.T @ wf @ Phi) + (C_I * nu / h) * (Phi.T @ wf @ Phi)
    return sp.csr_matrix(out)


def load_vector(disc, f):
    """F = [l(N^v_i); 0] with l(v) = (v, f); f maps points (n, d) -> (n, d)."""
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    X = tensor_points(pts)
    fv = f(X)
    parts = []
    for c, blk in enumerate(disc.vel):
        Phi = tensor_eval(disc, blk, pts)
        parts.append(Phi.T @ (w * fv[:, c]))
    parts.append(np.zeros(disc.n_q))
    return np.concatenate(parts)


def pressure_integrals(disc):
    """w_j = integral of pressure basis function j over the unit square/cube,
    by quadrature (used for the zero-mean pressure constraint)."""
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    Phi_q = tensor_eval(disc, disc.pre, pts)
    return np.asarray(Phi_q.T @ w).ravel()


def rotation_field(c):
    """Advection a = c * (-(y - 1/2), x - 1/2) (2D rigid rotation about the centre)."""
    def a(X):
        out = np.zeros_like(X)
        out[:, 0] = -c * (X[:, 1] - 0.5)
        out[:, 1] = c * (X[:, 0] - 0.5)
        return out
    return a


def build(d, n_elem, k, nu, sigma, advection=None):
    disc = Discretization(d, n_elem, k)
    mats = assemble(disc, nu, sigma, advection)
    return disc, mats

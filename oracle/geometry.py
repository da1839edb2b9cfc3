"""Mapped geometries and the assembly of K on them (oracle; test
infrastructure only).

Follows the paper's construction of compatible B-splines on a physical
domain Omega = F(Omega_hat) (equations physical_2D and physical_3D of the
section on isogeometric compatible B-splines): potentials pulled back by
composition (2D) or the covariant map (3D), velocities by the contravariant
Piola map  v o F = J v_hat / det J,  pressures by  q o F = q_hat / det J,
J = d F / d xi.  The discrete complex, and with it every parametric
coefficient map (curl, prolongation, subdomains), carries over unchanged;
only the bilinear forms are integrated on Omega:

  mass       sigma (v, u)            = sigma  int v . u  det J dxi
  viscous    nu (grad v : grad u)    = nu     int grad v : grad u  det J dxi
  divergence (div v, q)              =        int div v  q_hat dxi
  Nitsche    -nu (v, grad u n) - nu (grad v n, u) + C_I nu / h (v, u) on
             every boundary face, ds = det J |J^-T n_hat| dxi_face,
             h = 1 / (N |J^-T n_hat|) (the element size normal to the wall)
  load       (v, f)                  = int (J v_hat) . f(F(xi)) dxi

with the physical gradient of a velocity basis function
  grad v = d/dxi (J v_hat / det J) J^-1,
whose derivatives of J and det J (d det J = det J tr(J^-1 dJ)) come from the
map's second derivatives.  Quadrature as in ``assemble`` (k+3 Gauss points
per direction per element).  The pressure mean constraint is unchanged:
int_Omega p dx = int q_hat dxi.

Geometries: ``QuarterAnnulus`` (the paper's 2D mapped test: radii r_i, r_o;
xi_1 radial and linear from r_i to r_o, xi_2 the quarter circle from the
x axis to the y axis as a quadratic rational Bezier curve) and, in 3D, that
annulus extruded along z by a depth (the hollow cylinder section, xi_3
linear).  ``IdentityMap`` is the unit square / cube.
"""
import numpy as np
import scipy.sparse as sp

from .assemble import quadrature, tensor_eval, tensor_points, tensor_weights


class IdentityMap:
    """F(xi) = xi on the unit square / cube."""

    def __init__(self, d):
        self.d = d

    def geometry(self, Xi):
        n, d = Xi.shape
        J = np.broadcast_to(np.eye(d), (n, d, d)).copy()
        return Xi.copy(), J, np.zeros((n, d, d, d))


class QuarterAnnulus:
    """Quarter annulus (d = 2) or hollow cylinder section (d = 3)."""

    def __init__(self, d=2, r_in=0.075, r_out=0.225, depth=0.1):
        self.d, self.r_in, self.r_out, self.depth = d, r_in, r_out, depth

    @staticmethod
    def arc(t):
        """The unit quarter circle as the quadratic rational Bezier curve with
        control points (1,0), (1,1), (0,1) and weights 1, 1/sqrt(2), 1: point,
        first and second derivatives, each (n, 2)."""
        w = 1.0 / np.sqrt(2.0)
        b = [(1 - t) ** 2, 2 * t * (1 - t), t ** 2]
        db = [-2 * (1 - t), 2 - 4 * t, 2 * t]
        ddb = [2.0 + 0 * t, -4.0 + 0 * t, 2.0 + 0 * t]
        P = np.array([[1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
        wt = np.array([1.0, w, 1.0])

        def comb(bb):
            num = sum(wt[j] * bb[j][:, None] * P[j] for j in range(3))
            den = sum(wt[j] * bb[j] for j in range(3))
            return num, den
        f, g = comb(b)
        f1, g1 = comb(db)
        f2, g2 = comb(ddb)
        c = f / g[:, None]
        c1 = (f1 - c * g1[:, None]) / g[:, None]
        c2 = (f2 - 2 * c1 * g1[:, None] - c * g2[:, None]) / g[:, None]
        return c, c1, c2

    def geometry(self, Xi):
        """x = F(xi) (n, d), J[:, i, m] = dx_i / dxi_m, and
        dJ[:, q, i, m] = d^2 x_i / dxi_q dxi_m."""
        n, d = Xi.shape
        dr = self.r_out - self.r_in
        r = self.r_in + dr * Xi[:, 0]
        c, c1, c2 = self.arc(Xi[:, 1])
        x = np.zeros((n, d))
        J = np.zeros((n, d, d))
        dJ = np.zeros((n, d, d, d))
        x[:, :2] = r[:, None] * c
        J[:, :2, 0] = dr * c
        J[:, :2, 1] = r[:, None] * c1
        dJ[:, 0, :2, 1] = dr * c1
        dJ[:, 1, :2, 0] = dr * c1
        dJ[:, 1, :2, 1] = r[:, None] * c2
        if d == 3:
            x[:, 2] = self.depth * Xi[:, 2]
            J[:, 2, 2] = self.depth
        return x, J, dJ


def physical_basis(disc, geom, c, pts):
    """Values and physical gradients of the velocity basis of component c at
    the tensor grid ``pts``: V[i] (points x functions) is component i of the
    physical field, T[i][j] its derivative d/dx_j; also det J."""
    d = disc.d
    Xi = tensor_points(pts)
    _, J, dJ = geom.geometry(Xi)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    ddet = det[:, None] * np.einsum("pmn,pqnm->pq", Jinv, dJ)
    beta = J[:, :, c] / det[:, None]                                     # (p, i)
    alpha = dJ[:, :, :, c].transpose(0, 2, 1) / det[:, None, None] \
        - J[:, :, c][:, :, None] * (ddet / det[:, None] ** 2)[:, None, :]  # (p, i, q)
    acoef = np.einsum("piq,pqj->pij", alpha, Jinv)                       # (p, i, j)
    blk = disc.vel[c]
    Phi = tensor_eval(disc, blk, pts)
    dPhi = [tensor_eval(disc, blk, pts, deriv_dir=q) for q in range(d)]
    V = [sp.diags(beta[:, i]) @ Phi for i in range(d)]
    T = [[sp.diags(acoef[:, i, j]) @ Phi
          + sum(sp.diags(beta[:, i] * Jinv[:, q, j]) @ dPhi[q] for q in range(d))
          for j in range(d)] for i in range(d)]
    return [sp.csr_matrix(v) for v in V], [[sp.csr_matrix(t) for t in row] for row in T], det


def assemble_mapped(disc, geom, nu, sigma, C_I=None):
    """K = [[A, -B], [B^T, 0]] of the generalized Stokes problem on F(Omega_hat);
    A couples every pair of velocity components."""
    d, k = disc.d, disc.k
    C_I = 4.0 * k if C_I is None else C_I
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    Phi_q = tensor_eval(disc, disc.pre, pts)
    VT = [physical_basis(disc, geom, c, pts) for c in range(d)]
    det = VT[0][2]
    Wd = sp.diags(w * det)
    A = [[None] * d for _ in range(d)]
    for c in range(d):
        for c2 in range(d):
            Vc, Tc, _ = VT[c]
            Vc2, Tc2, _ = VT[c2]
            blk = sigma * sum(Vc[i].T @ Wd @ Vc2[i] for i in range(d))
            blk = blk + nu * sum(Tc[i][j].T @ Wd @ Tc2[i][j] for i in range(d) for j in range(d))
            A[c][c2] = blk
    _nitsche_mapped(disc, geom, nu, C_I, A)
    B_blocks = []
    for c in range(d):
        Tc = VT[c][1]
        div = sum(Tc[i][i] for i in range(d))
        B_blocks.append(sp.csr_matrix(div.T @ Wd @ sp.diags(1.0 / det) @ Phi_q))
    A = sp.csr_matrix(sp.bmat(A))
    B = sp.vstack(B_blocks, format="csr")
    K = sp.bmat([[A, -B], [B.T, None]], format="csr")
    K.sort_indices()
    return {"K": K, "A": A, "B": B}


def _nitsche_mapped(disc, geom, nu, C_I, A):
    d = disc.d
    pts, wts = quadrature(disc)
    for e in range(d):
        for side, sgn in ((0.0, -1.0), (1.0, 1.0)):
            fp, fw = list(pts), list(wts)
            fp[e], fw[e] = np.array([side]), np.array([1.0])
            Xi = tensor_points(fp)
            _, J, _ = geom.geometry(Xi)
            nhat = np.zeros(d)
            nhat[e] = sgn
            m = np.einsum("pji,j->pi", np.linalg.inv(J), nhat)          # J^-T n_hat
            mlen = np.linalg.norm(m, axis=1)
            n = m / mlen[:, None]
            ds = tensor_weights(fw) * np.linalg.det(J) * mlen
            h = 1.0 / (disc.N * mlen)
            VT = [physical_basis(disc, geom, c, fp) for c in range(d)]
            Dn = [[sum(sp.diags(n[:, j]) @ VT[c][1][i][j] for j in range(d)) for i in range(d)] for c in range(d)]
            Ws, Wh = sp.diags(ds), sp.diags(ds / h)
            for c in range(d):
                for c2 in range(d):
                    Vc, Vc2 = VT[c][0], VT[c2][0]
                    A[c][c2] = A[c][c2] + sum(
                        -nu * (Vc[i].T @ Ws @ Dn[c2][i]) - nu * (Dn[c][i].T @ Ws @ Vc2[i])
                        + C_I * nu * (Vc[i].T @ Wh @ Vc2[i]) for i in range(d))


def load_vector_mapped(disc, geom, f):
    """[int_Omega N_i . f dx]_i for f a callable on physical points (n, d)
    returning (n, d); pressure rows zero."""
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    x, J, _ = geom.geometry(tensor_points(pts))
    fx = f(x)
    parts = []
    for c, blk in enumerate(disc.vel):
        Phi = tensor_eval(disc, blk, pts)
        parts.append(Phi.T @ (w * np.einsum("pi,pi->p", J[:, :, c], fx)))
    parts.append(np.zeros(disc.n_q))
    return np.concatenate(parts)


def smooth_forcing(geom):
    """A smooth load on the mapped domain (the tests' right-hand side):
    f = (sin(pi x / r_o) cos(pi y / r_o), x y / r_o^2[, cos(pi z / depth)])."""
    ro = geom.r_out

    def f(x):
        out = np.zeros_like(x)
        out[:, 0] = np.sin(np.pi * x[:, 0] / ro) * np.cos(np.pi * x[:, 1] / ro)
        out[:, 1] = x[:, 0] * x[:, 1] / ro ** 2
        if x.shape[1] == 3:
            out[:, 2] = np.cos(np.pi * x[:, 2] / geom.depth)
        return out
    return f


def div_norm_mapped(disc, geom, U):
    """||div u_h||_{L2(Omega)}: div u = div_hat u_hat / det J and dx = det J dxi
    give the integral of (div_hat u_hat)^2 / det J over the parametric domain."""
    from .diagnostics import div_values
    pts, wts = quadrature(disc)
    w = tensor_weights(wts)
    _, J, _ = geom.geometry(tensor_points(pts))
    dv = div_values(disc, U, pts)
    return float(np.sqrt(np.sum(w * dv * dv / np.linalg.det(J))))

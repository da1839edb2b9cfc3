"""Multigrid V-cycle with the additive Schwarz smoother (oracle).

Follows Algorithm 1 of the paper (the recursive V-cycle MGV: exact solve on the
coarsest level; nu1 pre-smoothing steps U <- U + S^{-1}(F - K U); restriction
G = R (F - K U); coarse correction from Delta U = 0; prolongation
U <- U + P Delta U; nu2 post-smoothing steps), the additive Schwarz smoother
S^{-1} = eta sum_i E_i^T K_i^{-1} E_i (equation ASM), and the solution
protocol of the numerical-results section (repeat V-cycles; additional cycles
are additional calls).

The multiplicative Schwarz smoother (equation MSM) solves the same local
problems one subdomain after the other, each on the residual left by the
previous ones, with no damping (the update formula of the subsection on
preservation of the divergence-free constraint).  The paper does not fix the
order of the subdomains; the oracle visits them colour by colour in the
coupling-free colouring of ``coupling_free_colours`` (inside a colour in
subdomain order), and ``smooth_multiplicative`` is the plain sequential sweep
in that order.

The coarsest-level solve uses the global zero-mean pressure multiplier of the
paper's footnote: the bordered system [[K_0, e], [e^T, 0]] with e = [0; w_0].
"""
import numpy as np
import scipy.sparse as sp

from .spaces import Discretization
from .assemble import assemble, load_vector, pressure_integrals
from .refine import prolongation, galerkin
from .patches import build_patches, local_inverses


class Level:
    def __init__(self, disc, K):
        self.disc = disc
        self.K = K
        self.w = pressure_integrals(disc)
        self.P = None        # prolongation from this level to the next finer one (None on the finest)
        self.patches = None
        self.groups = None
        self.coarse_inv = None


class Hierarchy:
    """Levels 0 (coarsest) .. L-1 (finest); K on the finest level is
    assembled (on the unit square / cube, or on a mapped domain), coarser
    ones are Galerkin products."""

    def __init__(self, d, n_elem, k, n_levels, nu, sigma, advection=None, geometry=None):
        assert n_elem % (2 ** (n_levels - 1)) == 0
        self.d, self.k, self.L = d, k, n_levels
        self.nu, self.sigma = nu, sigma
        finest = Discretization(d, n_elem, k)
        if geometry is None:
            mats = assemble(finest, nu, sigma, advection)
        else:  # a mapped domain (generalized Stokes)
            assert advection is None
            from .geometry import assemble_mapped
            mats = assemble_mapped(finest, geometry, nu, sigma)
        levels = [Level(finest, mats["K"])]
        self.A, self.B = mats["A"], mats["B"]
        for _ in range(n_levels - 1):
            fine = levels[0]
            coarse_disc = Discretization(d, fine.disc.N // 2, k)
            P = prolongation(coarse_disc, fine.disc)
            Kc = galerkin(fine.K, P)
            lv = Level(coarse_disc, Kc)
            lv.P = P
            levels.insert(0, lv)
        self.levels = levels
        for l, lv in enumerate(levels):
            if l == 0:
                n = lv.disc.n
                e = np.concatenate([np.zeros(lv.disc.n_v), lv.w])
                bord = np.zeros((n + 1, n + 1))
                bord[:n, :n] = lv.K.toarray()
                bord[:n, n] = e
                bord[n, :n] = e
                lv.coarse_inv = np.linalg.inv(bord)[:n, :n]
            else:
                lv.patches = build_patches(lv.disc)
                lv.groups = local_inverses(lv.K, lv.patches, lv.w, lv.disc.n_v)

    @property
    def finest(self):
        return self.levels[-1]


def schwarz_correction(level, r):
    """sum_i E_i^T M_i E_i r  (the sum in equation ASM, before eta)."""
    out = np.zeros_like(r)
    for ids, I, M in level.groups:
        delta = np.einsum("mij,mj->mi", M, r[I])
        out += np.bincount(I.ravel(), weights=delta.ravel(), minlength=r.size)
    return out


def smooth(level, U, F, eta):
    """One additive Schwarz step U <- U + eta sum_i E_i^T K_i^{-1} E_i (F - K U)."""
    r = F - level.K @ U
    return U + eta * schwarz_correction(level, r)


def coupling_free_colours(disc, patches):
    """Colour of every subdomain such that two subdomains of one colour share
    no DOF and no matrix entry couples a DOF of one with a DOF of the other.
    A subdomain is the support of a potential basis function, a box of at
    most k+2 elements per direction, and every DOF of the subdomain has its
    support inside that box; two subdomains of one orientation whose
    potential indices differ by k+2 or more in some direction therefore have
    disjoint boxes in that direction, and the basis functions inside them do
    not overlap.  Colour = (o, a mod (k+2), b mod (k+2)[, c mod (k+2)]) in
    lexicographic order: 9 / 16 colours in 2D (k = 1 / 2), 3 (k+2)^3 in 3D."""
    k, d = disc.k, disc.d
    pot = patches["pot"]
    col = pot[:, 0].copy()
    for j in range(d):
        col = col * (k + 2) + pot[:, 1 + j] % (k + 2)
    return col


def sweep_order(level):
    """Subdomain visiting order of the multiplicative smoother: colour-major
    (coupling-free colours), subdomain order inside a colour."""
    col = coupling_free_colours(level.disc, level.patches)
    return np.argsort(col, kind="stable")


def local_inverse_table(level):
    """Subdomain id -> (index set, M_i)."""
    out = {}
    for ids, I, M in level.groups:
        for m, i in enumerate(ids):
            out[int(i)] = (I[m], M[m])
    return out


def smooth_multiplicative(level, U, F):
    """One multiplicative Schwarz step (equation MSM), plainly sequential:
    for every subdomain i in ``sweep_order``, r_i = E_i (F - K U) with the
    current U, then U <- U + E_i^T M_i r_i (no damping)."""
    K = level.K.tocsr()
    tab = local_inverse_table(level)
    U = U.copy()
    for i in sweep_order(level):
        I, M = tab[int(i)]
        r = F[I] - K[I, :] @ U
        U[I] += M @ r
    return U


def smooth_multiplicative_colours(level, U, F):
    """The same step with the subdomains of one coupling-free colour solved
    together: one residual per colour, then every subdomain of the colour
    corrects its own DOFs.  Equal to ``smooth_multiplicative`` up to
    rounding because the subdomains of a colour neither share DOFs nor couple
    through K, so no update inside a colour changes another's residual."""
    col = coupling_free_colours(level.disc, level.patches)
    tab = local_inverse_table(level)
    for c in np.unique(col):
        r = F - level.K @ U
        dU = np.zeros_like(U)
        for i in np.nonzero(col == c)[0]:
            I, M = tab[int(i)]
            dU[I] += M @ r[I]
        U = U + dU
    return U


def _smooth_step(lv, U, F, e, smoother):
    if smoother == "additive":
        return smooth(lv, U, F, e)
    if smoother == "multiplicative":
        return smooth_multiplicative_colours(lv, U, F)
    if smoother == "multiplicative-sequential":
        return smooth_multiplicative(lv, U, F)
    raise ValueError(smoother)


def mgv(h, l, U, F, nu1, nu2, eta, smoother="additive"):
    """Algorithm 1, MGV(l, U, F); eta[l] is the damping on level l (a number,
    or a pair (pre, post) of per-step damping sequences), nu1 and nu2 the
    smoothing steps (a number, or one per level indexed by level).  smoother:
    "additive" (equation ASM with eta), "multiplicative" (equation MSM, eta
    unused; coupling-free colours at a time) or "multiplicative-sequential"
    (the same, one subdomain at a time).  Returns the updated U (the paper
    updates U in place)."""
    lv = h.levels[l]
    if l == 0:
        return lv.coarse_inv @ F
    n1 = nu1 if np.isscalar(nu1) else nu1[l]
    n2 = nu2 if np.isscalar(nu2) else nu2[l]
    e = eta[l]
    pre = list(e[0]) if isinstance(e, tuple) else [e] * n1
    post = list(e[1]) if isinstance(e, tuple) else [e] * n2
    for j in range(n1):
        U = _smooth_step(lv, U, F, pre[j], smoother)
    P = h.levels[l - 1].P
    G = P.T @ (F - lv.K @ U)
    dU = np.zeros(h.levels[l - 1].disc.n)
    dU = mgv(h, l - 1, dU, G, nu1, nu2, eta, smoother)
    U = U + P @ dU
    for j in range(n2):
        U = _smooth_step(lv, U, F, post[j], smoother)
    return U


# Fixed additive-Schwarz damping per (dimension, pressure degree k).  Read
# literally (local zero-mean pressure, plain sum of equation ASM), the smoothed
# operator S^{-1} K has its largest eigenvalues on pressure modes, because the
# local pressure corrections of all subdomains holding a pressure function are
# summed (4 subdomains in the 2D interior, 12 in 3D, up to 9 / 24 / 81 near the
# boundary): about 4.94 (2D, k=1), 9.01 (2D, k=2), 24.1 (3D, k=1) and 80.0
# (3D, k=2).  The paper's eta = 0.5 is then unstable (eta lambda_max > 2), so
# the fixed damping is the value of the sweep SWEEP_ETA with the fewest V(2,2)
# cycles to 1e-8 among those with eta lambda_max <= ETA_MARGIN, a margin below
# the stability limit 2 that covers the slow growth of lambda_max with the
# grid (24.1 on 8^3, 24.5 on 32^3 for 3D k = 1).
SWEEP_ETA = {(2, 1): (0.2, 0.25, 0.3, 0.35, 0.4), (2, 2): (0.1, 0.15, 0.2, 0.25),
             (3, 1): (0.04, 0.05, 0.06, 0.07, 0.08), (3, 2): (0.01, 0.015, 0.02, 0.025)}
ETA_MARGIN = 1.85
DEFAULT_ETA = {(2, 1): 0.35, (2, 2): 0.2, (3, 1): 0.07, (3, 2): 0.02}


def default_eta(d, k):
    return DEFAULT_ETA[(d, k)]


def eta_levels(h, eta):
    """Per-level damping array indexed by level (entry 0 unused); an entry
    given as a pair (pre, post) of per-step sequences is kept as such."""
    if eta is None:
        eta = default_eta(h.d, h.k)
    if np.isscalar(eta):
        return [float(eta)] * h.L
    eta = list(eta)
    assert len(eta) == h.L - 1, "one damping per smoothed level, finest first"
    # given finest -> coarsest; level l = L-1 .. 1
    out = [0.0] * h.L
    for i, e in enumerate(eta):
        out[h.L - 1 - i] = (tuple(e[0]), tuple(e[1])) if isinstance(e, tuple) else float(e)
    return out


def chebyshev_dampings(b, alpha, nu, reverse=False):
    """Dampings of nu additive Schwarz steps whose error polynomial in the
    preconditioned operator X = S^{-1} K is the Chebyshev polynomial of
    degree nu scaled to the interval [a, b], a = b / alpha, with value 1 at 0
    (Chebyshev semi-iteration; Adams, Brezina, Hu, Tuminaro 2003 use it as a
    multigrid smoother): prod_j (1 - x / theta_j) has the zeros theta_j of
    T_nu((b + a - 2 x) / (b - a)), so eta_j = 1 / theta_j with
    theta_j = (b + a) / 2 + (b - a) / 2 cos(pi (2 j + 1) / (2 nu)).  The steps
    take j = 0, 1, ... (largest theta first), or the reverse order."""
    a = b / alpha
    js = range(nu - 1, -1, -1) if reverse else range(nu)
    return [1.0 / ((b + a) / 2 + (b - a) / 2 * np.cos(np.pi * (2 * j + 1) / (2 * nu))) for j in js]


def chebyshev_schedule(h, lmax, alpha, nu1, nu2, safety=1.05):
    """Finest-first list of (pre, post) damping sequences for eta_levels:
    level i (finest first) has b = safety * lmax[i], ratio alpha (a number or
    alpha[i]), nu1[i] pre-smoothing dampings in the order of
    chebyshev_dampings and nu2[i] post-smoothing dampings in the reverse
    order."""
    m = h.L - 1
    n1 = [nu1] * m if np.isscalar(nu1) else list(nu1)
    n2 = [nu2] * m if np.isscalar(nu2) else list(nu2)
    al = [alpha] * m if np.isscalar(alpha) else list(alpha)
    return [(tuple(chebyshev_dampings(safety * lmax[i], al[i], n1[i])),
             tuple(chebyshev_dampings(safety * lmax[i], al[i], n2[i], reverse=True))) for i in range(m)]


def smoother_matrix(level):
    """Dense S^{-1} = sum_i E_i^T M_i E_i of a smoothed level (tiny grids)."""
    n = level.disc.n
    S = np.zeros((n, n))
    for ids, I, M in level.groups:
        for m in range(I.shape[0]):
            S[np.ix_(I[m], I[m])] += M[m]
    return S


def lmax_dense(level):
    """Largest |eigenvalue| of S^{-1} K (undamped smoother operator) of a
    smoothed level, from the dense eigenvalues (tiny grids)."""
    X = smoother_matrix(level) @ level.K.toarray()
    return float(np.max(np.abs(np.linalg.eigvals(X))))


def steps_levels(h, nu):
    """Smoothing steps indexed by level from a number or a finest-first list
    (one per smoothed level)."""
    if np.isscalar(nu):
        return nu
    nu = list(nu)
    assert len(nu) == h.L - 1, "one step count per smoothed level, finest first"
    out = [0] * h.L
    for i, s in enumerate(nu):
        out[h.L - 1 - i] = int(s)
    return out


def vcycles(h, U, F, m, nu1=2, nu2=2, eta=None, smoother="additive"):
    et = eta_levels(h, eta)
    n1, n2 = steps_levels(h, nu1), steps_levels(h, nu2)
    for _ in range(m):
        U = mgv(h, h.L - 1, U, F, n1, n2, et, smoother)
    return U


def residual_norm(h, U, F):
    return float(np.linalg.norm(F - h.finest.K @ U))


def normalize_pressure(h, U):
    """p <- p - (w^T p) * 1, so that the discrete pressure has zero integral
    (the basis is a partition of unity and |Omega| = 1)."""
    lv = h.finest
    U = U.copy()
    nv = lv.disc.n_v
    U[nv:] -= lv.w @ U[nv:]
    return U


def solve(h, F, tol=1e-8, U0=None, nu1=2, nu2=2, eta=None, max_cycles=200, smoother="additive"):
    """Repeat V-cycles until ||F - K U||_2 <= tol ||F||_2 (starting residual
    included), then normalize the pressure.  Returns (U, history)."""
    U = np.zeros_like(F) if U0 is None else U0.copy()
    et = eta_levels(h, eta)
    n1, n2 = steps_levels(h, nu1), steps_levels(h, nu2)
    fn = np.linalg.norm(F)
    hist = [residual_norm(h, U, F)]
    cycles = 0
    while hist[-1] > tol * fn and cycles < max_cycles:
        U = mgv(h, h.L - 1, U, F, n1, n2, et, smoother)
        cycles += 1
        hist.append(residual_norm(h, U, F))
    return normalize_pressure(h, U), np.array(hist)

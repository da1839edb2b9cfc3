"""Topology-respecting subdomains and local saddle-point inverses (oracle).

Follows the paper's subsection on overlapping Schwarz smoothers on compatible
subdomains: subdomain i is the support of streamfunction basis function i (2D)
or vector-potential basis function i (3D); the local spaces V_i, Q_i, Psi_i
hold every basis function whose support lies inside that subdomain; E_i
restricts to those functions; the local problem matrix is K_i = E_i K E_i^T.
The local pressure space Q_i carries the zero-mean constraint of the paper's
footnote on dim Q_i, imposed with a multiplier: the local system solved is
[[K_i, e_i], [e_i^T, 0]] with e_i = [0; w_i], w_i the integrals of the local
pressure functions; M_i is the leading block of its inverse.

Containment is tested by brute force, direction by direction, on the knot
values of the supports (a tensor-product support is the product of its
per-direction supports, so box containment is per-direction containment).
"""
import numpy as np
import scipy.sparse as sp

from .bspline import open_knots


def _contain_1d(disc, pot_degree, pot_lo, pot_hi, fun_degree, fun_lo, fun_hi):
    """Boolean (n_patch_coords, n_funcs) : support of function inside support
    of potential function, in one direction."""
    kp = open_knots(disc.N, pot_degree)
    kf = open_knots(disc.N, fun_degree)
    a = np.arange(pot_lo, pot_hi)
    i = np.arange(fun_lo, fun_hi)
    p_lo, p_hi = kp[a], kp[a + pot_degree + 1]
    f_lo, f_hi = kf[i], kf[i + fun_degree + 1]
    return (f_lo[None, :] >= p_lo[:, None]) & (f_hi[None, :] <= p_hi[:, None])


_PATCH_CACHE = {}


def build_patches(disc):
    """Subdomain DOF lists of a level, computed once per (d, N, k): they depend
    on the mesh only.  The returned arrays are shared and must not be
    modified.  See ``find_patches``."""
    key = (disc.d, disc.N, disc.k)
    if key not in _PATCH_CACHE:
        _PATCH_CACHE[key] = find_patches(disc)
    return _PATCH_CACHE[key]


def find_patches(disc):
    """Subdomain DOF lists for one level.

    Returns dict with
      ptr   (n_patch+1,)  offsets into dofs
      dofs  (sum n_i,)    global DOF indices, ascending inside each patch
      nv    (n_patch,)    number of velocity DOFs of each patch
      npsi  (n_patch,)    number of potential functions inside each patch
      pot   (n_patch, d+1) orientation and true potential multi-index
      color (n_patch,)    DOF-disjoint colour
    """
    d, k = disc.d, disc.k
    ptr, dofs, nv, npsi, pot_ids, colors = [0], [], [], [], [], []
    for o, pb in enumerate(disc.pot):
        # containment tables per (target block, direction)
        cont = []
        for b in disc.blocks + disc.pot:
            cont.append([_contain_1d(disc, pb.degrees[j], pb.lo[j], pb.hi[j],
                                     b.degrees[j], b.lo[j], b.hi[j]) for j in range(d)])
        nblk = len(disc.blocks)
        for mi in pb.multi_index():
            loc = mi - np.array(pb.lo)
            lst = []
            nvel = 0
            for bi, b in enumerate(disc.blocks):
                sel = [np.nonzero(cont[bi][j][loc[j]])[0] for j in range(d)]
                if any(s.size == 0 for s in sel):
                    continue
                grids = np.meshgrid(*sel[::-1], indexing="ij")
                idx = [g.ravel() for g in grids[::-1]]
                shape = b.shape
                flat = idx[0].copy()
                stride = 1
                for j in range(1, d):
                    stride *= shape[j - 1]
                    flat = flat + idx[j] * stride
                g = disc.offsets[bi] + np.sort(flat)
                lst.append(g)
                if bi < d:
                    nvel += g.size
            cnt_psi = 0
            for pi, b in enumerate(disc.pot):
                sel = [np.nonzero(cont[nblk + pi][j][loc[j]])[0] for j in range(d)]
                cnt_psi += int(np.prod([s.size for s in sel]))
            lst = np.concatenate(lst)
            dofs.append(lst)
            ptr.append(ptr[-1] + lst.size)
            nv.append(nvel)
            npsi.append(cnt_psi)
            pot_ids.append(np.concatenate([[o], mi]))
            m = (mi % (k + 1)).tolist()
            col = o
            for j in range(d):
                col = col * (k + 1) + m[j]
            colors.append(col)
    return {
        "ptr": np.array(ptr, dtype=np.int64),
        "dofs": np.concatenate(dofs).astype(np.int64),
        "nv": np.array(nv, dtype=np.int64),
        "npsi": np.array(npsi, dtype=np.int64),
        "pot": np.array(pot_ids, dtype=np.int64),
        "color": np.array(colors, dtype=np.int64),
    }


def submatrices(K, index_sets):
    """Dense K[I][:, I] for a stack of equal-size index sets I (m, n)."""
    K = sp.csr_matrix(K)
    K.sort_indices()
    n = K.shape[1]
    rows = np.repeat(np.arange(K.shape[0]), np.diff(K.indptr))
    keys = rows.astype(np.int64) * n + K.indices
    m, s = index_sets.shape
    q = index_sets[:, :, None].astype(np.int64) * n + index_sets[:, None, :]
    pos = np.searchsorted(keys, q.ravel())
    pos = np.minimum(pos, keys.size - 1)
    hit = keys[pos] == q.ravel()
    vals = np.where(hit, K.data[pos], 0.0)
    return vals.reshape(m, s, s)


def local_inverses(K, patches, w_pressure, n_v):
    """M_i = leading block of inv([[K_i, e_i], [e_i^T, 0]]) for every patch.

    Patches are grouped by size; returns list of (patch_ids, index_sets, M)."""
    ptr, dofs = patches["ptr"], patches["dofs"]
    sizes = np.diff(ptr)
    groups = []
    for s in np.unique(sizes):
        ids = np.nonzero(sizes == s)[0]
        I = np.stack([dofs[ptr[i]:ptr[i + 1]] for i in ids])
        Ki = submatrices(K, I)
        e = np.where(I >= n_v, w_pressure[np.maximum(I - n_v, 0)], 0.0)
        m = ids.size
        bord = np.zeros((m, s + 1, s + 1))
        bord[:, :s, :s] = Ki
        bord[:, :s, s] = e
        bord[:, s, :s] = e
        inv = np.linalg.inv(bord)
        groups.append((ids, I, inv[:, :s, :s].copy()))
    return groups

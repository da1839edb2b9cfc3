"""Compatible B-spline spaces and their canonical numbering (oracle).

Follows the paper's definition of the 2D spaces (streamfunction, velocity,
pressure) and 3D spaces (vector potential, velocity, pressure) on the unit
square / cube, with the paper's degree p of the streamfunction (2D) / scalar
potential (3D) written here as p = k + 1, k being the pressure degree:

* velocity component c: degree k+1 in direction c and k in the others; the two
  end functions in direction c are removed, which is the strong v.n = 0
  condition (only those two functions are non-zero on the faces normal to c);
* pressure: degree k in every direction; the full basis is kept and the
  zero-mean condition is imposed by a Lagrange multiplier, as the paper's
  footnote on the pressure basis says;
* 2D streamfunction: degree k+1 in both directions, both end functions removed
  (psi = 0 on the boundary);
* 3D vector-potential component o: degree k in direction o and k+1 in the
  others; the end functions are removed in every direction except o
  (psi x n = 0 on the boundary).

Global order is [u_0 | u_1 (| u_2) | p]; inside a block the multi-index runs
x fastest.
"""
import numpy as np
from dataclasses import dataclass

from .bspline import open_knots


@dataclass(frozen=True)
class Block:
    """Tensor-product block: per-direction degree and kept index range [lo, hi)."""
    degrees: tuple
    lo: tuple
    hi: tuple

    @property
    def shape(self):
        return tuple(h - l for l, h in zip(self.lo, self.hi))

    @property
    def size(self):
        return int(np.prod(self.shape))

    def multi_index(self):
        """True B-spline multi-indices of the block's functions in canonical
        order, shape (size, d), x fastest."""
        ranges = [np.arange(l, h) for l, h in zip(self.lo, self.hi)]
        grids = np.meshgrid(*ranges[::-1], indexing="ij")
        return np.stack([g.ravel() for g in grids[::-1]], axis=1)


def n_funcs(n_elem, degree):
    return n_elem + degree


def velocity_blocks(d, n_elem, k):
    blocks = []
    for c in range(d):
        deg = tuple(k + 1 if j == c else k for j in range(d))
        lo = tuple(1 if j == c else 0 for j in range(d))
        hi = tuple(n_funcs(n_elem, deg[j]) - (1 if j == c else 0) for j in range(d))
        blocks.append(Block(deg, lo, hi))
    return blocks


def pressure_block(d, n_elem, k):
    deg = (k,) * d
    return Block(deg, (0,) * d, (n_funcs(n_elem, k),) * d)


def potential_blocks(d, n_elem, k):
    """Streamfunction (2D, one block) or vector-potential components (3D)."""
    if d == 2:
        deg = (k + 1, k + 1)
        return [Block(deg, (1, 1), (n_funcs(n_elem, k + 1) - 1,) * 2)]
    blocks = []
    for o in range(3):
        deg = tuple(k if j == o else k + 1 for j in range(3))
        lo = tuple(0 if j == o else 1 for j in range(3))
        hi = tuple(n_funcs(n_elem, deg[j]) - (0 if j == o else 1) for j in range(3))
        blocks.append(Block(deg, lo, hi))
    return blocks


class Discretization:
    """All blocks of one grid level: N elements per direction, degree k."""

    def __init__(self, d, n_elem, k):
        self.d, self.N, self.k = d, n_elem, k
        self.vel = velocity_blocks(d, n_elem, k)
        self.pre = pressure_block(d, n_elem, k)
        self.pot = potential_blocks(d, n_elem, k)
        self.blocks = self.vel + [self.pre]
        sizes = [b.size for b in self.blocks]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.n_v = int(sum(b.size for b in self.vel))
        self.n_q = self.pre.size
        self.n = self.n_v + self.n_q
        self.pot_offsets = np.concatenate([[0], np.cumsum([b.size for b in self.pot])]).astype(np.int64)
        self.n_psi = int(self.pot_offsets[-1])

    def knots(self, degree):
        return open_knots(self.N, degree)

    def dofs(self):
        """DOF count used for DOF/s: dim V_h + dim Q_h = n_v + n_q - 1."""
        return self.n_v + self.n_q - 1

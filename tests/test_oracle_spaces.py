"""Pins of the oracle's space dimensions against the paper's tables and the
exactness of the discrete complexes."""
import json
import os

import numpy as np

from oracle.spaces import Discretization

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_dof_tables.json")))


def _full_counts(block):
    """Per-direction count of the spline space before boundary functions are removed."""
    return [h + (1 if l == 1 else 0) for l, h in zip(block.lo, block.hi)]


def test_2d_dof_columns_match_tables_1_and_2():
    for p, col in (("p2", GOLD["table1_2d"]["p2"]), ("p3", GOLD["table1_2d"]["p3"])):
        k = int(p[1]) - 1
        for nl, dofs in enumerate(col, start=1):
            disc = Discretization(2, 2 ** nl, k)
            assert int(np.prod(_full_counts(disc.pot[0]))) == dofs
    assert GOLD["table2_2d_additive_p2"] == GOLD["table1_2d"]["p2"]


def test_3d_dof_columns_match_table_4():
    for p in ("p2", "p3"):
        k = int(p[1]) - 1
        for nl, dofs in enumerate(GOLD["table4_3d"][p], start=1):
            disc = Discretization(3, 2 ** nl, k)
            assert sum(int(np.prod(_full_counts(b))) for b in disc.pot) == dofs


def test_exact_sequence_dimensions():
    """Euler characteristic of the exact complexes with boundary conditions:
    2D  dim Psi - dim V + dim Q = 0;  3D  dim Phi - dim Psi + dim V - dim Q = 0
    (Q carrying the zero-mean constraint, Phi the scalar potentials vanishing on
    the boundary, degree k+1)."""
    for k in (1, 2):
        for N in (1, 2, 5, 16):
            disc = Discretization(2, N, k)
            assert disc.n_psi - disc.n_v + (disc.n_q - 1) == 0
            d3 = Discretization(3, N, k)
            n_phi = (N + k - 1) ** 3
            assert n_phi - d3.n_psi + d3.n_v - (d3.n_q - 1) == 0


def test_counts_of_named_workloads():
    d = Discretization(2, 256, 2)
    assert (d.n_v, d.n_q, d.n) == (132612, 66564, 199176)
    d = Discretization(3, 32, 1)
    assert (d.n_v, d.n_q, d.n) == (104544, 35937, 140481)
    d = Discretization(2, 16, 1)
    assert d.n == 833

"""Closed forms for special networks.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* All-ones tensors (the inputs of the paper's timing experiments, §6):
  every bond assignment contributes 1, so Z = product of all bond dims.
* Product (rank-1) tensors T_s = outer product over legs of vectors u_{s,leg}:
  the sum factorises bond by bond, Z = prod over bonds <u_{a->b}, u_{b->a}>.
* Ising at K = 0: Z = 2^N.  One row of L spins: Z = 2 (2 cosh K)^(L-1).
  A 2 x 2 plaquette is a ring of 4 spins: Z = (2 cosh K)^4 + (2 sinh K)^4.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

from .network import bonds, site_bonds


def all_ones_log(rows: int, cols: int, D: int) -> float:
    nb = rows * (cols - 1) + (rows - 1) * cols
    return nb * math.log(D)


def product_sites(rows: int, cols: int, vecs: Dict[Tuple, np.ndarray]):
    """Build rank-1 sites from per-(site, bond) vectors: vecs[(r, c, bond)]."""
    out = []
    for r in range(rows):
        for c in range(cols):
            t = np.array(1.0)
            for b in site_bonds(rows, cols, r, c):
                t = np.multiply.outer(t, vecs[(r, c, b)])
            out.append(t)
    return out


def product_value(rows: int, cols: int, vecs: Dict[Tuple, np.ndarray],
                  scalars: Sequence[float] = ()) -> float:
    """Z of product_sites(...): one inner product per bond."""
    z = 1.0
    for b in bonds(rows, cols):
        kind, r, c = b
        r2, c2 = (r, c + 1) if kind == "h" else (r + 1, c)
        z *= float(np.dot(vecs[(r, c, b)], vecs[(r2, c2, b)]))
    for s in scalars:
        z *= s
    return z


def ising_row(L: int, K: float) -> float:
    return 2.0 * (2.0 * math.cosh(K)) ** (L - 1)


def ising_plaquette(K: float) -> float:
    return (2.0 * math.cosh(K)) ** 4 + (2.0 * math.sinh(K)) ** 4


def ising_zero(rows: int, cols: int) -> float:
    return 2.0 ** (rows * cols)

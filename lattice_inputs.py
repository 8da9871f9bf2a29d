"""Seeded synthetic inputs for planar Lh x Lw square-lattice tensor networks.

This module only *builds* networks (shapes, bond dimensions and tensor
entries).  It performs no contraction: both the CPU oracle and the HIP path
receive the arrays it returns, unchanged.

Conventions (the paper fixes none of them; §4 of the paper only states that
corners have order two, edges order three and bulk tensors order four):

* ``rows`` = Lh, ``cols`` = Lw; site (r, c) with (0, 0) at the top-left; sites
  are listed row-major.
* Bond ``h[r][c]`` joins (r, c)-(r, c+1); bond ``v[r][c]`` joins (r, c)-(r+1, c).
* A site tensor's legs are ordered (left, up, right, down), absent legs
  omitted, stored C-order as float64.

Generators (``numpy.random.default_rng(seed)``, PCG64, sites drawn row-major):
``uniform`` = ``rng.random``; ``normal`` = ``rng.standard_normal``; ``ones``;
``ising`` (classical Ising, h = 0); ``replica`` (leg-wise Kronecker product of
two networks, bond dims multiply).
"""
from __future__ import annotations

import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

LEFT, UP, RIGHT, DOWN = 0, 1, 2, 3


def bond_dims(rows: int, cols: int, D: int = 2,
              hdim: Optional[Sequence[Sequence[int]]] = None,
              vdim: Optional[Sequence[Sequence[int]]] = None
              ) -> Tuple[np.ndarray, np.ndarray]:
    """Return (hdim[rows][cols-1], vdim[rows-1][cols]) as int64 arrays."""
    if rows < 1 or cols < 1:
        raise ValueError("rows and cols must be >= 1")
    if hdim is None:
        h = np.full((rows, max(cols - 1, 0)), D, dtype=np.int64)
    else:
        h = np.asarray(hdim, dtype=np.int64).reshape(rows, max(cols - 1, 0))
    if vdim is None:
        v = np.full((max(rows - 1, 0), cols), D, dtype=np.int64)
    else:
        v = np.asarray(vdim, dtype=np.int64).reshape(max(rows - 1, 0), cols)
    if (h.size and h.min() < 1) or (v.size and v.min() < 1):
        raise ValueError("bond dimensions must be >= 1")
    return h, v


def site_legs(rows: int, cols: int, r: int, c: int) -> List[int]:
    """Canonical legs present at site (r, c), as LEFT/UP/RIGHT/DOWN codes."""
    legs = []
    if c > 0:
        legs.append(LEFT)
    if r > 0:
        legs.append(UP)
    if c < cols - 1:
        legs.append(RIGHT)
    if r < rows - 1:
        legs.append(DOWN)
    return legs


def site_shape(rows: int, cols: int, r: int, c: int,
               h: np.ndarray, v: np.ndarray) -> Tuple[int, ...]:
    shape = []
    for leg in site_legs(rows, cols, r, c):
        if leg == LEFT:
            shape.append(int(h[r][c - 1]))
        elif leg == UP:
            shape.append(int(v[r - 1][c]))
        elif leg == RIGHT:
            shape.append(int(h[r][c]))
        else:
            shape.append(int(v[r][c]))
    return tuple(shape)


def shapes(rows: int, cols: int, D: int = 2, hdim=None, vdim=None):
    h, v = bond_dims(rows, cols, D, hdim, vdim)
    return [site_shape(rows, cols, r, c, h, v)
            for r in range(rows) for c in range(cols)]


def uniform(rows: int, cols: int, D: int, seed: int, hdim=None, vdim=None):
    """Entries i.i.d. uniform[0, 1)."""
    rng = np.random.default_rng(seed)
    return [rng.random(s) for s in shapes(rows, cols, D, hdim, vdim)]


def normal(rows: int, cols: int, D: int, seed: int, hdim=None, vdim=None):
    """Entries i.i.d. N(0, 1)."""
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(s) for s in shapes(rows, cols, D, hdim, vdim)]


def ones(rows: int, cols: int, D: int, hdim=None, vdim=None):
    """All-ones tensors: the inputs of the paper's timing experiments."""
    return [np.ones(s) for s in shapes(rows, cols, D, hdim, vdim)]


def ising_root(K: float) -> np.ndarray:
    """Symmetric square root M of the bond Boltzmann matrix W = [[e^K, e^-K],
    [e^-K, e^K]] (spin index 0 = +1, 1 = -1), i.e. M @ M = W, K > 0."""
    if not (K > 0.0):
        raise ValueError("ising inputs need beta*J > 0")
    p = math.sqrt(2.0 * math.cosh(K))
    q = math.sqrt(2.0 * math.sinh(K))
    a = 0.5 * (p + q)
    b = 0.5 * (p - q)
    return np.array([[a, b], [b, a]])


def ising(rows: int, cols: int, K: float):
    """Classical Ising partition-function network at beta*J = K, h = 0, open
    boundaries, bond dim 2: T[i_1..i_n] = sum_s prod_k M[s, i_k]."""
    M = ising_root(K)
    out = []
    for r in range(rows):
        for c in range(cols):
            n = len(site_legs(rows, cols, r, c))
            t = np.zeros((2,) * n)
            for s in range(2):
                term = np.array(1.0)
                for _ in range(n):
                    term = np.multiply.outer(term, M[s])
                t = t + term
            out.append(t)
    return out


def replica(a: Sequence[np.ndarray], b: Sequence[np.ndarray]):
    """Leg-wise Kronecker product: new leg index = i_a * dim_b + i_b."""
    out = []
    for ta, tb in zip(a, b):
        n = ta.ndim
        assert tb.ndim == n
        t = np.multiply.outer(ta, tb)  # axes a0..a(n-1), b0..b(n-1)
        order = [x for k in range(n) for x in (k, n + k)]
        t = t.transpose(order).reshape(
            tuple(ta.shape[k] * tb.shape[k] for k in range(n)))
        out.append(np.ascontiguousarray(t))
    return out


def ising_d4(rows: int, cols: int, K: float):
    """Two-replica Ising network (bond dim 4); its value is Z(K)**2."""
    s = ising(rows, cols, K)
    return replica(s, s)


def make(kind: str, rows: int, cols: int, D: int = 2, seed: int = 0,
         K: float = 0.44):
    """One entry point used by tests and benchmarks."""
    if kind == "uniform":
        return uniform(rows, cols, D, seed)
    if kind == "normal":
        return normal(rows, cols, D, seed)
    if kind == "ones":
        return ones(rows, cols, D)
    if kind == "ising":
        if D == 2:
            return ising(rows, cols, K)
        if D == 4:
            return ising_d4(rows, cols, K)
        raise ValueError("ising networks exist for D in {2, 4}")
    raise ValueError(f"unknown input kind {kind!r}")


def batch_mix(n: int, base_seed: int, sides=(4, 8), dims=(2, 3, 4)):
    """A mixed batch of independent lattices: a master
    ``default_rng(base_seed)`` draws Lh and Lw independently and uniformly
    from ``sides`` (inclusive) and D uniformly from ``dims``; lattice i's
    entries are i.i.d. uniform[0, 1) from ``default_rng(base_seed + 1 + i)``.
    Returns a list of (rows, cols, D, sites)."""
    master = np.random.default_rng(base_seed)
    out = []
    for i in range(n):
        r = int(master.integers(sides[0], sides[1] + 1))
        c = int(master.integers(sides[0], sides[1] + 1))
        D = int(master.choice(dims))
        out.append((r, c, D, uniform(r, c, D, base_seed + 1 + i)))
    return out


# ------------------------------------------------------------------ PEPS
def peps(rows: int, cols: int, chi: int, seed: int, d: int = 2, kind: str = "normal"):
    """Real PEPS site tensors: the spin index first (dimension d), then the
    bond legs in canonical order with bond dimension chi (rank 5 in the bulk,
    4 on edges, 3 at corners).  Entries i.i.d. N(0, 1) (``kind="normal"``) or
    uniform[0, 1) (``kind="uniform"``) from ``default_rng(seed)``, row-major."""
    rng = np.random.default_rng(seed)
    draw = rng.standard_normal if kind == "normal" else rng.random
    return [draw((d,) + s) for s in shapes(rows, cols, chi)]


def spin_half():
    """Spin-1/2 operators (S^x, S^z) in the basis (up, down), S = sigma / 2."""
    sx = np.array([[0.0, 0.5], [0.5, 0.0]])
    sz = np.array([[0.5, 0.0], [0.0, -0.5]])
    return sx, sz

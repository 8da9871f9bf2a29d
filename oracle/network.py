"""The plain definition of the network value and textbook cross-checks.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Paper §4: a planar L x L (here Lh x Lw) network whose corner tensors have
order two, edge tensors order three and bulk tensors order four; physical
quantities need only the sum over all internal indices, giving a scalar.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

LEFT, UP, RIGHT, DOWN = 0, 1, 2, 3


def bonds(rows: int, cols: int) -> List[Tuple[str, int, int]]:
    """Every internal bond once: ('h', r, c) joins (r,c)-(r,c+1), ('v', r, c)
    joins (r,c)-(r+1,c)."""
    out = [("h", r, c) for r in range(rows) for c in range(cols - 1)]
    out += [("v", r, c) for r in range(rows - 1) for c in range(cols)]
    return out


def site_bonds(rows: int, cols: int, r: int, c: int) -> List[Tuple[str, int, int]]:
    """The bonds on the legs of site (r, c) in canonical (left, up, right,
    down) order, absent legs omitted (§4: order 2 / 3 / 4 by position)."""
    out = []
    if c > 0:
        out.append(("h", r, c - 1))
    if r > 0:
        out.append(("v", r - 1, c))
    if c < cols - 1:
        out.append(("h", r, c))
    if r < rows - 1:
        out.append(("v", r, c))
    return out


def dims_of(sites: Sequence[np.ndarray], rows: int, cols: int) -> Dict:
    """Read bond dimensions off the site shapes and check that both ends of
    every bond agree (the network is well formed)."""
    d: Dict = {}
    if len(sites) != rows * cols:
        raise ValueError("site count does not match the grid")
    for r in range(rows):
        for c in range(cols):
            t = sites[r * cols + c]
            bl = site_bonds(rows, cols, r, c)
            if t.ndim != len(bl):
                raise ValueError(f"site ({r},{c}) has order {t.ndim}, expected {len(bl)}")
            for b, n in zip(bl, t.shape):
                if d.setdefault(b, n) != n:
                    raise ValueError(f"bond {b} has mismatched dimensions")
    return d


def brute_bonds(sites: Sequence[np.ndarray], rows: int, cols: int,
                chunk: int = 1 << 18) -> float:
    """Z as literally defined: the sum, over every assignment of every bond
    index, of the product of all site entries (§4).  Cost D^#bonds; use only
    for tiny networks.  Pinned by: the Ising spin sum and closed forms."""
    d = dims_of(sites, rows, cols)
    bl = bonds(rows, cols)
    radix = [d[b] for b in bl]
    pos = {b: i for i, b in enumerate(bl)}
    total_assign = 1
    for x in radix:
        total_assign *= x
    if total_assign > (1 << 26):
        raise ValueError("too many bond assignments for brute force")
    flat = [np.asarray(t, dtype=np.float64) for t in sites]
    z = 0.0
    for start in range(0, total_assign, chunk):
        idx = np.arange(start, min(start + chunk, total_assign), dtype=np.int64)
        digits = np.empty((len(bl), idx.size), dtype=np.int64)
        rem = idx.copy()
        for i in range(len(bl) - 1, -1, -1):
            digits[i] = rem % radix[i]
            rem //= radix[i]
        prod = np.ones(idx.size)
        for r in range(rows):
            for c in range(cols):
                t = flat[r * cols + c]
                sb = site_bonds(rows, cols, r, c)
                if sb:
                    prod *= t[tuple(digits[pos[b]] for b in sb)]
                else:
                    prod *= float(t)
        z += float(prod.sum())
    return z


def brute_spins(rows: int, cols: int, K: float) -> float:
    """Classical Ising partition function with open boundaries and no field:
    Z = sum over s in {+1,-1}^N of exp(K * sum over nearest-neighbour pairs of
    s_i s_j).  This is the h = 0 spin-spin term of the paper's Hamiltonian
    (§3), read as a classical Boltzmann sum.  N <= 22."""
    n = rows * cols
    if n > 22:
        raise ValueError("too many spins for brute force")
    cfg = np.arange(1 << n, dtype=np.int64)
    spin = np.empty((n, cfg.size), dtype=np.int8)
    for k in range(n):
        spin[k] = 1 - 2 * ((cfg >> k) & 1)
    energy = np.zeros(cfg.size, dtype=np.int64)
    for r in range(rows):
        for c in range(cols):
            k = r * cols + c
            if c + 1 < cols:
                energy += spin[k].astype(np.int64) * spin[k + 1]
            if r + 1 < rows:
                energy += spin[k].astype(np.int64) * spin[k + cols]
    return float(np.exp(K * energy.astype(np.float64)).sum())


def transfer_log_z(rows: int, cols: int, K: float) -> float:
    """log Z of the open-boundary Ising model by the textbook row transfer
    matrix: psi over the 2^cols configurations of one row; each new row
    applies the vertical Boltzmann factor one column at a time (a 2x2 matrix
    on one spin axis) and then the new row's horizontal factor; psi is
    rescaled by its maximum after each row and the log accumulated.
    Exact in FP64 up to rounding; cols <= 20."""
    if cols > 20:
        raise ValueError("row too wide for the transfer matrix")
    n = cols
    cfg = np.arange(1 << n, dtype=np.int64)
    # spin of column j in configuration cfg: bit (n-1-j) of cfg (0 -> +1)
    sp = np.stack([1 - 2 * ((cfg >> (n - 1 - j)) & 1) for j in range(n)])
    horiz = np.zeros(cfg.size)
    for j in range(n - 1):
        horiz += sp[j] * sp[j + 1]
    hw = np.exp(K * horiz)
    W = np.array([[math.exp(K), math.exp(-K)], [math.exp(-K), math.exp(K)]])
    psi = hw.copy()
    logz = 0.0
    for _ in range(rows - 1):
        t = psi.reshape((2,) * n)
        for j in range(n):
            t = np.tensordot(W, t, axes=([1], [j]))   # new axis 0
            t = np.moveaxis(t, 0, j)
        psi = t.reshape(-1) * hw
        m = psi.max()
        logz += math.log(m)
        psi = psi / m
    return logz + math.log(psi.sum())


def einsum_value(sites: Sequence[np.ndarray], rows: int, cols: int) -> float:
    """Z through numpy.einsum over every bond at once, with numpy choosing
    the pairwise order ('optimal' path search off, greedy on): a library
    routine applied to the plain definition, for mid-sized cross-checks."""
    dims_of(sites, rows, cols)
    names = {}
    letters = [chr(c) for c in range(ord('a'), ord('z') + 1)] + \
              [chr(c) for c in range(ord('A'), ord('Z') + 1)]
    if len(bonds(rows, cols)) > len(letters):
        raise ValueError("einsum supports at most 52 bonds")
    for b in bonds(rows, cols):
        names[b] = letters[len(names)]
    ops = []
    subs = []
    for r in range(rows):
        for c in range(cols):
            subs.append("".join(names[b] for b in site_bonds(rows, cols, r, c)))
            ops.append(sites[r * cols + c])
    expr = ",".join(subs) + "->"
    return float(np.einsum(expr, *ops, optimize="greedy"))

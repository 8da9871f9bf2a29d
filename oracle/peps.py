"""Norm and expectation-value networks of a real PEPS, in FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper (§3) represents the amplitudes A({sigma}) of an N-spin state as a
planar network of rank-5 tensors (four bonds and the spin index; three and
two bonds on edges and corners).  The norm is the sum over all spin
configurations of A* A; the local magnetisations are m^x_k = <S^x_k> and
m^z_k = <S^z_k>, and the correlation of a pair is
c_ij = <S^z_i S^z_j> - <S^z_i><S^z_j>, each <O> being <Psi|O|Psi> / <Psi|Psi>.
§5 computes each of these by contracting O|Psi> with <Psi| along every spin
index: one planar network per site (m^x) and per nearest-neighbour pair
(c_ij), L^2 and 2L(L-1) of them on an L x L lattice.

Contracting the spin index of a site between the ket layer, the operator and
the bra layer leaves a single-layer site whose every bond pairs a ket index a
and a bra index a' (dimension chi^2):

    E[(a_1 a_1') ... (a_r a_r')] = sum_{s, s'} A[s][a_1..a_r] O[s'][s] A[s'][a_1'..a_r']

(O = identity for the norm), so every network here is a planar network of
the kind ``contract.py`` evaluates.

Readings where the paper is silent:
  * tensors are real (A* = A), as imaginary-time evolution of a real
    Hamiltonian from a real state keeps them;
  * the paired bond index is a * chi + a' (ket-major), on both ends of a bond;
  * spin operators are S = sigma / 2 in the basis (up, down);
  * the pairs of c_ij are the nearest-neighbour bonds, the 2L(L-1) pairs §5
    counts.
"""
from __future__ import annotations

import math
import string
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import contract as C
from . import plan as P


def double_layer(A: np.ndarray, op: Optional[np.ndarray] = None) -> np.ndarray:
    """The single-layer site of one PEPS tensor A[s][legs] with the operator
    O[s'][s] (identity if None) between ket and bra: legs of dimension chi^2,
    index a * chi + a'."""
    A = np.asarray(A, dtype=np.float64)
    d = A.shape[0]
    legs = A.shape[1:]
    O = np.eye(d) if op is None else np.asarray(op, dtype=np.float64)
    # (O A)[s'][a] = sum_s O[s'][s] A[s][a]: the operator acts on the ket
    OA = np.tensordot(O, A, axes=([1], [0]))
    # sum over s' of (O A)[s'][a] A[s'][a']: legs a_1..a_r then a_1'..a_r'
    E = np.tensordot(OA, A, axes=([0], [0]))
    r = len(legs)
    E = E.transpose([x for i in range(r) for x in (i, r + i)])
    return E.reshape(tuple(n * n for n in legs)).copy()   # C-contiguous, rank 0 kept


def network(peps: Sequence[np.ndarray], ops: Optional[Dict[int, np.ndarray]] = None):
    """Single-layer sites of <Psi| prod_k O_k |Psi>; ops maps a site index
    (row-major) to its operator, the other sites get the identity."""
    ops = ops or {}
    return [double_layer(A, ops.get(i)) for i, A in enumerate(peps)]


def ratio(num: C.Result, den: C.Result) -> float:
    """num / den for two exact contraction results (mantissa * 2^exp2)."""
    if den.sign == 0:
        raise ZeroDivisionError("zero norm")
    if num.sign == 0:
        return 0.0
    return num.sign * den.sign * math.ldexp(abs(num.mantissa) / abs(den.mantissa),
                                            num.exp2 - den.exp2)


def bonds(rows: int, cols: int):
    """Nearest-neighbour pairs (i, j), i < j, site index = r * cols + c:
    horizontal bonds row by row, then vertical bonds."""
    out = [(r * cols + c, r * cols + c + 1) for r in range(rows) for c in range(cols - 1)]
    out += [(r * cols + c, (r + 1) * cols + c) for r in range(rows - 1) for c in range(cols)]
    return out


def networks_for_observables(peps, rows: int, cols: int, sx, sz):
    """All networks of one observable evaluation, in this order: the norm,
    S^x at every site, S^z at every site, S^z S^z on every bond."""
    n = rows * cols
    out = [network(peps)]
    out += [network(peps, {k: sx}) for k in range(n)]
    out += [network(peps, {k: sz}) for k in range(n)]
    out += [network(peps, {i: sz, j: sz}) for i, j in bonds(rows, cols)]
    return out


def observables(results: Sequence[C.Result], rows: int, cols: int):
    """m^x, m^z (per site) and c_ij (per bond) from the results of the
    networks of ``networks_for_observables``, in that order."""
    n = rows * cols
    norm = results[0]
    mx = [ratio(results[1 + k], norm) for k in range(n)]
    mz = [ratio(results[1 + n + k], norm) for k in range(n)]
    czz = []
    for b, (i, j) in enumerate(bonds(rows, cols)):
        czz.append(ratio(results[1 + 2 * n + b], norm) - mz[i] * mz[j])
    return {"norm": norm, "mx": mx, "mz": mz, "czz": czz}


def expectation_values(peps, rows: int, cols: int, sx, sz, order=P.COLSWEEP):
    """m^x, m^z and c_ij of the state, each network contracted by ``contract``."""
    nets = networks_for_observables(peps, rows, cols, sx, sz)
    return observables([C.contract_grid(s, rows, cols, order) for s in nets], rows, cols)


def amplitudes(peps: Sequence[np.ndarray], rows: int, cols: int) -> np.ndarray:
    """Brute force: the amplitude A(s_1 .. s_N) of every spin configuration,
    the sum over all bond indices of the product of the site tensors (one
    einsum over all bond letters).  Axis k of the result is the spin of site k
    (row-major).  Tiny lattices only."""
    letters = iter(string.ascii_letters)
    hb = {(r, c): next(letters) for r in range(rows) for c in range(cols - 1)}
    vb = {(r, c): next(letters) for r in range(rows - 1) for c in range(cols)}
    phys = []
    terms = []
    for r in range(rows):
        for c in range(cols):
            s = next(letters)
            phys.append(s)
            sub = s
            if c > 0:
                sub += hb[(r, c - 1)]
            if r > 0:
                sub += vb[(r - 1, c)]
            if c < cols - 1:
                sub += hb[(r, c)]
            if r < rows - 1:
                sub += vb[(r, c)]
            terms.append(sub)
    spec = ",".join(terms) + "->" + "".join(phys)
    return np.einsum(spec, *[np.asarray(t, dtype=np.float64) for t in peps])


def apply_site(psi: np.ndarray, k: int, op: np.ndarray) -> np.ndarray:
    """(O_k psi)[.., s', ..] = sum_s O[s'][s] psi[.., s, ..] on spin axis k."""
    return np.moveaxis(np.tensordot(op, psi, axes=([1], [k])), 0, k)

"""Imaginary-time evolution of a PEPS and exact diagonalisation, in FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The model (§3): the transverse-field Ising model on an open rows x cols
lattice, H = H_J + H_Gamma with H_J = -J sum_<ij> S^z_i S^z_j over nearest
neighbours and H_Gamma = -Gamma sum_i S^x_i.  §3 gives S^z the values +1 and
-1 and puts the critical point near Gamma = 3J; both hold for the Pauli
matrices, so S = sigma here, in the basis (up, down).

The method (§5): starting from the uniform superposition of product states
(bond dimension 1), repeat m times the second-order Trotter-Suzuki step
U = U^Gamma(dtau/2) U^J(dtau) U^Gamma(dtau/2), with U^Gamma = exp(-H_Gamma t)
a product of one-body gates contracted into each site's spin index, and
U^J = exp(-H_J dtau) a product of two-body gates, one per nearest-neighbour
pair: the two sites are contracted over their shared bond and the gate over
their spin indices, the result is folded into a matrix (one site's open
indices against the other's), decomposed by a singular value decomposition,
and the two sites are replaced by U sqrt(lambda) and sqrt(lambda) V^T.  The
state is normalised after each set of operators; the energy <H> is
evaluated every two steps.

Readings where the paper is silent:
  * truncation: singular values below eps times the largest are dropped
    (eps = 0.01 in §6), and at most chi_max are kept; every bond is stored
    with chi_max entries, the dropped ones as zeros (a zero-padded bond gives
    the same network values);
  * the order of the pair gates: all horizontal bonds whose left site is in
    an even column, then those in an odd column, then vertical bonds whose
    upper site is in an even row, then odd rows (the gates of one class
    touch disjoint sites);
  * the sign of each kept singular pair: the first entry of the left vector
    whose magnitude exceeds 1e-6 of its largest is made positive;
  * normalisation: every site tensor is scaled by N_sites-th root of
    1 / sqrt(<Psi|Psi>), so the state's norm becomes 1;
  * the energy is -J sum_<ij> <S^z_i S^z_j> - Gamma sum_i <S^x_i>, from the
    expectation-value networks of §5.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

from . import contract as C
from . import peps as Q
from . import plan as P

SX = np.array([[0.0, 1.0], [1.0, 0.0]])
SZ = np.array([[1.0, 0.0], [0.0, -1.0]])


# ---------------------------------------------------------------- exact
def hamiltonian(rows: int, cols: int, J: float, gamma: float) -> np.ndarray:
    """Dense H on all 2^N configurations; bit k of the basis index is the
    spin of site k (row-major), 0 = up (S^z = +1), 1 = down."""
    n = rows * cols
    dim = 1 << n
    idx = np.arange(dim)
    spin = 1 - 2 * ((idx[:, None] >> np.arange(n)[None, :]) & 1)   # +1 / -1
    diag = np.zeros(dim)
    for i, j in Q.bonds(rows, cols):
        diag -= J * spin[:, i] * spin[:, j]
    H = np.diag(diag.astype(np.float64))
    for k in range(n):
        H[idx, idx ^ (1 << k)] -= gamma
    return H


def ground_energy(rows: int, cols: int, J: float, gamma: float) -> float:
    """Lowest eigenvalue of H by dense diagonalisation (N <= 12)."""
    return float(np.linalg.eigvalsh(hamiltonian(rows, cols, J, gamma))[0])


def chain_ground_energy(L: int, J: float, gamma: float) -> float:
    """Textbook free-fermion solution of the open chain (a 1 x L lattice):
    after the Jordan-Wigner transformation H is quadratic in fermions and
    E0 = -sum_k e_k, with e_k the singular values of the L x L bidiagonal
    matrix with gamma on the diagonal and J on the superdiagonal."""
    B = np.diag(np.full(L, float(gamma))) + np.diag(np.full(L - 1, float(J)), 1)
    return -float(np.sum(np.linalg.svd(B, compute_uv=False)))


# ------------------------------------------------------------------ gates
def gate_one(gamma: float, t: float) -> np.ndarray:
    """exp(-t H_Gamma) on one site: exp(gamma t sigma^x)."""
    return math.cosh(gamma * t) * np.eye(2) + math.sinh(gamma * t) * SX


def gate_two(J: float, t: float) -> np.ndarray:
    """exp(-t H_J) on one pair, G[(s'_i s'_j)][(s_i s_j)] (s_i slowest):
    diagonal with exp(J t s_i s_j)."""
    z = np.array([1.0, -1.0])
    return np.diag(np.exp(J * t * np.outer(z, z).reshape(-1)))


# ------------------------------------------------------------------ state
def product_state(rows: int, cols: int, chi_max: int) -> List[np.ndarray]:
    """The uniform superposition prod_k (|up> + |down>) / sqrt(2): bond
    dimension 1, stored zero-padded to chi_max."""
    out = []
    for r in range(rows):
        for c in range(cols):
            rank = (c > 0) + (r > 0) + (c < cols - 1) + (r < rows - 1)
            A = np.zeros((2,) + (chi_max,) * rank)
            A[(slice(None),) + (0,) * rank] = 1.0 / math.sqrt(2.0)
            out.append(A)
    return out


def _leg_axis(rows, cols, k, leg):
    """Axis of canonical leg (0 left, 1 up, 2 right, 3 down) in site k's
    tensor (axis 0 is the spin)."""
    r, c = divmod(k, cols)
    present = [c > 0, r > 0, c < cols - 1, r < rows - 1]
    assert present[leg]
    return 1 + sum(present[:leg])


def apply_one(peps: Sequence[np.ndarray], G: np.ndarray) -> List[np.ndarray]:
    """A'[s'] = sum_s G[s'][s] A[s] at every site."""
    return [np.tensordot(G, A, axes=([1], [0])) for A in peps]


def apply_two(peps: List[np.ndarray], rows: int, cols: int, i: int, j: int, G: np.ndarray,
              chi_max: int, eps: float) -> Tuple[List[np.ndarray], int]:
    """The pair gate on sites i < j (j to the right of or below i), split
    back by an SVD; returns the new state and the number of kept values."""
    horizontal = j == i + 1
    li, lj = (2, 0) if horizontal else (3, 1)          # shared legs
    ai, aj = _leg_axis(rows, cols, i, li), _leg_axis(rows, cols, j, lj)
    Ai = np.moveaxis(peps[i], ai, -1)                  # [s_i][rest_i][b]
    Aj = np.moveaxis(peps[j], aj, 1)                   # [s_j][b][rest_j]
    ri, rj = Ai.shape[1:-1], Aj.shape[2:]
    chi = Ai.shape[-1]
    # theta[s_i][rest_i][s_j][rest_j] = sum_b Ai Aj, then the gate on (s_i, s_j)
    th = np.tensordot(Ai, Aj, axes=([Ai.ndim - 1], [1]))
    th = np.moveaxis(th, 1 + len(ri), 1)               # [s_i][s_j][rest_i][rest_j]
    shp = th.shape
    th = np.tensordot(G, th.reshape((4,) + shp[2:]), axes=([1], [0])).reshape(shp)
    th = np.moveaxis(th, 1, 1 + len(ri))               # [s_i][rest_i][s_j][rest_j]
    m = 2 * int(np.prod(ri, dtype=np.int64))
    M = th.reshape(m, -1)
    U, lam, Vt = np.linalg.svd(M, full_matrices=False)
    keep = 0
    while keep < min(chi_max, len(lam)) and lam[keep] > 0 and lam[keep] >= eps * lam[0]:
        keep += 1
    Ui = np.zeros((m, chi))
    Vj = np.zeros((chi, M.shape[1]))
    for q in range(keep):
        u, v = U[:, q], Vt[q, :]
        p = int(np.argmax(np.abs(u) > 1e-6 * np.max(np.abs(u))))
        if u[p] < 0:
            u, v = -u, -v
        Ui[:, q] = u * math.sqrt(lam[q])
        Vj[q, :] = math.sqrt(lam[q]) * v
    out = list(peps)
    out[i] = np.moveaxis(Ui.reshape((2,) + ri + (chi,)), -1, ai)
    out[j] = np.moveaxis(Vj.reshape((chi, 2) + rj), 0, 1)
    out[j] = np.moveaxis(out[j], 1, aj)
    return out, keep


def bond_classes(rows: int, cols: int) -> List[List[Tuple[int, int]]]:
    """Nearest-neighbour pairs in the order the pair gates are applied."""
    h = [[(r * cols + c, r * cols + c + 1) for r in range(rows) for c in range(cols - 1)
          if c % 2 == par] for par in (0, 1)]
    v = [[(r * cols + c, (r + 1) * cols + c) for r in range(rows - 1) for c in range(cols)
          if r % 2 == par] for par in (0, 1)]
    return [x for x in h + v if x]


def norm(peps, rows: int, cols: int) -> C.Result:
    """<Psi|Psi> by contracting the double-layer network (§5)."""
    return C.contract_grid(Q.network(peps), rows, cols, P.COLSWEEP)


def normalize(peps, rows: int, cols: int) -> List[np.ndarray]:
    """|Psi> -> |Psi> / sqrt(<Psi|Psi>), the factor shared by all sites."""
    z = norm(peps, rows, cols)
    f = math.exp(-z.log_abs / (2 * rows * cols))
    return [A * f for A in peps]


def energy(peps, rows: int, cols: int, J: float, gamma: float) -> float:
    """<H> / <Psi|Psi> from the expectation-value networks of §5."""
    ev = Q.expectation_values(peps, rows, cols, SX, SZ)
    zz = [c + ev["mz"][i] * ev["mz"][j] for c, (i, j) in zip(ev["czz"], Q.bonds(rows, cols))]
    return -J * float(np.sum(zz)) - gamma * float(np.sum(ev["mx"]))


def ite_step(peps, rows: int, cols: int, J: float, gamma: float, dtau: float, chi_max: int,
             eps: float) -> List[np.ndarray]:
    """One Trotter step U^Gamma(dtau/2) U^J(dtau) U^Gamma(dtau/2), normalised
    after each set of operators."""
    g1 = gate_one(gamma, dtau / 2)
    g2 = gate_two(J, dtau)
    peps = normalize(apply_one(peps, g1), rows, cols)
    for cls in bond_classes(rows, cols):
        for i, j in cls:
            peps, _ = apply_two(peps, rows, cols, i, j, g2, chi_max, eps)
    peps = normalize(peps, rows, cols)
    return normalize(apply_one(peps, g1), rows, cols)


def ite(rows: int, cols: int, J: float, gamma: float, tau: float, steps: int, chi_max: int,
        eps: float = 0.01, energy_every: int = 2):
    """Evolve the product state for `steps` steps of dtau = tau / steps;
    returns the final state and [(step, energy)] every `energy_every` steps."""
    dtau = tau / steps
    peps = product_state(rows, cols, chi_max)
    out = []
    for k in range(1, steps + 1):
        peps = ite_step(peps, rows, cols, J, gamma, dtau, chi_max, eps)
        if energy_every and k % energy_every == 0:
            out.append((k, energy(peps, rows, cols, J, gamma)))
    return peps, out

"""Pins of the imaginary-time-evolution and exact-diagonalisation oracle
(paper §3 and §5) against results that do not go through it.

* Exact diagonalisation: the open chain's free-fermion solution, two spins
  in closed form, and the limits J = 0 (E0 = -Gamma N) and Gamma = 0
  (E0 = -J times the number of bonds).
* One pair gate with room for the full Schmidt rank: the state it leaves,
  contracted to amplitudes by brute force, equals the gate applied to the
  amplitude tensor directly.
* Chains of two and three spins at chi = 2 never truncate: the evolution is
  exact up to the Trotter error (a state error of second order in dtau, so
  an energy error of fourth order: halving dtau divides it by about 16) and
  reaches the exact ground energy.
* The regime of the paper's comparison with exact diagonalisation (§6,
  Fig. 4: 2 x 2 and 3 x 3, chi = 2, tau = 3, 200 steps, J = 1): the energy
  is variational (never below E0) and within 2 % of it, and halving dtau
  moves it by less than 1e-3 of E0.
* Planted mistakes (a one-body gate of the wrong sign, a pair gate on the
  wrong legs) fail these pins.
"""
import math

import numpy as np
import pytest

from oracle import ite as I
from oracle import peps as Q


@pytest.mark.parametrize("L", [2, 3, 4, 6, 9])
@pytest.mark.parametrize("J,G", [(1.0, 0.5), (1.0, 1.0), (0.7, 2.0), (1.0, 3.0)])
def test_ed_matches_free_fermion_chain(L, J, G):
    assert abs(I.ground_energy(1, L, J, G) - I.chain_ground_energy(L, J, G)) <= 1e-12 * L


def test_ed_closed_forms_and_limits():
    for J, G in [(1.0, 0.5), (0.3, 1.7)]:
        assert abs(I.ground_energy(1, 2, J, G) + math.sqrt(J * J + 4 * G * G)) <= 1e-13
    for r, c in [(2, 2), (2, 3), (3, 3)]:
        nb = len(Q.bonds(r, c))
        assert abs(I.ground_energy(r, c, 0.0, 1.3) + 1.3 * r * c) <= 1e-12
        assert abs(I.ground_energy(r, c, 0.8, 0.0) + 0.8 * nb) <= 1e-12
        H = I.hamiltonian(r, c, 1.0, 0.7)
        assert np.array_equal(H, H.T)
        plus = np.full(H.shape[0], 2.0 ** (-r * c / 2))     # |+...+>: <H> = -Gamma N
        assert abs(plus @ H @ plus + 0.7 * r * c) <= 1e-12


def _amp(peps, rows, cols):
    return Q.amplitudes(peps, rows, cols)


@pytest.mark.parametrize("rows,cols,pair", [(1, 2, (0, 1)), (2, 2, (0, 1)), (2, 2, (1, 3)),
                                            (2, 3, (1, 2)), (3, 3, (4, 7)), (3, 3, (3, 4))])
def test_pair_gate_exact_with_room(rows, cols, pair):
    # bond dimension 1 stored in chi_max = 2: the gated pair has Schmidt rank
    # at most 2 across the bond, so nothing is truncated
    rng = np.random.default_rng(rows * 10 + cols)
    peps = I.product_state(rows, cols, 2)
    peps = [np.where(A != 0, rng.standard_normal(A.shape), 0.0) for A in peps]
    i, j = pair
    G = I.gate_two(0.9, 0.3) @ np.kron(I.gate_one(0.4, 0.2), np.eye(2))   # not diagonal
    new, keep = I.apply_two(peps, rows, cols, i, j, G, 2, 0.0)
    assert keep == 2
    psi = _amp(peps, rows, cols)
    want = np.moveaxis(np.tensordot(G.reshape(2, 2, 2, 2), np.moveaxis(psi, [i, j], [0, 1]),
                                    axes=([2, 3], [0, 1])), [0, 1], [i, j])
    got = _amp(new, rows, cols)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


@pytest.mark.parametrize("cols,G", [(2, 1.0), (3, 0.6), (3, 1.5)])
def test_untruncated_chain_converges_at_second_order(cols, G):
    E0 = I.ground_energy(1, cols, 1.0, G)
    errs = []
    for steps in (100, 200):
        _, es = I.ite(1, cols, 1.0, G, 8.0, steps, 2, 0.0, energy_every=steps)
        errs.append(es[-1][1] - E0)
    assert errs[0] >= -1e-12 and errs[1] >= -1e-12        # variational
    assert errs[1] <= 1e-5 * abs(E0)
    # the second-order product formula leaves a state error O(dtau^2), and
    # the energy error is quadratic in it: halving dtau divides it by ~16
    assert 12.0 <= errs[0] / errs[1] <= 20.0


def test_no_coupling_keeps_the_product_ground_state():
    peps, es = I.ite(3, 3, 0.0, 1.3, 1.0, 10, 2, 0.01)
    assert all(abs(e + 1.3 * 9) <= 1e-12 for _, e in es)
    assert abs(I.norm(peps, 3, 3).log_abs) <= 1e-12


@pytest.mark.parametrize("rows,cols", [(2, 2), (3, 3)])
@pytest.mark.parametrize("G", [0.5, 1.0, 2.0])
def test_paper_regime_agrees_with_exact_diagonalisation(rows, cols, G):
    E0 = I.ground_energy(rows, cols, 1.0, G)
    e = {}
    for steps in (200, 400):
        _, es = I.ite(rows, cols, 1.0, G, 3.0, steps, 2, 1e-10, energy_every=steps)
        e[steps] = es[-1][1]
    assert e[200] >= E0 - 1e-10
    assert (e[200] - E0) <= 0.02 * abs(E0)
    assert abs(e[200] - e[400]) <= 1e-3 * abs(E0)


def test_pins_catch_a_wrong_sign_one_body_gate(monkeypatch):
    E0 = I.ground_energy(2, 2, 1.0, 1.0)
    real = I.gate_one
    monkeypatch.setattr(I, "gate_one", lambda g, t: real(g, -t))
    _, es = I.ite(2, 2, 1.0, 1.0, 3.0, 100, 2, 1e-10, energy_every=100)
    assert es[-1][1] - E0 > 0.1 * abs(E0)


def test_pins_catch_a_pair_gate_on_the_wrong_legs(monkeypatch):
    rows, cols = 2, 2
    rng = np.random.default_rng(3)
    peps = [np.where(A != 0, rng.standard_normal(A.shape), 0.0)
            for A in I.product_state(rows, cols, 2)]
    G = I.gate_two(0.9, 0.3) @ np.kron(I.gate_one(0.4, 0.2), np.eye(2))
    psi = _amp(peps, rows, cols)
    # the vertical pair (0, 2): site 0's down leg is its second bond axis
    want = np.moveaxis(np.tensordot(G.reshape(2, 2, 2, 2), np.moveaxis(psi, [0, 2], [0, 1]),
                                    axes=([2, 3], [0, 1])), [0, 1], [0, 2])
    good, _ = I.apply_two(peps, rows, cols, 0, 2, G, 2, 0.0)
    assert np.max(np.abs(_amp(good, rows, cols) - want)) <= 1e-13 * np.max(np.abs(want))
    monkeypatch.setattr(I, "_leg_axis", lambda r, c, k, leg: 1)   # always the first leg
    new, _ = I.apply_two(peps, rows, cols, 0, 2, G, 2, 0.0)
    assert np.max(np.abs(_amp(new, rows, cols) - want)) > 1e-6

"""Pins of the PEPS norm / observable oracle (paper §3 and §5) against
definitions that do not go through it.

* Brute force: the amplitude of every spin configuration (one einsum over
  all bonds) gives <Psi|Psi>, <S^x_k>, <S^z_k> and c_ij directly; the
  double-layer networks, contracted by the plan-following oracle, must agree.
  A site whose ket and bra bond indices were paired differently from its
  neighbour's, an operator on the wrong site or a dropped term fails here.
* Product states (chi = 1): the norm is the product of the local norms and
  every <O_k> is a^T O a / a^T a of site k alone, at sizes brute force cannot
  reach; c_ij of a product state is 0.
* The norm site (no operator) is symmetric under swapping ket and bra.
"""
import math

import numpy as np
import pytest

import lattice_inputs as li
from oracle import contract as C
from oracle import peps as Q
from oracle import plan as P

SX, SZ = li.spin_half()


def brute_observables(peps, rows, cols):
    psi = Q.amplitudes(peps, rows, cols)
    norm = float(np.vdot(psi, psi))
    n = rows * cols
    mx = [float(np.vdot(psi, Q.apply_site(psi, k, SX))) / norm for k in range(n)]
    mz = [float(np.vdot(psi, Q.apply_site(psi, k, SZ))) / norm for k in range(n)]
    czz = []
    for i, j in Q.bonds(rows, cols):
        zz = float(np.vdot(psi, Q.apply_site(Q.apply_site(psi, j, SZ), i, SZ))) / norm
        czz.append(zz - mz[i] * mz[j])
    return norm, mx, mz, czz


@pytest.mark.parametrize("rows,cols,seed", [(2, 2, 0), (2, 3, 1), (3, 2, 2), (3, 3, 3)])
@pytest.mark.parametrize("order", [P.COLSWEEP, P.HEURISTIC])
def test_observables_equal_brute_force(rows, cols, seed, order):
    peps = li.peps(rows, cols, 2, seed)
    norm, mx, mz, czz = brute_observables(peps, rows, cols)
    got = Q.expectation_values(peps, rows, cols, SX, SZ, order)
    assert got["norm"].value == pytest.approx(norm, rel=1e-12)
    np.testing.assert_allclose(got["mx"], mx, rtol=0, atol=1e-12)
    np.testing.assert_allclose(got["mz"], mz, rtol=0, atol=1e-12)
    np.testing.assert_allclose(got["czz"], czz, rtol=0, atol=1e-12)
    # the brute-force values are not trivially zero
    assert max(abs(x) for x in mx) > 1e-3 and max(abs(x) for x in czz) > 1e-4


def test_general_operator_pair_equals_brute_force():
    # two different non-symmetric operators on two sites of a 3x3 chi=2 state
    rows, cols = 3, 3
    peps = li.peps(rows, cols, 2, 11)
    o1 = np.array([[0.3, -1.1], [0.7, 0.2]])
    o2 = np.array([[-0.4, 0.9], [0.1, 1.3]])
    psi = Q.amplitudes(peps, rows, cols)
    want = float(np.vdot(psi, Q.apply_site(Q.apply_site(psi, 7, o2), 2, o1)))
    got = C.contract_grid(Q.network(peps, {2: o1, 7: o2}), rows, cols, P.COLSWEEP)
    assert got.value == pytest.approx(want, rel=1e-12)


@pytest.mark.parametrize("rows,cols", [(4, 5), (6, 6)])
def test_product_state_closed_form(rows, cols):
    peps = li.peps(rows, cols, 1, 5, kind="uniform")
    vecs = [A.reshape(-1) for A in peps]
    local = [float(a @ a) for a in vecs]
    got = Q.expectation_values(peps, rows, cols, SX, SZ)
    want_log = sum(math.log(x) for x in local)
    assert got["norm"].log_abs == pytest.approx(want_log, rel=1e-13)
    np.testing.assert_allclose(got["mx"], [float(a @ SX @ a) / n for a, n in zip(vecs, local)],
                               rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(got["mz"], [float(a @ SZ @ a) / n for a, n in zip(vecs, local)],
                               rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(got["czz"], 0.0, atol=1e-14)
    assert len(got["czz"]) == 2 * rows * cols - rows - cols


@pytest.mark.parametrize("shape", [(2,), (2, 3), (2, 2, 3), (3, 2, 2, 2), (2, 2, 3, 2, 2)])
def test_norm_site_is_ket_bra_symmetric(shape):
    rng = np.random.default_rng(len(shape))
    A = rng.standard_normal(shape)
    E = Q.double_layer(A)
    legs = shape[1:]
    r = len(legs)
    assert E.shape == tuple(n * n for n in legs)
    F = E.reshape([x for n in legs for x in (n, n)])
    swap = [x for i in range(r) for x in (2 * i + 1, 2 * i)]
    np.testing.assert_array_equal(F, F.transpose(swap))
    # the scalar site (rank 0) is the squared norm of its spin vector
    if r == 0:
        assert float(E) == pytest.approx(float(A @ A), rel=1e-15)

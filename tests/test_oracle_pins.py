"""Pins for the CPU oracle: brute force, closed forms, a textbook method and
invariants, none of which is the oracle checking itself."""
import math
import itertools

import numpy as np
import pytest

import lattice_inputs as li
from oracle import closed_forms as cf
from oracle import contract as C
from oracle import invariants as inv
from oracle import network as nw
from oracle import plan as P

ORDERS = [P.COLSWEEP, P.QUADRANT, P.HEURISTIC, P.ROWS, P.ROWS_T]


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("K", [0.1, 0.4, 0.9])
def test_spin_sum_plaquette_closed_form(K):
    assert rel(nw.brute_spins(2, 2, K), cf.ising_plaquette(K)) < 1e-14


@pytest.mark.parametrize("L", [1, 2, 5, 9])
def test_spin_sum_row_closed_form(L):
    assert rel(nw.brute_spins(1, L, 0.37), cf.ising_row(L, 0.37)) < 1e-13
    assert rel(nw.brute_spins(L, 1, 0.37), cf.ising_row(L, 0.37)) < 1e-13


def test_spin_sum_zero_coupling():
    assert nw.brute_spins(3, 4, 0.0) == 2.0 ** 12


@pytest.mark.parametrize("rows,cols", [(2, 3), (3, 3), (3, 4), (4, 4), (2, 6), (4, 3)])
def test_transfer_matrix_vs_spins(rows, cols):
    for K in (0.2, 0.44):
        a = nw.transfer_log_z(rows, cols, K)
        b = math.log(nw.brute_spins(rows, cols, K))
        assert abs(a - b) < 1e-13 * max(1, abs(b))


@pytest.mark.parametrize("rows,cols,K", [(2, 2, 0.3), (2, 3, 0.5), (3, 3, 0.4), (4, 4, 0.4)])
def test_ising_network_by_bonds_equals_spin_sum(rows, cols, K):
    # the network built from sqrt(W) summed literally over its bonds equals
    # the Boltzmann sum over spins: pins both the site construction and the
    # literal bond sum (4x4 = 2^24 bond assignments, configuration 1)
    z = nw.brute_bonds(li.ising(rows, cols, K), rows, cols)
    assert rel(z, nw.brute_spins(rows, cols, K)) < 1e-13


def test_brute_bonds_all_ones_and_product():
    for (r, c, D) in [(2, 2, 3), (3, 3, 2), (2, 4, 2), (1, 5, 3)]:
        z = nw.brute_bonds(li.ones(r, c, D), r, c)
        assert rel(z, math.exp(cf.all_ones_log(r, c, D))) < 1e-13
    rng = np.random.default_rng(3)
    r, c = 3, 3
    vecs = {}
    for rr in range(r):
        for cc in range(c):
            for b in nw.site_bonds(r, c, rr, cc):
                vecs[(rr, cc, b)] = rng.standard_normal(2)
    sites = cf.product_sites(r, c, vecs)
    assert rel(nw.brute_bonds(sites, r, c), cf.product_value(r, c, vecs)) < 1e-12


# ------------------------------------------------------ plan-based contraction

def _random_dims(rng, rows, cols, dmax):
    h = rng.integers(1, dmax + 1, size=(rows, max(cols - 1, 0)))
    v = rng.integers(1, dmax + 1, size=(max(rows - 1, 0), cols))
    return h, v


@pytest.mark.parametrize("rows,cols", [(1, 1), (1, 2), (2, 1), (1, 5), (5, 1), (2, 2),
                                       (2, 3), (3, 2), (3, 3), (2, 4), (4, 2), (3, 4)])
def test_contract_every_order_equals_brute_force(rows, cols):
    rng = np.random.default_rng(rows * 10 + cols)
    for trial in range(3):
        h, v = _random_dims(rng, rows, cols, 3)
        nb = int(np.prod(h)) * int(np.prod(v))
        if nb > (1 << 22):
            continue
        sites = li.normal(rows, cols, 0, seed=trial, hdim=h, vdim=v)
        ref = nw.brute_bonds(sites, rows, cols)
        for order in ORDERS:
            if order == P.QUADRANT and (rows < 2 or cols < 2):
                continue
            got = C.contract_grid(sites, rows, cols, order).value
            assert abs(got - ref) <= 1e-12 * max(abs(ref), 1e-300) + 1e-14 * \
                nw.brute_bonds([np.abs(s) for s in sites], rows, cols)


def test_every_quadrant_split_equals_brute_force():
    rows, cols = 3, 4
    sites = li.uniform(rows, cols, 2, seed=5)
    ref = nw.brute_bonds(sites, rows, cols)
    for h in range(1, rows):
        for w in range(1, cols):
            got = C.contract_grid(sites, rows, cols, P.QUADRANT, h, w).value
            assert rel(got, ref) < 1e-13


@pytest.mark.parametrize("rows,cols,D", [(5, 5, 2), (4, 6, 2), (3, 7, 3), (6, 4, 2)])
def test_contract_equals_library_einsum(rows, cols, D):
    sites = li.uniform(rows, cols, D, seed=11)
    ref = nw.einsum_value(sites, rows, cols)
    for order in ORDERS:
        assert rel(C.contract_grid(sites, rows, cols, order).value, ref) < 1e-12


@pytest.mark.parametrize("K", [0.2, 0.44, 0.6])
def test_ising_10x10_contract_equals_transfer_matrix(K):
    tm = nw.transfer_log_z(10, 10, K)
    for order in (P.COLSWEEP, P.QUADRANT):
        r = C.contract_grid(li.ising(10, 10, K), 10, 10, order)
        assert r.sign == 1 and abs(r.log_abs - tm) <= 1e-12


def test_ising_replica_is_square_of_z():
    tm = nw.transfer_log_z(6, 7, 0.44)
    r = C.contract_grid(li.ising_d4(6, 7, 0.44), 6, 7, P.HEURISTIC)
    assert abs(r.log_abs - 2 * tm) <= 1e-12


def test_all_ones_closed_form_large():
    # the paper's timing inputs; Z = D^(#bonds) is exact in the mantissa
    for (L, D) in [(8, 2), (6, 4), (5, 3)]:
        r = C.contract_grid(li.ones(L, L, D), L, L, P.HEURISTIC)
        assert abs(r.log_abs - cf.all_ones_log(L, L, D)) <= 1e-12
        if D in (2, 4):
            assert r.mantissa == 0.5


# ---------------------------------------------------------------- rescaling

def test_rescale_is_exact_in_the_mantissa():
    sites = li.uniform(4, 4, 3, seed=2)
    p = P.plan_grid(4, 4, 3)
    scaled = C.contract(sites, p)
    B = None
    for s in p.steps:   # the same steps without any rescale
        S = C.staged(sites[s.site[0] * 4 + s.site[1]], s)
        if s.kind == "INIT":
            B = S.reshape(-1)
        else:
            B = np.tensordot(B.reshape(s.pre, s.K, s.post), S, axes=([1], [0]))
            B = np.ascontiguousarray(B.transpose(0, 2, 1)).reshape(-1)
    f, e = math.frexp(float(B[0]))
    assert scaled.mantissa == f and scaled.exp2 == e


# ---------------------------------------------------------------- invariants

def _val(sites, rows, cols, order=P.COLSWEEP):
    return C.contract_grid(sites, rows, cols, order).value


def test_gauge_rotation_reflection_pad_scale_multilinearity():
    rows, cols, D = 4, 5, 3
    s = li.normal(rows, cols, D, seed=7)
    z = _val(s, rows, cols)
    rng = np.random.default_rng(0)
    g = inv.gauge(s, rows, cols, ("h", 1, 2), rng.standard_normal((D, D)) + 3 * np.eye(D))
    g = inv.gauge(g, rows, cols, ("v", 2, 0), rng.standard_normal((D, D)) + 3 * np.eye(D))
    assert rel(_val(g, rows, cols, P.QUADRANT), z) < 1e-10
    rs, nr, nc = inv.rotate90(s, rows, cols)
    assert rel(_val(rs, nr, nc), z) < 1e-12
    assert rel(_val(inv.reflect(s, rows, cols), rows, cols, P.QUADRANT), z) < 1e-12
    assert rel(_val(inv.pad(s, 5), rows, cols, P.HEURISTIC), z) < 1e-12
    z2 = _val(inv.scale_site(s, 7, 9), rows, cols)
    assert z2 == math.ldexp(z, 9)
    extra = li.normal(rows, cols, D, seed=8)[3]
    z3 = _val(inv.add_site(s, 3, extra), rows, cols)
    other = list(s)
    other[3] = extra
    assert rel(z3, z + _val(other, rows, cols)) < 1e-10


def test_replica_product():
    s1 = li.uniform(3, 4, 2, seed=1)
    s2 = li.uniform(3, 4, 3, seed=2)
    z = _val(inv.replica(s1, s2), 3, 4, P.QUADRANT)
    assert rel(z, _val(s1, 3, 4) * _val(s2, 3, 4)) < 1e-12


def test_input_replica_matches_oracle_replica():
    a = li.ising(3, 3, 0.3)
    for x, y in zip(li.replica(a, a), inv.replica(a, a)):
        assert np.array_equal(x, y)


# ---------------------------------------------------------------- plans

def _colsweep_flops(R, C_, D):
    col0 = sum(2 * D ** (r + 3) for r in range(1, R - 1)) + 2 * D ** (R + 1)
    mid = 4 * D ** (R + 2) + 2 * (R - 2) * D ** (R + 3)
    last = 2 * D ** (R + 1) + sum(2 * D ** (R - r + 2) for r in range(1, R - 1)) + 2 * D ** 2
    return col0 + (C_ - 2) * mid + last


@pytest.mark.parametrize("R,C_,D", [(r, c, d) for r in range(2, 9) for c in range(3, 9)
                                    for d in (1, 2, 3, 5)])
def test_colsweep_closed_forms(R, C_, D):
    p = P.plan_grid(R, C_, D, order=P.COLSWEEP)
    assert p.peak == D ** (R + 1) or (D == 1 and p.peak == 1)
    assert p.flops == _colsweep_flops(R, C_, D)
    assert len(p.steps) == R * C_
    assert p.slots == C_ - 1


@pytest.mark.parametrize("R,C_", [(r, c) for r in range(3, 11) for c in range(3, 11)])
def test_sweep_auto_closed_forms(R, C_):
    # §4: the sequential row scheme keeps a boundary of one bond per lattice
    # line it crosses, so sweeping along the longer side keeps the smaller
    # boundary; SWEEP_AUTO must pick that orientation (untransposed on ties).
    for D in (2, 3):
        p = P.plan_grid(R, C_, D, order=P.SWEEP_AUTO)
        short, long_ = min(R, C_), max(R, C_)
        assert p.order == P.COLSWEEP and p.requested == P.SWEEP_AUTO
        assert p.transpose == (1 if R > C_ else 0)
        assert p.peak == D ** (short + 1)
        assert p.flops == _colsweep_flops(short, long_, D)
        # the first line of sites absorbed runs along the shorter side:
        # down column 0 untransposed, along row 0 transposed
        first = [s.site for s in p.steps[:short]]
        if p.transpose:
            assert first == [(0, j) for j in range(short)]
        else:
            assert first == [(i, 0) for i in range(short)]
        assert p.slots == long_ - 1


def _rows_flops(R, C_, D):
    # edge rows: joining site j (1 <= j <= C-2) makes D^(j+1) down legs times
    # the right leg from D^j down legs, the right leg and the site's two new
    # legs; the last site closes the right leg.  Bulk rows carry up and down
    # legs alike.  Links: D^C x D^C products, the last one D^C x 1.
    edge = sum(2 * D ** (j + 3) for j in range(1, C_ - 1)) + 2 * D ** (C_ + 1)
    bulk = sum(2 * D ** (2 * j + 4) for j in range(1, C_ - 1)) + 2 * D ** (2 * C_ + 1)
    return 2 * edge + (R - 2) * bulk + (R - 2) * 2 * D ** (2 * C_) + 2 * D ** C_


@pytest.mark.parametrize("R,C_", [(r, c) for r in range(3, 9) for c in range(3, 8)])
def test_rows_closed_forms(R, C_):
    # §4, row scheme: contracting along the rows leaves a chain of row tensors
    # whose bulk members carry chi^L legs up and chi^L down
    for D in (2, 3):
        p = P.plan_grid(R, C_, D, order=P.ROWS)
        assert p.order == P.ROWS and p.transpose == 0
        assert len(p.units) == R and len(p.chain) == R - 1
        assert [u.result for u in p.units] == [D ** C_] + [D ** (2 * C_)] * (R - 2) + [D ** C_]
        assert p.peak == D ** (2 * C_)
        assert p.flops == _rows_flops(R, C_, D)
        assert p.buffers == 6 * D ** C_ + (R - 2) * 2 * D ** (2 * C_)
        assert [lk.N for lk in p.chain] == [D ** C_] * (R - 2) + [1]
        t = P.plan_grid(C_, R, D, order=P.ROWS_T)       # the same over columns
        assert (t.peak, t.flops, t.transpose) == (p.peak, p.flops, 1)


def test_heuristic_with_a_storage_budget():
    # §4 / §6: the order decides what fits.  Under a budget between the
    # sweep's and the quadrant's storage the heuristic falls back to the
    # sweep; below every candidate nothing fits.
    for L, D in [(6, 2), (8, 2), (10, 4), (12, 4)]:
        q = P.plan_grid(L, L, D, order=P.QUADRANT)
        sw = P.plan_grid(L, L, D, order=P.COLSWEEP)
        assert sw.buffers == 2 * D ** (L + 1) and sw.buffers < q.buffers
        assert P.plan_grid(L, L, D, order=P.HEURISTIC).order == P.QUADRANT
        got = P.plan_grid(L, L, D, order=P.HEURISTIC, budget=q.buffers - 1)
        assert got.order == P.COLSWEEP and got.buffers <= q.buffers - 1
        with pytest.raises(P.PlanTooLarge):
            P.plan_grid(L, L, D, order=P.HEURISTIC, budget=sw.buffers - 1)
        with pytest.raises(P.PlanTooLarge):
            P.plan_grid(L, L, D, order=P.QUADRANT, budget=q.buffers - 1)
    # the row scheme is the first to run out (§6): at 10 x 10, D = 4 its bulk
    # row tensors hold 4^20 entries each
    with pytest.raises(P.PlanTooLarge):
        P.plan_grid(10, 10, 4, order=P.ROWS, budget=1 << 31)


def test_paper_row_and_quadrant_bond_sizes():
    # §4: sweeping whole rows/columns leaves boundary legs of total size
    # chi^L (the chain); quadrants meet in a ring whose bonds carry chi^(L/2)
    for L in (4, 6, 8, 12):
        for D in (2, 4):
            sw = P.plan_grid(L, L, D, order=P.COLSWEEP)
            # the boundary between columns holds exactly L bonds
            col_ends = [s.out for s in sw.steps if s.rescale >= 0]
            assert all(o == D ** L for o in col_ends)
            q = P.plan_grid(L, L, D, order=P.QUADRANT)
            g = q.ring
            assert g.m == g.n == g.kx == g.ky == D ** (L // 2)
            assert q.peak == D ** L


def test_heuristic_choices():
    for L in (4, 6, 10, 12):
        assert P.plan_grid(L, L, 4, order=P.HEURISTIC).order == P.QUADRANT
    for L in (5, 7, 11, 13):
        # odd L: no split beats the sweep's bottleneck D^(L+1); flops break the tie
        p = P.plan_grid(L, L, 4, order=P.HEURISTIC)
        sw = P.plan_grid(L, L, 4, order=P.COLSWEEP)
        assert p.peak == sw.peak == 4 ** (L + 1) and p.flops <= sw.flops
    assert P.plan_grid(13, 13, 4, order=P.HEURISTIC).order == P.COLSWEEP
    assert P.plan_grid(5, 5, 4, order=P.HEURISTIC).quad == (2, 2)
    p = P.plan_grid(3, 8, 2, order=P.HEURISTIC)   # wide: boundary follows the short side
    assert p.order == P.COLSWEEP and p.transpose == 0 and p.peak == 2 ** 4
    p = P.plan_grid(8, 3, 2, order=P.HEURISTIC)
    assert p.order == P.COLSWEEP and p.transpose == 1 and p.peak == 2 ** 4


def test_plan_overflow_is_reported():
    with pytest.raises(P.PlanOverflow):
        P.plan_grid(40, 40, 64, order=P.COLSWEEP)


# ------------------------------------------- planted mistakes must be caught

def test_pins_catch_a_transposed_site_fold(monkeypatch):
    sites = li.uniform(3, 3, 2, seed=4)
    ref = nw.brute_bonds(sites, 3, 3)
    real = C.staged

    def wrong(site, step):   # contract the two K legs in swapped order
        if step.K > 2 and len(step.perm) >= 2:
            p = list(step.perm)
            p[0], p[1] = p[1], p[0]
            step = P.Step(**{**step.__dict__, "perm": tuple(p)})
        return real(site, step)
    monkeypatch.setattr(C, "staged", wrong)
    assert rel(C.contract_grid(sites, 3, 3).value, ref) > 1e-6


def test_pins_catch_a_dropped_rescale_exponent(monkeypatch):
    sites = li.uniform(4, 4, 2, seed=4)
    ref = nw.brute_bonds(sites, 4, 4)
    real = C._rescale
    monkeypatch.setattr(C, "_rescale", lambda B: (real(B)[0], 0))
    assert rel(C.contract_grid(sites, 4, 4).value, ref) > 1e-6


def test_pins_catch_a_wrong_ring_pairing(monkeypatch):
    sites = li.uniform(4, 4, 2, seed=4)
    ref = nw.brute_bonds(sites, 4, 4)
    p = P.plan_grid(4, 4, 2, order=P.QUADRANT)
    p.ring.ya, p.ring.yb = p.ring.yb, p.ring.ya    # pair BL with TR instead
    assert rel(C.contract(sites, p).value, ref) > 1e-6


def test_pins_catch_a_perturbed_site():
    s = li.ising(3, 3, 0.5)
    ref = nw.brute_spins(3, 3, 0.5)
    # perturbing a single entry of one site changes the value
    bad2 = [t.copy() for t in s]
    bad2[4].flat[3] *= 1.01
    assert rel(nw.brute_bonds(bad2, 3, 3), ref) > 1e-6


def test_pins_catch_a_wrong_chain_side(monkeypatch):
    sites = li.uniform(4, 3, 2, seed=5)
    ref = nw.brute_bonds(sites, 4, 3)
    p = P.plan_grid(4, 3, 2, order=P.ROWS)
    p.chain[0].side = 1 - p.chain[0].side     # read the row tensor transposed
    assert rel(C.contract(sites, p).value, ref) > 1e-6

"""Chained small steps (paper §4: the pairwise sequential contraction fixes
the value, not the launch structure).  Runs of consecutive small single
steps of a unit (the edge columns, every step of a D = 2 lattice) run as one
launch with one workgroup per unit, with the same per-step arithmetic as one
launch per step: the results must be bitwise identical with chains on and
off, and chains must actually replace launches."""
import pytest

import lattice_inputs as li
from oracle import contract as C
from oracle import plan as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tn():
    import torch
    assert torch.cuda.is_available()
    import paper_1908_08553_amd as tn
    tn.tn_set_option(tn.TN_OPT_KERNEL_IMPL, 0)
    tn.tn_set_option(tn.TN_OPT_FUSE_STEPS, 2)
    yield tn
    tn.tn_set_option(tn.TN_OPT_CHAIN_STEPS, 1)


def run(tn, sites, rows, cols, D, order, prec, chain):
    tn.tn_set_option(tn.TN_OPT_CHAIN_STEPS, chain)
    plan = tn.tn_plan_grid(rows, cols, D, order=order)
    print(f"[gpu] chain={chain} {rows}x{cols} D={D} order={order} {prec}", flush=True)
    tn.tn_profile_enable(True)
    try:
        res = tn.contract_grid(plan, tn.device_sites(sites), prec)
        stats = {k["name"]: k["launches"] for k in tn.tn_profile_read()}
    finally:
        tn.tn_profile_enable(False)
        tn.tn_set_option(tn.TN_OPT_CHAIN_STEPS, 1)
    return res, stats


CASES = [
    (10, 10, 4, "normal", P.COLSWEEP, "f64"),
    (12, 12, 2, "ising", P.COLSWEEP, "f32"),
    (12, 12, 2, "ising", P.COLSWEEP, "bf16x3"),
    (6, 6, 4, "uniform", P.QUADRANT, "f32"),
    (10, 10, 4, "uniform", P.QUADRANT, "f64"),
    (5, 7, 3, "uniform", P.HEURISTIC, "bf16x3"),
    (7, 5, 3, "normal", P.COLSWEEP, "f64"),
    (1, 9, 2, "uniform", P.COLSWEEP, "f64"),
    (4, 4, 2, "uniform", P.COLSWEEP, "f32"),
]


@pytest.mark.parametrize("rows,cols,D,kind,order,prec", CASES)
def test_chains_bitwise_equal_to_single_launches(tn, rows, cols, D, kind, order, prec):
    sites = li.make(kind, rows, cols, D, seed=rows * cols + D, K=0.44)
    on, s_on = run(tn, sites, rows, cols, D, order, prec, 1)
    off, s_off = run(tn, sites, rows, cols, D, order, prec, 0)
    assert (on.status, on.sign, on.exp2_sum) == (off.status, off.sign, off.exp2_sum)
    assert on.mantissa == off.mantissa and on.log_abs == off.log_abs
    chained = sum(v for k, v in s_on.items() if k.startswith("absorb_chain_"))
    assert chained > 0, s_on
    assert not any(k.startswith("absorb_chain_") for k in s_off), s_off
    assert sum(s_on.values()) < sum(s_off.values())


def test_chained_d2_ising_matches_oracle(tn):
    rows, cols = 12, 12
    sites = li.make("ising", rows, cols, 2, K=0.44)
    ref = C.contract_grid(sites, rows, cols, P.COLSWEEP)
    got, stats = run(tn, sites, rows, cols, 2, P.COLSWEEP, "f64", 1)
    assert stats.get("absorb_chain_f64", 0) >= 10
    assert got.sign == ref.sign
    assert abs(got.log_abs - ref.log_abs) <= 1e-12

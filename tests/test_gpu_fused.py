"""Fused absorption of two consecutive bulk steps (one pass over the boundary
for rows i and i+1 of a column, D = 4 legs between them).

The fused kernel performs the same products in the same order as the two
single-step launches and keeps the intermediate in the boundary's own element
type, so the results must be bitwise identical to TN_OPT_FUSE_STEPS = 0; the
oracle then pins both (paper §4: the pairwise sequential contraction fixes the
value, not the launch structure)."""
import numpy as np
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
    tn.tn_set_option(tn.TN_OPT_FUSE_STEPS, 1)
    yield tn
    tn.tn_set_option(tn.TN_OPT_FUSE_STEPS, 1)


def run(tn, sites, rows, cols, order, prec, fuse, hdim=None, vdim=None, qh=0, qw=0):
    tn.tn_set_option(tn.TN_OPT_FUSE_STEPS, fuse)
    D = 1 if hdim is not None else int(sites[0].shape[0])
    plan = tn.tn_plan_grid(rows, cols, D, hdim, vdim, order, qh, qw)
    print(f"[gpu] fused={fuse} {rows}x{cols} order={order} prec={prec}", flush=True)
    tn.tn_profile_enable(True)
    try:
        res = tn.contract_grid(plan, tn.device_sites(sites), prec)
        names = {k["name"]: k["launches"] for k in tn.tn_profile_read()}
    finally:
        tn.tn_profile_enable(False)
        tn.tn_set_option(tn.TN_OPT_FUSE_STEPS, 1)
    return res, names


def pair_launches(names):
    return sum(v for k, v in names.items() if k.startswith("absorb_pair_"))


def same_bits(a, b):
    assert (a.status, a.sign, a.exp2_sum) == (b.status, b.sign, b.exp2_sum)
    assert a.mantissa == b.mantissa and a.log_abs == b.log_abs, (a, b)


@pytest.fixture(scope="module")
def uniform12():
    return li.uniform(12, 12, 4, 0)


@pytest.mark.parametrize("order", [P.COLSWEEP, P.HEURISTIC])
@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f64"])
def test_fused_equals_unfused_12x12_d4(tn, uniform12, order, prec):
    fused, nf = run(tn, uniform12, 12, 12, order, prec, 1)
    plain, npl = run(tn, uniform12, 12, 12, order, prec, 0)
    assert pair_launches(nf) > 0, nf
    assert pair_launches(npl) == 0, npl
    same_bits(fused, plain)


def test_fused_sweep_last_column_not_fused(tn, uniform12):
    # the float32 sweep's last column (float64, no right legs: N = D = 4) has
    # no fusable pair; its middle columns fuse rows (1,2) (3,4) (5,6) (7,8)
    _, names = run(tn, uniform12, 12, 12, P.COLSWEEP, "f32", 1)
    assert names.get("absorb_pair_f64", 0) == 0, names
    assert names.get("absorb_pair_f32", 0) == 10 * 4, names


@pytest.fixture(scope="module")
def mixed10():
    # bond dimensions drawn from {2, 4, 8}: only pairs whose three shared
    # inner legs are 4 fuse; the rest run one step at a time
    rows, cols = 10, 10
    rng = np.random.default_rng(5)
    h = rng.choice([2, 4, 4, 4, 4], size=(rows, cols - 1))
    v = rng.choice([2, 4, 4, 4, 4, 8], size=(rows - 1, cols))
    s = li.uniform(rows, cols, 0, 33, hdim=h, vdim=v)
    return s, h, v, C.contract_grid(s, rows, cols, P.QUADRANT, 0, 0)


@pytest.mark.parametrize("order", [P.COLSWEEP, P.QUADRANT])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fused_mixed_bond_dims_vs_oracle(tn, mixed10, order, prec):
    s, h, v, ref = mixed10
    fused, nf = run(tn, s, 10, 10, order, prec, 1, hdim=h, vdim=v)
    plain, _ = run(tn, s, 10, 10, order, prec, 0, hdim=h, vdim=v)
    assert pair_launches(nf) > 0, nf
    same_bits(fused, plain)
    assert fused.sign == ref.sign == 1
    tol = 1e-12 if prec == "f64" else 1e-5 * abs(ref.log_abs)
    assert abs(fused.log_abs - ref.log_abs) <= tol, (fused.log_abs, ref.log_abs)


def test_fused_ising_d4_13x13_f64(tn):
    # 13x13 two-replica Ising: its value is Z^2 of the transfer-matrix value
    import os
    gold = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "ising_logz.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                r, c, K, val = line.split()
                gold[(int(r), int(c), float(K))] = float(val)
    tm = 2 * gold[(13, 13, 0.44)]
    got, names = run(tn, li.ising_d4(13, 13, 0.44), 13, 13, P.COLSWEEP, "f64", 1)
    assert pair_launches(names) > 0
    assert got.sign == 1 and abs(got.log_abs - tm) <= 1e-12 * tm

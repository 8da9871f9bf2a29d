"""Fused absorption: several consecutive rows of one column in one pass over
the boundary (paper §4: the pairwise sequential contraction fixes the value,
not the launch structure).

* Pairs (TN_OPT_FUSE_STEPS = 1): the same products in the same order as two
  single-step launches, the intermediate kept in the boundary's element type,
  so the results are bitwise identical to TN_OPT_FUSE_STEPS = 0.
* Column chunks (TN_OPT_FUSE_STEPS = 2, the default): up to 4 rows (3 in
  FP64) on a slice held on chip, products in a different order; checked
  against the FP64 oracle at the stated tolerances and against the
  transfer-matrix value of the Ising network.  Two chunk kernels: the slice
  in one wavefront's registers (TN_OPT_CHUNK_SCHEDULE 0, the default, where
  the suffix is 1 or a multiple of 16; 2 = at most 3 rows) and the slice in
  LDS (schedule 1, and the fallback for other suffixes)."""
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
    yield tn
    tn.tn_set_option(tn.TN_OPT_FUSE_STEPS, 2)


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
        tn.tn_set_option(tn.TN_OPT_FUSE_STEPS, 2)
    return res, names


def pair_launches(names):
    return sum(v for k, v in names.items() if k.startswith("absorb_pair_"))


def chunk_launches(names):
    return sum(v for k, v in names.items() if k.startswith("absorb_chunk_"))


def reg_launches(names):
    return sum(v for k, v in names.items() if k.startswith("absorb_chunk_reg_"))


def lds_launches(names):
    return chunk_launches(names) - reg_launches(names)


def run_sched(tn, sched, *args, **kw):
    tn.tn_set_option(tn.TN_OPT_CHUNK_SCHEDULE, sched)
    try:
        return run(tn, *args, **kw)
    finally:
        tn.tn_set_option(tn.TN_OPT_CHUNK_SCHEDULE, 0)


def close(got, ref, prec):
    assert got.status == 0 and got.sign == ref.sign == 1
    tol = 1e-12 if prec == "f64" else 1e-5 * max(1.0, abs(ref.log_abs))
    assert abs(got.log_abs - ref.log_abs) <= tol, (prec, got.log_abs, ref.log_abs)


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
    chunked, nc = run(tn, s, 10, 10, order, prec, 2, hdim=h, vdim=v)
    assert pair_launches(nf) > 0, nf
    assert chunk_launches(nc) > 0, nc
    same_bits(fused, plain)
    close(fused, ref, prec)
    close(chunked, ref, prec)


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
    sites = li.ising_d4(13, 13, 0.44)
    for fuse, count in ((1, pair_launches), (2, chunk_launches)):
        got, names = run(tn, sites, 13, 13, P.COLSWEEP, "f64", fuse)
        assert count(names) > 0, names
        assert got.sign == 1 and abs(got.log_abs - tm) <= 1e-12, (fuse, got.log_abs, tm)


@pytest.fixture(scope="module")
def oracle12(uniform12):
    return C.contract_grid(uniform12, 12, 12, P.QUADRANT, 0, 0)


@pytest.mark.parametrize("order", [P.COLSWEEP, P.HEURISTIC])
@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f64"])
def test_chunks_12x12_d4_vs_oracle(tn, uniform12, oracle12, order, prec):
    got, names = run(tn, uniform12, 12, 12, order, prec, 2)
    print(f"  chunks {prec} order={order}: {got.log_abs!r} oracle {oracle12.log_abs!r}")
    assert chunk_launches(names) > 0, names
    close(got, oracle12, prec)


@pytest.mark.parametrize("prec,per_column", [("f32", 3), ("bf16x3", 3), ("f64", 4)])
def test_chunk_partition_of_the_sweep(tn, uniform12, prec, per_column):
    # 12 rows: chunks of 4 rows (rows 0-3 with the top edge's K = 4, 4-7, 8-11
    # with the bottom edge's N = 4), of 3 rows in FP64; the middle columns
    # 1..10 only (column 0 has no suffix to shrink, the last column no right legs)
    _, names = run(tn, uniform12, 12, 12, P.COLSWEEP, prec, 2)
    assert chunk_launches(names) == 10 * per_column, names


def test_chunk_quadrant_launches_are_grouped(tn, uniform12):
    # 6x6 quadrants: columns 1..5 of each unit as two chunks of 3 rows (the
    # fewest passes a 4-row chunk allows, lengths as equal as possible), the
    # four units' work in one launch each
    _, names = run(tn, uniform12, 12, 12, P.QUADRANT, "f32", 2)
    assert chunk_launches(names) == 5 * 2, names
    assert pair_launches(names) == 0, names


@pytest.mark.parametrize("rows,cols", [(6, 12), (12, 6), (9, 7), (5, 13)])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_chunks_thin_and_odd_lattices(tn, rows, cols, prec):
    s = li.uniform(rows, cols, 4, 100 + rows * cols)
    ref = C.contract_grid(s, rows, cols, P.QUADRANT, 0, 0)
    for order in (P.COLSWEEP, P.HEURISTIC):
        got, _ = run(tn, s, rows, cols, order, prec, 2)
        close(got, ref, prec)


@pytest.mark.parametrize("sched", [1, 2])
@pytest.mark.parametrize("order", [P.COLSWEEP, P.HEURISTIC])
@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f64"])
def test_chunk_schedules_12x12_d4_vs_oracle(tn, uniform12, oracle12, sched, order, prec):
    got, names = run_sched(tn, sched, uniform12, 12, 12, order, prec, 2)
    print(f"  sched {sched} {prec} order={order}: {got.log_abs!r} oracle {oracle12.log_abs!r}")
    if sched == 1:
        assert reg_launches(names) == 0 and lds_launches(names) > 0, names
    else:
        assert reg_launches(names) > 0, names
        if order == P.COLSWEEP:   # suffixes 4^9, 4^6, 4^3 and 1: all register shapes
            assert lds_launches(names) == 0, names
    close(got, oracle12, prec)


def edge_launches(names):
    return {k: v for k, v in names.items() if k.startswith("absorb_edge_")}


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f64"])
def test_edge_pairs_12x12_d4(tn, uniform12, oracle12, prec):
    # the first column's rows 10-11 (suffix 1) and the last column's rows 0-1
    # (prefix 1) run as fused pairs; the last column is FP64 in every
    # precision, the first column's pair has no BF16x3 form
    got, names = run(tn, uniform12, 12, 12, P.COLSWEEP, prec, 2)
    want = {"f64": {"absorb_edge_f64": 2},
            "f32": {"absorb_edge_f32": 1, "absorb_edge_f64": 1},
            "bf16x3": {"absorb_edge_f64": 1}}[prec]
    assert edge_launches(names) == want, names
    close(got, oracle12, prec)
    plain, pn = run(tn, uniform12, 12, 12, P.COLSWEEP, prec, 0)
    assert not edge_launches(pn), pn
    tol = 1e-12 if prec == "f64" else 1e-5 * abs(plain.log_abs)
    assert got.sign == plain.sign and abs(got.log_abs - plain.log_abs) <= tol


@pytest.mark.parametrize("rows,cols", [(13, 5), (10, 3), (11, 11)])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_edge_pairs_ragged_and_signed(tn, rows, cols, prec):
    # N(0,1) sites (signs, cancellation) on odd sizes: both pairs fuse, and
    # the rescale slot the bottom pair measures feeds the next column
    s = li.normal(rows, cols, 4, 300 + rows * cols)
    ref = C.contract_grid(s, rows, cols, P.QUADRANT, 0, 0)
    got, names = run(tn, s, rows, cols, P.COLSWEEP, prec, 2)
    assert sum(edge_launches(names).values()) == 2, names
    assert got.status == 0 and got.sign == ref.sign
    tol = 1e-12 if prec == "f64" else 1e-5 * max(1.0, abs(ref.log_abs))
    assert abs(got.log_abs - ref.log_abs) <= tol, (got.log_abs, ref.log_abs)


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f64"])
def test_register_chunks_take_the_sweep(tn, uniform12, prec):
    # 12 rows: every chunk of the middle columns has suffix 4^8, 4^4 (or 4^9,
    # 4^6, 4^3 in FP64) or 1 at the bottom edge, all register-kernel shapes
    _, names = run(tn, uniform12, 12, 12, P.COLSWEEP, prec, 2)
    assert reg_launches(names) == chunk_launches(names) > 0, names


def test_register_and_lds_chunks_in_one_contraction(tn, uniform12, oracle12):
    # 12x12 quadrant order in FP32: the 3-row chunks of the quadrant columns
    # in registers, the first chunked column's short suffix on the LDS kernel
    got, names = run(tn, uniform12, 12, 12, P.QUADRANT, "f32", 2)
    assert reg_launches(names) > 0 and lds_launches(names) > 0, names
    close(got, oracle12, "f32")


@pytest.mark.parametrize("sched", [0, 1, 2])
def test_chunk_schedules_mixed_dims_and_ising(tn, mixed10, sched):
    s, h, v, ref = mixed10
    for order in (P.COLSWEEP, P.QUADRANT):
        for prec in ("f64", "f32", "bf16x3"):
            got, names = run_sched(tn, sched, s, 10, 10, order, prec, 2, hdim=h, vdim=v)
            assert chunk_launches(names) > 0, names
            close(got, ref, prec)
    import os
    gold = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "ising_logz.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                r, c, K, val = line.split()
                gold[(int(r), int(c), float(K))] = float(val)
    tm = 2 * gold[(13, 13, 0.44)]
    got, _ = run_sched(tn, sched, li.ising_d4(13, 13, 0.44), 13, 13, P.COLSWEEP, "f64", 2)
    assert got.sign == 1 and abs(got.log_abs - tm) <= 1e-12, (sched, got.log_abs, tm)


@pytest.mark.parametrize("rows,cols", [(6, 12), (12, 6), (9, 7), (5, 13), (13, 4)])
@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f64"])
def test_chunk_schedule_2_thin_and_odd_lattices(tn, rows, cols, prec):
    s = li.uniform(rows, cols, 4, 200 + rows * cols)
    ref = C.contract_grid(s, rows, cols, P.QUADRANT, 0, 0)
    for order in (P.COLSWEEP, P.HEURISTIC):
        got, _ = run_sched(tn, 2, s, rows, cols, order, prec, 2)
        close(got, ref, prec)

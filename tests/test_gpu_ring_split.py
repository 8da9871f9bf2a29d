"""Split-K ring products (paper §4, Fig. 2b: the four quadrant tensors closed
as a ring).

When the ring's output has too few 128 x 128 tiles to give every CU two
workgroups, both ring products cut their k extent into S ranges: the stored
product X leaves S slices whose sum the fused-dot product reads, and the fused
dot writes one partial sum per range.  Checked against the FP64 oracle at the
stated tolerances, against the unsplit vector-ALU ring in FP64, and for
run-to-run bitwise repeatability (the summation order is fixed)."""
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
    tn.tn_set_option(tn.TN_OPT_KERNEL_IMPL, 0)


def run(tn, sites, rows, cols, prec, impl=0):
    tn.tn_set_option(tn.TN_OPT_KERNEL_IMPL, impl)
    plan = tn.tn_plan_grid(rows, cols, int(sites[0].shape[0]), None, None, P.QUADRANT, 0, 0)
    print(f"[gpu] ring split {rows}x{cols} prec={prec} impl={impl}", flush=True)
    tn.tn_profile_enable(True)
    try:
        res = tn.contract_grid(plan, tn.device_sites(sites), prec)
        stats = {k["name"]: k for k in tn.tn_profile_read()}
    finally:
        tn.tn_profile_enable(False)
        tn.tn_set_option(tn.TN_OPT_KERNEL_IMPL, 0)
    return res, stats, plan.info()


def close(got, ref, prec):
    assert got.status == 0 and got.sign == ref.sign
    tol = 1e-12 if prec == "f64" else 1e-5 * max(1.0, abs(ref.log_abs))
    assert abs(got.log_abs - ref.log_abs) <= tol, (prec, got.log_abs, ref.log_abs)


RING = {"f64": "ring_mfma_f64", "f32": "ring_mfma_f32", "bf16x3": "ring_mfma_bf16x3"}
PREC = {"f64": 0, "f32": 1, "bf16x3": 2}


@pytest.mark.parametrize("rows,cols,slices", [(10, 10, 8), (9, 7, 8), (8, 8, 2), (7, 9, 2)])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_split_ring_vs_oracle(tn, rows, cols, slices, prec):
    s = li.uniform(rows, cols, 4, 7)
    ref = C.contract_grid(s, rows, cols, P.QUADRANT, 0, 0)
    got, stats, info = run(tn, s, rows, cols, prec)
    assert info["ring_slices"][PREC[prec]] == slices
    assert stats[RING[prec]]["launches"] == 2, stats
    print(f"  {prec}: {got.log_abs!r} oracle {ref.log_abs!r}")
    close(got, ref, prec)


@pytest.mark.parametrize("rows,cols", [(10, 10), (9, 7)])
def test_split_ring_vs_unsplit_valu_f64(tn, rows, cols):
    s = li.normal(rows, cols, 4, 3)
    split, st, _ = run(tn, s, rows, cols, "f64", impl=0)
    plain, sv, _ = run(tn, s, rows, cols, "f64", impl=1)
    assert "ring_mfma_f64" in st and "ring_valu_f64" in sv
    assert split.status == plain.status == 0 and split.sign == plain.sign
    assert abs(split.log_abs - plain.log_abs) <= 1e-12, (split.log_abs, plain.log_abs)


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f64"])
def test_split_ring_repeatable(tn, prec):
    s = li.uniform(10, 10, 4, 11)
    a, _, _ = run(tn, s, 10, 10, prec)
    b, _, _ = run(tn, s, 10, 10, prec)
    assert (a.mantissa, a.exp2_sum, a.sign) == (b.mantissa, b.exp2_sum, b.sign)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_split_ring_with_ragged_tiles(tn, prec):
    # 10x10, quadrant 5,5, mixed bond dimensions: the ring output is m = 4*4*3*4*1 = 192
    # (one full and one half 128-row tile) by n = 4*4*3*4*4 = 768, over k = 4^5 = 1024:
    # 12 tiles, so both products run in 8 k ranges with ragged edge tiles
    import numpy as np
    rows, cols = 10, 10
    h = np.full((rows, cols - 1), 4)
    v = np.tile(np.array([4, 4, 3, 4, 1, 4, 4, 3, 4, 4]), (rows - 1, 1))
    s = li.uniform(rows, cols, 0, 5, hdim=h, vdim=v)
    ref = C.contract_grid(s, rows, cols, P.QUADRANT, 5, 5)
    plan = tn.tn_plan_grid(rows, cols, 1, h, v, P.QUADRANT, 5, 5)
    assert plan.info()["ring_slices"][PREC[prec]] == 8
    print(f"[gpu] ring split ragged 10x10 prec={prec}", flush=True)
    tn.tn_set_option(tn.TN_OPT_KERNEL_IMPL, 0)
    got = tn.contract_grid(plan, tn.device_sites(s), prec)
    close(got, ref, prec)


@pytest.mark.parametrize("rows,cols,kind", [(12, 12, "uniform"), (10, 10, "normal"),
                                            (9, 7, "normal")])
def test_ring_operand_scaling_paths_agree(tn, rows, cols, kind):
    # The FP64 ring products apply 2^-(ea+eb) to their results, or to every
    # staged operand (TN_OPT_RING_OPERAND_SCALE = 1: the path they take by
    # themselves for exponent sums beyond +-512, which normalised inputs never
    # reach).  Power-of-two scaling is exact: the same bits either way, split
    # (10x10, 9x7) and unsplit (12x12) products alike.
    s = li.make(kind, rows, cols, 4, 31 + rows)
    ref = C.contract_grid(s, rows, cols, P.QUADRANT, 0, 0)
    a, sa, _ = run(tn, s, rows, cols, "f64")
    tn.tn_set_option(tn.TN_OPT_RING_OPERAND_SCALE, 1)
    try:
        b, sb, _ = run(tn, s, rows, cols, "f64")
    finally:
        tn.tn_set_option(tn.TN_OPT_RING_OPERAND_SCALE, 0)
    assert sa["ring_mfma_f64"]["launches"] == sb["ring_mfma_f64"]["launches"] == 2
    assert (a.status, a.sign, a.mantissa, a.exp2_sum) == (b.status, b.sign, b.mantissa, b.exp2_sum)
    close(a, ref, "f64")

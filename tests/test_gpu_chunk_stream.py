"""Streamed bottom chunks (TN_OPT_CHUNK_STREAM): the register chunks that end
a column with the most rows (4 in FP32 and split BF16x3, 3 in FP64) run with
each wavefront taking several tiles, the next tile's slice filled into LDS while the current
tile's register-only steps run.  The products and their order are those of
one tile per wavefront, so the results are bitwise identical to
TN_OPT_CHUNK_STREAM = 0; they are also checked against the FP64 oracle (paper
§4: the pairwise, sequential contraction fixes the value, not the schedule).
Small workgroup caps make each wavefront take many tiles and end on a
ragged share.  (Quadrant units never end a column with suffix 1, so grouped
launches keep the one-tile form.)"""
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
    tn.tn_set_option(tn.TN_OPT_FUSE_STEPS, 2)
    yield tn
    tn.tn_set_option(tn.TN_OPT_CHUNK_STREAM, 1)


def run(tn, plan, sites, prec, stream):
    tn.tn_set_option(tn.TN_OPT_CHUNK_STREAM, stream)
    print(f"[gpu] chunk stream={stream} prec={prec}", flush=True)
    tn.tn_profile_enable(True)
    try:
        res = tn.contract_grid(plan, sites, prec)
        names = {k["name"]: k["launches"] for k in tn.tn_profile_read()}
    finally:
        tn.tn_profile_enable(False)
        tn.tn_set_option(tn.TN_OPT_CHUNK_STREAM, 1)
    return res, names


def streamed(names):
    return sum(v for k, v in names.items() if k.startswith("absorb_chunk_reg_stream_"))


def close(got, want, prec):
    assert got.status == 0 and got.sign == want.sign
    tol = 1e-12 if prec == "f64" else 1e-5 * max(1.0, abs(want.log_abs))
    assert abs(got.log_abs - want.log_abs) <= tol, (prec, got, want)


# (rows, cols, order, qh, qw, caps): 12-row columns end in 4096-tile bottom
# chunks, 8-row columns in 16-tile ones (FP64: 3-row chunks, 9- and 6-row
# columns end in them)
CASES = [
    (12, 12, P.COLSWEEP, 0, 0, (1, 1000, 7)),
    (8, 9, P.COLSWEEP, 0, 0, (1, 3)),
    (12, 5, P.COLSWEEP, 0, 0, (1, 13)),
    (9, 7, P.COLSWEEP, 0, 0, (1, 5)),
]


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f64"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}o{c[2]}")
def test_streamed_bottoms_bitwise_equal_one_tile_form(tn, case, prec):
    rows, cols, order, qh, qw, caps = case
    s = li.uniform(rows, cols, 4, 7 * rows + cols)
    plan = tn.tn_plan_grid(rows, cols, 4, order=order, quad_h=qh, quad_w=qw)
    sites = tn.device_sites(s)
    base, names0 = run(tn, plan, sites, prec, 0)
    assert streamed(names0) == 0, names0
    # the oracle's value in its quickest order (the value does not depend on it)
    close(base, C.contract_grid(s, rows, cols, P.HEURISTIC, 0, 0), prec)
    # columns split into chunks of the longest length end in a streamed one
    expect = rows % (3 if prec == "f64" else 4) == 0
    for cap in caps:
        got, names = run(tn, plan, sites, prec, cap)
        assert (streamed(names) > 0) == expect, (cap, names)
        assert (got.sign, got.mantissa, got.exp2_sum) == (base.sign, base.mantissa, base.exp2_sum), cap


def test_streamed_bottoms_signed_entries(tn):
    # N(0, 1) entries: signs and cancellations through the same tiles
    s = li.normal(12, 8, 4, 77)
    plan = tn.tn_plan_grid(12, 8, 4, order=P.COLSWEEP)
    sites = tn.device_sites(s)
    base, _ = run(tn, plan, sites, "f32", 0)
    for cap in (1, 9):
        got, names = run(tn, plan, sites, "f32", cap)
        assert streamed(names) > 0
        assert (got.sign, got.mantissa, got.exp2_sum) == (base.sign, base.mantissa, base.exp2_sum)
    want = C.contract_grid(s, 12, 8, P.QUADRANT, 0, 0)
    assert base.sign == want.sign
    assert abs(base.log_abs - want.log_abs) <= 1e-5 * max(1.0, abs(want.log_abs))


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f64"])
def test_streamed_bottoms_flag_nonfinite(tn, prec):
    # a NaN in a site of the bottom row of an inner column (absorbed by the
    # streamed bottom chunk): the contraction reports TN_ENONFINITE with the
    # streamed and the one-tile forms alike
    rows, cols = 12, 5
    s = li.uniform(rows, cols, 4, 5)
    s[(rows - 1) * cols + 2] = s[(rows - 1) * cols + 2].copy()
    s[(rows - 1) * cols + 2].flat[7] = np.nan
    plan = tn.tn_plan_grid(rows, cols, 4, order=P.COLSWEEP)
    sites = tn.device_sites(s)
    for cap in (0, 1, 3):
        got, _ = run(tn, plan, sites, prec, cap)
        assert got.status == tn.TN_ENONFINITE, (prec, cap, got)

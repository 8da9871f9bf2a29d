"""The C++ planner behind the C ABI emits byte-identical canonical plan text
to the oracle's independent planner, and its statistics match the plan."""
import numpy as np
import pytest

import paper_1908_08553_amd as tn
from oracle import plan as P

ORDERS = [P.COLSWEEP, P.QUADRANT, P.HEURISTIC, P.SWEEP_AUTO, P.ROWS, P.ROWS_T]


def both(rows, cols, D=2, hdim=None, vdim=None, order=P.COLSWEEP, qh=0, qw=0):
    ref = P.plan_text(P.plan_grid(rows, cols, D, hdim, vdim, order, qh, qw))
    got = tn.tn_plan_text(tn.tn_plan_grid(rows, cols, D, hdim, vdim, order, qh, qw))
    return got, ref


@pytest.mark.parametrize("rows", range(1, 17))
@pytest.mark.parametrize("cols", [1, 2, 3, 5, 8, 12, 16])
def test_uniform_plans_bit_exact(rows, cols):
    for D in (1, 2, 3, 4, 5):
        for order in ORDERS:
            if order == P.QUADRANT and (rows < 2 or cols < 2):
                continue
            if order == P.HEURISTIC and rows * cols > 100 and D > 2:
                continue
            if order in (P.ROWS, P.ROWS_T):
                try:
                    P.plan_grid(rows, cols, D, order=order)
                except P.PlanOverflow:
                    with pytest.raises(tn.TnError) as e:
                        tn.tn_plan_grid(rows, cols, D, order=order)
                    assert e.value.status == tn.TN_EOVERFLOW
                    continue
            got, ref = both(rows, cols, D, order=order)
            assert got == ref


def test_nonuniform_plans_bit_exact():
    rng = np.random.default_rng(0)
    for _ in range(60):
        rows, cols = (int(x) for x in rng.integers(1, 7, size=2))
        h = rng.integers(1, 5, size=(rows, max(cols - 1, 0)))
        v = rng.integers(1, 5, size=(max(rows - 1, 0), cols))
        for order in ORDERS:
            if order == P.QUADRANT and (rows < 2 or cols < 2):
                continue
            got, ref = both(rows, cols, 0, h, v, order)
            assert got == ref


def test_every_quadrant_split_bit_exact():
    for h in range(1, 7):
        for w in range(1, 5):
            got, ref = both(7, 5, 3, order=P.QUADRANT, qh=h, qw=w)
            assert got == ref


def test_stats_match_oracle_plan():
    for (L, D, order) in [(10, 4, P.COLSWEEP), (12, 4, P.COLSWEEP), (12, 4, P.QUADRANT),
                          (10, 4, P.HEURISTIC), (13, 4, P.HEURISTIC)]:
        ref = P.plan_grid(L, L, D, order=order)
        info = tn.tn_plan_stats(tn.tn_plan_grid(L, L, D, order=order))
        assert info["peak_entries"] == ref.peak
        assert info["flops"] == ref.flops
        assert info["moved_entries"] == ref.moved
        assert info["n_steps"] == len(ref.steps)
        assert info["order"] == ref.order
    info = tn.tn_plan_stats(tn.tn_plan_grid(12, 12, 4))
    assert info["peak_entries"] == 4 ** 13 and info["flops"] == 226112132128


def test_errors():
    with pytest.raises(tn.TnError) as e:
        tn.tn_plan_grid(0, 3, 2)
    assert e.value.status == tn.TN_EINVAL
    with pytest.raises(tn.TnError) as e:
        tn.tn_plan_grid(3, 3, 0)
    assert e.value.status == tn.TN_EINVAL
    with pytest.raises(tn.TnError) as e:
        tn.tn_plan_grid(1, 5, 2, order=P.QUADRANT)
    assert e.value.status == tn.TN_EINVAL
    with pytest.raises(tn.TnError) as e:
        tn.tn_plan_grid(4, 4, 2, order=P.QUADRANT, quad_h=4)
    assert e.value.status == tn.TN_EINVAL
    with pytest.raises(tn.TnError) as e:
        tn.tn_plan_grid(40, 40, 64)
    assert e.value.status == tn.TN_EOVERFLOW
    with pytest.raises(tn.TnError) as e:
        tn.tn_plan_grid(3, 3, 2, order=7)
    assert e.value.status == tn.TN_EINVAL
    with pytest.raises(tn.TnError):
        tn.tn_plan_grid(3, 3, 2, hdim=[[2, 0], [2, 2], [2, 2]])


def test_batch_workspace_host_only():
    plans = [tn.tn_plan_grid(r, c, 3, order=tn.TN_ORDER_SWEEP_AUTO) for r, c in [(4, 5), (6, 3)]]
    n = tn.tn_batch_workspace(plans, "f32")
    assert n > 0
    with pytest.raises(tn.TnError) as e:
        tn.tn_batch_workspace([tn.tn_plan_grid(4, 4, 2, order=tn.TN_ORDER_QUADRANT)], "f32")
    assert e.value.status == tn.TN_EINVAL


def test_ring_split_slices_host_only():
    # Split-K of the ring products (1024 x 1024 output at D = 4 on 10 x 10 has
    # 64 tiles of 128 x 128: eight k ranges fill 512 workgroups); the
    # workspace holds that many slices of the stored product X.  A 12 x 12
    # ring has 1024 tiles (FP64) or 256 of 256 x 256 (FP32) and is not split.
    cases = {(10, 10): 8, (9, 7): 8, (8, 8): 2, (7, 9): 2, (12, 12): 1, (13, 13): 1}
    for (r, c), s in cases.items():
        info = tn.tn_plan_grid(r, c, 4, order=tn.TN_ORDER_QUADRANT).info()
        assert info["ring_slices"] == [s, s, s], (r, c, info["ring_slices"])
    one = tn.tn_plan_grid(10, 10, 4, order=tn.TN_ORDER_QUADRANT).info()
    assert one["workspace_bytes"][0] >= 8 * 1024 * 1024 * 8
    # no ring: sweeps; no MFMA ring: D = 3 gives m = 243
    assert tn.tn_plan_grid(10, 10, 4).info()["ring_slices"] == [0, 0, 0]
    assert tn.tn_plan_grid(10, 10, 3, order=tn.TN_ORDER_QUADRANT).info()["ring_slices"] == [1, 1, 1]


def test_row_scheme_and_budget_bit_exact():
    # every explicit order and the heuristic under budgets around each
    # candidate's storage: the same plan, or "too large" on both sides
    rng = np.random.default_rng(11)
    for _ in range(40):
        rows, cols = (int(x) for x in rng.integers(1, 8, size=2))
        D = int(rng.integers(1, 4))
        sizes = sorted({P.plan_grid(rows, cols, D, order=o).buffers
                        for o in (P.COLSWEEP, P.ROWS, P.ROWS_T)})
        if rows >= 2 and cols >= 2:
            sizes.append(P.plan_grid(rows, cols, D, order=P.QUADRANT).buffers)
        for b in sorted({s + d for s in sizes for d in (-1, 0)} | {0}):
            for order in (P.HEURISTIC, P.SWEEP_AUTO, P.COLSWEEP, P.ROWS, P.ROWS_T):
                try:
                    ref = P.plan_text(P.plan_grid(rows, cols, D, order=order, budget=b))
                except P.PlanTooLarge:
                    ref = None
                try:
                    got = tn.tn_plan_text(tn.tn_plan_grid(rows, cols, D, order=order, budget=b))
                except tn.TnError as e:
                    assert e.status == tn.TN_ENOMEM, (rows, cols, D, order, b)
                    got = None
                if b <= 0:
                    assert got is not None
                assert got == ref, (rows, cols, D, order, b)


def test_buffer_entries_match_oracle():
    for (r, c, D) in [(6, 6, 2), (8, 8, 2), (6, 6, 4), (12, 12, 4), (5, 7, 3), (1, 9, 2)]:
        for order in (P.COLSWEEP, P.HEURISTIC, P.ROWS, P.ROWS_T):
            ref = P.plan_grid(r, c, D, order=order)
            info = tn.tn_plan_grid(r, c, D, order=order).info()
            assert info["buffer_entries"] == ref.buffers
            assert info["n_links"] == len(ref.chain)
            assert info["peak_entries"] == ref.peak and info["flops"] == ref.flops

"""tn_contract_grid_static (the allocation-free entry point) against
tn_contract_grid on the same plans and sites, through the C ABI.

Two or more calls in a row, each later one on a smaller network, so a call
that depended on the static workspace's previous contents (counters, slots,
boundaries) would show.  The kernels are the same, so the results must be
bitwise equal; each is also checked against the FP64 oracle (|dlog Z| <=
1e-12 in FP64, 1e-5 max(1, |log Z|) in FP32 / BF16x3)."""
import pytest

import lattice_inputs as li
from oracle import contract as OC
from oracle import plan as OP

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tn():
    import torch
    assert torch.cuda.is_available()
    import paper_1908_08553_amd as tn
    return tn


def both(tn, plan, sites, prec, on_device=True):
    import torch
    pidx = {"f64": 0, "f32": 1, "bf16x3": 2}[prec]
    stream = torch.cuda.current_stream()
    if on_device:
        dev = tn.prepare_sites(tn.device_sites(sites))
        table, keep = dev.table, dev
    else:
        import ctypes
        import numpy as np
        keep = [np.ascontiguousarray(s, dtype=np.float64) for s in sites]
        table = (ctypes.c_void_p * len(keep))(*[a.ctypes.data for a in keep])
    ws = tn.workspace_for(plan, pidx)
    want = tn.tn_contract_grid(plan, table, on_device, pidx, ws.data_ptr(), ws.numel(),
                               stream.cuda_stream)
    got = tn.tn_contract_grid_static(plan, table, on_device, pidx, stream.cuda_stream)
    del keep
    return got, want


def check(got, want, ref, prec):
    assert got.status == want.status == 0
    assert (got.sign, got.mantissa, got.exp2_sum) == (want.sign, want.mantissa, want.exp2_sum)
    assert got.sign == ref.sign
    tol = 1e-12 if prec == "f64" else 1e-5 * max(1.0, abs(ref.log_abs))
    assert abs(got.log_abs - ref.log_abs) <= tol, (got.log_abs, ref.log_abs)


CASES = [  # largest first: each later call runs on a smaller workspace
    (10, 10, 4, "normal", OP.COLSWEEP, "f64"),     # 64.4 MiB of the 160 MiB
    (10, 10, 4, "uniform", OP.QUADRANT, "f32"),
    (8, 9, 3, "uniform", OP.HEURISTIC, "bf16x3"),
    (6, 6, 4, "normal", OP.QUADRANT, "f64"),
    (5, 7, 2, "uniform", OP.COLSWEEP, "f32"),
    (3, 3, 2, "normal", OP.COLSWEEP, "f64"),
]


def test_static_equals_workspace_calls(tn):
    for (r, c, D, kind, order, prec) in CASES:
        print(f"[gpu] static workspace {r}x{c} D={D} {kind} order={order} {prec}", flush=True)
        sites = li.make(kind, r, c, D, 7)
        plan = tn.tn_plan_grid(r, c, D, order=order)
        assert plan.info()["workspace_bytes"][{"f64": 0, "f32": 1, "bf16x3": 2}[prec]] \
            <= tn.TN_STATIC_SCRATCH_BYTES
        got, want = both(tn, plan, sites, prec)
        check(got, want, OC.contract_grid(sites, r, c, order), prec)


def test_static_host_sites_and_repeat(tn):
    sites = li.make("uniform", 7, 6, 3, 2)
    ref = OC.contract_grid(sites, 7, 6, OP.COLSWEEP)
    plan = tn.tn_plan_grid(7, 6, 3, order=tn.TN_ORDER_COLSWEEP)
    print("[gpu] static workspace 7x6 D=3 host sites, twice", flush=True)
    a, want = both(tn, plan, sites, "f64", on_device=False)
    check(a, want, ref, "f64")
    small = li.make("uniform", 4, 4, 2, 3)
    splan = tn.tn_plan_grid(4, 4, 2, order=tn.TN_ORDER_COLSWEEP)
    s, swant = both(tn, splan, small, "f64", on_device=False)
    check(s, swant, OC.contract_grid(small, 4, 4, OP.COLSWEEP), "f64")


def test_static_rejects_plans_beyond_its_size(tn):
    import torch
    plan = tn.tn_plan_grid(12, 12, 4, order=tn.TN_ORDER_HEURISTIC)   # 576 MiB in FP32
    assert plan.info()["workspace_bytes"][1] > tn.TN_STATIC_SCRATCH_BYTES
    table = tn.prepare_sites(tn.device_sites(li.make("uniform", 12, 12, 4, 0)))
    with pytest.raises(tn.TnError) as e:
        tn.tn_contract_grid_static(plan, table.table, True, 1,
                                   torch.cuda.current_stream().cuda_stream)
    assert e.value.status == tn.TN_ENOMEM

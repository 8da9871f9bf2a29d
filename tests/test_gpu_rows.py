"""The paper's row scheme (§4, Fig. 2a) on the GPU, through the C ABI: every
row contracted into one tensor, then the chain of row tensors closed by
float64 matrix-vector products.  Against the FP64 oracle on the same seeded
inputs: |d log Z| <= 1e-12 in FP64, <= 1e-5 max(1, |log Z|) in FP32 and
split BF16x3; sign exact."""
import numpy as np
import pytest

import lattice_inputs as li
from oracle import contract as C
from oracle import network as nw
from oracle import plan as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=["mfma", "valu"])
def tn(request):
    import torch
    assert torch.cuda.is_available()
    import paper_1908_08553_amd as tn
    tn.tn_set_option(tn.TN_OPT_KERNEL_IMPL, 0 if request.param == "mfma" else 1)
    yield tn
    tn.tn_set_option(tn.TN_OPT_KERNEL_IMPL, 0)


def run(tn, sites, rows, cols, order, prec, hdim=None, vdim=None):
    if hdim is None:
        dims = nw.dims_of(sites, rows, cols)
        hdim = [[dims[("h", r, c)] for c in range(cols - 1)] for r in range(rows)]
        vdim = [[dims[("v", r, c)] for c in range(cols)] for r in range(rows - 1)]
    plan = tn.tn_plan_grid(rows, cols, 1, hdim, vdim, order)
    assert plan.info()["order"] == tn.TN_ORDER_ROWS
    print(f"[gpu] rows {rows}x{cols} order={order} prec={prec}", flush=True)
    return tn.contract_grid(plan, tn.device_sites(sites), prec)


def check(got, ref, prec):
    assert got.status == 0 and got.sign == ref.sign, (got, ref)
    if ref.sign == 0:
        return
    tol = 1e-12 if prec == "f64" else 1e-5 * max(1.0, abs(ref.log_abs))
    assert abs(got.log_abs - ref.log_abs) <= tol, (got.log_abs, ref.log_abs)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("rows,cols,D,kind", [(6, 6, 2, "normal"), (6, 6, 3, "uniform"),
                                              (8, 8, 2, "uniform"), (5, 7, 2, "normal"),
                                              (7, 4, 3, "uniform")])
def test_rows_match_oracle(tn, rows, cols, D, kind, prec):
    s = li.make(kind, rows, cols, D, 13)
    ref = C.contract_grid(s, rows, cols, P.COLSWEEP)
    for order in (P.ROWS, P.ROWS_T):
        check(run(tn, s, rows, cols, order, prec), ref, prec)


@pytest.mark.parametrize("rows,cols", [(1, 1), (1, 6), (6, 1), (2, 2), (2, 5), (5, 2),
                                       (3, 3), (4, 5)])
def test_rows_thin_and_mixed_dims(tn, rows, cols):
    rng = np.random.default_rng(rows * 7 + cols)
    h = rng.integers(1, 5, size=(rows, max(cols - 1, 0)))
    v = rng.integers(1, 5, size=(max(rows - 1, 0), cols))
    s = li.normal(rows, cols, 0, 3, hdim=h, vdim=v)
    ref = C.contract_grid(s, rows, cols, P.COLSWEEP)
    for order in (P.ROWS, P.ROWS_T):
        for prec in ("f64", "f32"):
            check(run(tn, s, rows, cols, order, prec, h, v), ref, prec)


def test_rows_ising_8x8_matches_transfer_matrix(tn):
    for K in (0.1, 0.8):
        tm = nw.transfer_log_z(8, 8, K)
        got = run(tn, li.ising(8, 8, K), 8, 8, P.ROWS, "f64")
        assert got.sign == 1 and abs(got.log_abs - tm) <= 1e-12


def test_rows_6x6_d4_f64(tn):
    # bulk row tensors of 4^12 entries (134 MB in float64), chain links of
    # 4096 x 4096
    s = li.uniform(6, 6, 4, 2)
    ref = C.contract_grid(s, 6, 6, P.COLSWEEP)
    plan = tn.tn_plan_grid(6, 6, 4, order=tn.TN_ORDER_ROWS)
    info = plan.info()
    assert info["peak_entries"] == 4 ** 12 and info["n_links"] == 5
    print("[gpu] rows 6x6 D=4 f64", flush=True)
    got = tn.contract_grid(plan, tn.device_sites(s), "f64")
    check(got, ref, "f64")
    again = tn.contract_grid(plan, tn.device_sites(s), "f64")
    assert (again.mantissa, again.exp2_sum) == (got.mantissa, got.exp2_sum)


def test_rows_nonfinite_and_zero(tn):
    s = li.uniform(4, 4, 2, 1)
    s[5] = s[5].copy()
    s[5].flat[2] = np.nan
    got = run(tn, s, 4, 4, P.ROWS, "f64")
    assert got.status == tn.TN_ENONFINITE
    z = li.uniform(4, 4, 2, 1)
    z[9] = np.zeros_like(z[9])
    got = run(tn, z, 4, 4, P.ROWS, "f32")
    assert got.status == 0 and got.sign == 0

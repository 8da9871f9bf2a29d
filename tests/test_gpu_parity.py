"""HIP path vs the FP64 CPU oracle, through the C ABI, on seeded inputs.

Tolerances: FP64 1e-12 relative in Z; FP32 and split BF16x3 1e-5 relative in
log Z, read as |d log Z| <= 1e-5 * max(1, |log Z|) because log Z can be near 0
for tiny lattices."""
import math
import os

import numpy as np
import pytest

import lattice_inputs as li
from oracle import contract as C
from oracle import network as nw
from oracle import plan as P

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", params=["mfma", "valu"])
def tn(request):
    """The library, with absorption on the matrix cores where the step shape
    allows ("mfma") or forced onto the vector-ALU kernels ("valu")."""
    import torch
    assert torch.cuda.is_available()
    import paper_1908_08553_amd as tn
    tn.tn_set_option(tn.TN_OPT_KERNEL_IMPL, 0 if request.param == "mfma" else 1)
    yield tn
    tn.tn_set_option(tn.TN_OPT_KERNEL_IMPL, 0)


def ising_gold():
    out = {}
    with open(os.path.join(GOLD, "ising_logz.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                r, c, K, v = line.split()
                out[(int(r), int(c), float(K))] = float(v)
    return out


def gpu(tn, sites, rows, cols, order=P.COLSWEEP, prec="f64", qh=0, qw=0, D=None,
        hdim=None, vdim=None):
    if hdim is None:
        dims = nw.dims_of(sites, rows, cols)
        hdim = [[dims[("h", r, c)] for c in range(cols - 1)] for r in range(rows)]
        vdim = [[dims[("v", r, c)] for c in range(cols)] for r in range(rows - 1)]
    plan = tn.tn_plan_grid(rows, cols, 1, hdim, vdim, order, qh, qw)
    print(f"[gpu] {rows}x{cols} order={order} prec={prec}", flush=True)
    return tn.contract_grid(plan, tn.device_sites(sites), prec)


def oracle(sites, rows, cols, order=P.COLSWEEP, qh=0, qw=0):
    return C.contract_grid(sites, rows, cols, order, qh, qw)


def close_f64(got, ref, tol=1e-12):
    assert got.status == 0
    assert got.sign == ref.sign
    if ref.sign == 0:
        return
    # relative error in Z through log|Z| (exponents can exceed double range)
    assert abs(got.log_abs - ref.log_abs) <= tol, (got, ref)


def close_log(got, ref_log, tol=1e-5):
    assert got.status == 0 and got.sign == 1
    assert abs(got.log_abs - ref_log) <= tol * max(1.0, abs(ref_log)), (got.log_abs, ref_log)


# ------------------------------------------------- configuration 1 (4x4, D=2)

@pytest.mark.parametrize("seed", range(10))
def test_cfg1_uniform_4x4_f64(tn, seed):
    s = li.uniform(4, 4, 2, seed)
    got = gpu(tn, s, 4, 4)
    close_f64(got, oracle(s, 4, 4))
    assert abs(got.value - nw.brute_bonds(s, 4, 4)) <= 1e-12 * abs(got.value)


def test_cfg1_ising_4x4_equals_spin_sum(tn):
    got = gpu(tn, li.ising(4, 4, 0.4), 4, 4)
    z = nw.brute_spins(4, 4, 0.4)
    assert abs(got.value - z) <= 1e-12 * z


# ------------------------------------------------ configuration 2 (10x10, D=4)

@pytest.mark.parametrize("seed", range(5))
def test_cfg2_normal_10x10_f64(tn, seed):
    s = li.normal(10, 10, 4, seed)
    got = gpu(tn, s, 10, 10)
    ref = oracle(s, 10, 10)
    print(f"  log|Z| gpu {got.log_abs!r} oracle {ref.log_abs!r} sign {got.sign}")
    close_f64(got, ref)


@pytest.mark.parametrize("K", [0.2, 0.44, 0.6])
def test_cfg2_ising_10x10_f64(tn, K):
    tm = ising_gold()[(10, 10, K)]
    got = gpu(tn, li.ising(10, 10, K), 10, 10)
    assert got.sign == 1 and abs(got.log_abs - tm) <= 1e-12
    got4 = gpu(tn, li.ising_d4(10, 10, K), 10, 10)
    assert got4.sign == 1 and abs(got4.log_abs - 2 * tm) <= 1e-12


# -------------------------------------------------- every order, small sizes

@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
@pytest.mark.parametrize("order", [P.COLSWEEP, P.QUADRANT, P.HEURISTIC])
def test_orders_and_precisions_6x6_d4(tn, prec, order):
    s = li.uniform(6, 6, 4, 3)
    ref = oracle(s, 6, 6, P.COLSWEEP)
    got = gpu(tn, s, 6, 6, order, prec)
    if prec == "f64":
        close_f64(got, ref)
    else:
        close_log(got, ref.log_abs)


@pytest.mark.parametrize("rows,cols", [(1, 1), (1, 2), (2, 1), (1, 7), (7, 1), (2, 2),
                                       (2, 3), (3, 2), (5, 3), (3, 8), (9, 4)])
def test_thin_and_ragged_lattices(tn, rows, cols):
    rng = np.random.default_rng(rows * 31 + cols)
    h = rng.integers(1, 5, size=(rows, max(cols - 1, 0)))
    v = rng.integers(1, 5, size=(max(rows - 1, 0), cols))
    s = li.uniform(rows, cols, 0, 1, hdim=h, vdim=v)
    orders = [P.COLSWEEP, P.HEURISTIC] + ([P.QUADRANT] if rows > 1 and cols > 1 else [])
    for order in orders:
        ref = oracle(s, rows, cols, order)
        for prec in ("f64", "f32", "bf16x3"):
            got = gpu(tn, s, rows, cols, order, prec, hdim=h, vdim=v)
            if prec == "f64":
                close_f64(got, ref, 1e-13)
            else:
                close_log(got, ref.log_abs)


def test_bond_dim_one_and_three(tn):
    for D in (1, 3):
        s = li.uniform(5, 6, D, 2)
        ref = oracle(s, 5, 6)
        close_f64(gpu(tn, s, 5, 6), ref)
        close_log(gpu(tn, s, 5, 6, prec="f32"), ref.log_abs)


def test_all_ones_closed_form(tn):
    for (L, D) in [(8, 2), (6, 4), (12, 2)]:
        got = gpu(tn, li.ones(L, L, D), L, L, P.HEURISTIC)
        nb = 2 * L * (L - 1)
        assert got.mantissa == 0.5 and got.exp2_sum == nb * int(math.log2(D)) + 1


def test_zero_network_and_nonfinite_input(tn):
    s = li.uniform(4, 5, 3, 0)
    s[7] = np.zeros_like(s[7])
    got = gpu(tn, s, 4, 5)
    assert got.status == 0 and got.sign == 0 and got.log_abs == -math.inf
    s = li.uniform(4, 5, 3, 0)
    s[3] = s[3].copy()
    s[3].flat[2] = np.nan
    got = gpu(tn, s, 4, 5)
    assert got.status == tn.TN_ENONFINITE


def test_host_sites_and_workspace_errors(tn):
    import torch
    s = li.uniform(5, 5, 3, 4)
    plan = tn.tn_plan_grid(5, 5, 3)
    ref = oracle(s, 5, 5)
    got = tn.contract_grid(plan, s, "f64")           # numpy sites: host path
    close_f64(got, ref)
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(tn.TnError) as e:
        tn.contract_grid(plan, tn.device_sites(s), "f64", workspace=small)
    assert e.value.status == tn.TN_ENOMEM


def test_deterministic_bitwise(tn):
    s = li.normal(8, 8, 4, 9)
    for prec in ("f64", "f32", "bf16x3"):
        a = gpu(tn, s, 8, 8, P.QUADRANT, prec)
        b = gpu(tn, s, 8, 8, P.QUADRANT, prec)
        assert (a.mantissa, a.exp2_sum) == (b.mantissa, b.exp2_sum)


# ------------------------------------------ configuration 3 (12x12, D=4)

@pytest.fixture(scope="module")
def cfg3_uniform():
    s = li.uniform(12, 12, 4, 0)
    return s, oracle(s, 12, 12, P.QUADRANT)      # the oracle's fastest exact plan


@pytest.mark.parametrize("order", [P.COLSWEEP, P.HEURISTIC])
@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f64"])
def test_cfg3_uniform_12x12_d4(tn, cfg3_uniform, order, prec):
    s, ref = cfg3_uniform
    got = gpu(tn, s, 12, 12, order, prec)
    print(f"  12x12 D=4 {prec} order={order}: log|Z| {got.log_abs!r} oracle {ref.log_abs!r}")
    if prec == "f64":
        close_f64(got, ref)
    else:
        close_log(got, ref.log_abs)


@pytest.mark.parametrize("D", [2, 4])
@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_cfg3_ising_12x12(tn, D, prec):
    tm = ising_gold()[(12, 12, 0.44)] * (1 if D == 2 else 2)
    sites = li.ising(12, 12, 0.44) if D == 2 else li.ising_d4(12, 12, 0.44)
    for order in (P.COLSWEEP, P.HEURISTIC):
        close_log(gpu(tn, sites, 12, 12, order, prec), tm)


def test_cfg3_ising_13x13_d4_f64(tn):
    # the largest served size: 13x13 two-replica network, FP64 sweep (peak 4^14)
    tm = 2 * ising_gold()[(13, 13, 0.44)]
    got = gpu(tn, li.ising_d4(13, 13, 0.44), 13, 13, P.HEURISTIC, "f64")
    assert got.sign == 1 and abs(got.log_abs - tm) <= 1e-12


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f64"])
def test_ring_with_ragged_tiles(tn, prec):
    # 8x10 lattice whose quadrant cut gives m = n = 4*4*3*4*4 = 768 (three
    # 256-wide tiles, six 128-wide ones) and k = 2^4: edge tiles of every ring kernel
    rows, cols = 8, 10
    h = np.full((rows, cols - 1), 2)
    v = np.tile(np.array([4, 4, 3, 4, 4, 4, 4, 3, 4, 4]), (rows - 1, 1))
    s = li.uniform(rows, cols, 0, 21, hdim=h, vdim=v)
    ref = oracle(s, rows, cols, P.QUADRANT, 4, 5)
    got = gpu(tn, s, rows, cols, P.QUADRANT, prec, 4, 5, hdim=h, vdim=v)
    if prec == "f64":
        close_f64(got, ref)
    else:
        close_log(got, ref.log_abs)


def test_prepared_sites_same_result(tn):
    # a pointer table built once gives the same contraction as the site list
    s = li.uniform(6, 7, 3, 5)
    plan = tn.tn_plan_grid(6, 7, 3, order=P.HEURISTIC)
    dev = tn.device_sites(s)
    a = tn.contract_grid(plan, dev, "f64")
    prepared = tn.prepare_sites(dev)
    b = tn.contract_grid(plan, prepared, "f64")
    c = tn.contract_grid(plan, prepared, "f64")
    assert (a.mantissa, a.exp2_sum, a.sign) == (b.mantissa, b.exp2_sum, b.sign) == \
        (c.mantissa, c.exp2_sum, c.sign)
    with pytest.raises(ValueError):
        tn.prepare_sites([t.float() for t in dev])

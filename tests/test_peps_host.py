"""Host-side parts of the PEPS observable calls (no GPU): tn_observables
forms the paper's ratios (§3: <O> = <Psi|O|Psi> / <Psi|Psi>, c_ij connected)
from exact network results, and tn_double_layer rejects bad descriptors
before touching the device."""
import ctypes as C

import numpy as np
import pytest

import lattice_inputs as li
import paper_1908_08553_amd as tn
from oracle import contract as OC
from oracle import peps as Q
from oracle import plan as P

SX, SZ = li.spin_half()


def as_tn(r: OC.Result):
    return tn.Result(r.sign, 0, r.log_abs, r.value, r.mantissa, r.exp2)


@pytest.mark.parametrize("rows,cols,seed", [(3, 3, 0), (2, 4, 1), (1, 3, 2)])
def test_observables_from_oracle_results(rows, cols, seed):
    peps = li.peps(rows, cols, 2, seed)
    nets = Q.networks_for_observables(peps, rows, cols, SX, SZ)
    res = [OC.contract_grid(s, rows, cols, P.COLSWEEP) for s in nets]
    want = Q.observables(res, rows, cols)
    mx, mz, czz = tn.tn_observables([as_tn(r) for r in res], rows, cols)
    np.testing.assert_allclose(mx, want["mx"], rtol=1e-15, atol=1e-300)
    np.testing.assert_allclose(mz, want["mz"], rtol=1e-15, atol=1e-300)
    np.testing.assert_allclose(czz, want["czz"], rtol=1e-14, atol=1e-16)
    assert len(czz) == rows * (cols - 1) + (rows - 1) * cols


def test_observables_errors():
    rows, cols = 2, 2
    n = 1 + 2 * 4 + 4
    ok = tn.Result(1, 0, 0.0, 1.0, 0.5, 1)
    zero = tn.Result(0, 0, float("-inf"), 0.0, 0.0, 0)
    bad = tn.Result(1, tn.TN_ENONFINITE, 0.0, 1.0, 0.5, 1)
    with pytest.raises(tn.TnError) as e:
        tn.tn_observables([zero] + [ok] * (n - 1), rows, cols)
    assert e.value.status == tn.TN_EINVAL
    with pytest.raises(tn.TnError) as e:
        tn.tn_observables([ok] * (n - 1) + [bad], rows, cols)
    assert e.value.status == tn.TN_ENONFINITE
    with pytest.raises(ValueError):
        tn.tn_observables([ok] * (n - 1), rows, cols)
    # a zero numerator is a zero observable
    mx, mz, czz = tn.tn_observables([ok] + [zero] * (n - 1), rows, cols)
    assert mx == [0.0] * 4 and mz == [0.0] * 4 and czz == [0.0] * 4


def test_double_layer_rejects_bad_sites_without_a_device():
    site = tn._native.tn_double_layer_site
    fake = 0x1000   # never dereferenced: validation fails first
    bad = [
        site(fake, None, fake, 2, 5, (C.c_int32 * 4)(2, 2, 2, 2)),     # rank > 4
        site(fake, None, fake, 0, 2, (C.c_int32 * 4)(2, 2, 1, 1)),     # d < 1
        site(fake, None, fake, 2, 2, (C.c_int32 * 4)(2, 0, 1, 1)),     # dim < 1
        site(None, None, fake, 2, 1, (C.c_int32 * 4)(2, 1, 1, 1)),     # NULL A
        site(fake, None, None, 2, 1, (C.c_int32 * 4)(2, 1, 1, 1)),     # NULL E
        site(fake, None, fake, 2, 4, (C.c_int32 * 4)(256, 256, 256, 256)),   # > 2^30 entries
    ]
    for s in bad:
        arr = (site * 1)(s)
        assert tn.lib.tn_double_layer(arr, 1, None) == tn.TN_EINVAL
    assert tn.lib.tn_double_layer(None, 1, None) == tn.TN_EINVAL
    assert tn.lib.tn_double_layer(None, 0, None) == tn.TN_OK

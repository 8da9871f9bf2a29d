"""Quadrant plans with TN_OPT_QUADRANT_STREAMS = 1: the two bottom quadrants
are swept on a second stream while the top ones and the first ring product
run on the caller's stream.  Every unit does the same work in the same order
either way (only the grouping of launches differs), so the results must be
bitwise identical to the one-stream path, and the FP64 oracle pins both.

This file sorts after the server tests on purpose: the second stream takes
one of the process's hardware queues for the rest of the process."""
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
    tn.tn_set_option(tn.TN_OPT_QUADRANT_STREAMS, 0)


@pytest.fixture(scope="module")
def net():
    s = li.uniform(12, 12, 4, 0)
    return s, C.contract_grid(s, 12, 12, P.QUADRANT, 0, 0)


def run(tn, sites, prec, on):
    tn.tn_set_option(tn.TN_OPT_QUADRANT_STREAMS, 1 if on else 0)
    plan = tn.tn_plan_grid(12, 12, 4, order=tn.TN_ORDER_QUADRANT)
    print(f"[gpu] quadrant streams={on} prec={prec}", flush=True)
    return tn.contract_grid(plan, tn.device_sites(sites), prec)


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f64"])
def test_two_streams_equal_one_stream(tn, net, prec):
    s, ref = net
    one = run(tn, s, prec, False)
    two = run(tn, s, prec, True)
    assert (two.status, two.sign, two.exp2_sum, two.mantissa) == \
           (one.status, one.sign, one.exp2_sum, one.mantissa)
    tol = 1e-12 if prec == "f64" else 1e-5 * abs(ref.log_abs)
    assert abs(two.log_abs - ref.log_abs) <= tol


def test_two_streams_repeatable(tn, net):
    s, _ = net
    a = run(tn, s, "f32", True)
    b = run(tn, s, "f32", True)
    assert (a.mantissa, a.exp2_sum) == (b.mantissa, b.exp2_sum)

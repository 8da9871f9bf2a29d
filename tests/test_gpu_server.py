"""Served request loop: admission by footprint, overlap on the device,
results identical alone and in the mix, error paths."""
import math
import time

import numpy as np
import pytest

import lattice_inputs as li
from oracle import contract as OC
from oracle import network as nw

pytestmark = pytest.mark.gpu
GiB = 1 << 30


@pytest.fixture(scope="module")
def tn():
    import torch
    assert torch.cuda.is_available()
    import paper_1908_08553_amd as tn
    tn.tn_set_option(tn.TN_OPT_KERNEL_IMPL, 0)
    return tn


def ising_request(L, D, K):
    sites = li.ising(L, L, K) if D == 2 else li.ising_d4(L, L, K)
    want = nw.transfer_log_z(L, L, K) * (1 if D == 2 else 2)
    return sites, want


def test_mixed_requests_match_the_transfer_matrix(tn):
    srv = tn.Server(8 * GiB, max_slots=4)
    reqs = []
    rng = np.random.default_rng(5)
    for k in range(24):
        L = int(rng.integers(4, 12))
        D = int(rng.choice([2, 4]))
        K = float(rng.uniform(0.1, 0.8))
        prec = "f64" if k % 2 == 0 else "bf16x3"
        sites, want = ising_request(L, D, K)
        reqs.append((srv.submit(L, L, sites, D=D, precision=prec), want, prec, L, D))
    for t, want, prec, L, D in reqs:
        res, times = srv.wait(t)
        assert res.status == 0 and res.sign == 1
        tol = 1e-12 if prec == "f64" else 1e-5 * want
        assert abs(res.log_abs - want) <= tol, (L, D, prec, res.log_abs, want)
        assert times[0] <= times[1] <= times[2]
    st = srv.stats()
    assert st["completed"] == 24 and st["active"] == 0 and st["queued"] == 0
    srv.close()


def test_alone_equals_in_the_mix_bitwise(tn):
    # the 13x13 FP64 request runs long enough for the others to be admitted
    # beside it, whatever their own speed
    specs = [(13, 4, 0.44, "f64"), (5, 4, 0.3, "f64"), (9, 2, 0.5, "bf16x3"), (7, 4, 0.7, "f64"), (4, 2, 0.2, "bf16x3"),
             (10, 4, 0.44, "bf16x3"), (6, 4, 0.6, "f64")]
    srv = tn.Server(16 * GiB, max_slots=3)
    alone = []
    for L, D, K, prec in specs:
        sites, _ = ising_request(L, D, K)
        res, _ = srv.wait(srv.submit(L, L, sites, D=D, precision=prec))
        alone.append((res.mantissa, res.exp2_sum))
    tickets = []
    for L, D, K, prec in specs:
        sites, _ = ising_request(L, D, K)
        tickets.append(srv.submit(L, L, sites, D=D, precision=prec))
    mixed = []
    for t in tickets:
        res, _ = srv.wait(t)
        mixed.append((res.mantissa, res.exp2_sum))
    assert mixed == alone
    assert srv.stats()["peak_active"] >= 2
    srv.close()


def test_nonfinite_request_is_isolated_in_the_mix(tn):
    # A request whose sites hold a NaN (or an Inf) runs beside others: it
    # returns TN_ENONFINITE, and every other request's result is bitwise its
    # result alone.  The 13x13 FP64 request keeps the device busy while the
    # bad ones are admitted beside it.
    def bad_sites(L, D, K, value, where):
        sites, _ = ising_request(L, D, K)
        sites = [np.array(t, copy=True) for t in sites]
        sites[where].flat[0] = value
        return sites

    good = [(13, 4, 0.44, "f64"), (6, 4, 0.5, "f64"), (9, 2, 0.3, "bf16x3"), (8, 4, 0.6, "f64"),
            (5, 2, 0.7, "bf16x3"), (11, 4, 0.25, "bf16x3")]
    bad = [(7, 4, 0.4, "f64", np.nan, 24), (10, 4, 0.4, "bf16x3", np.inf, 55),
           (6, 2, 0.2, "f64", np.nan, 35)]
    srv = tn.Server(16 * GiB, max_slots=3)
    alone = []
    for L, D, K, prec in good:
        sites, want = ising_request(L, D, K)
        res, _ = srv.wait(srv.submit(L, L, sites, D=D, precision=prec))
        assert res.status == 0
        alone.append((res.sign, res.mantissa, res.exp2_sum))
    print("[gpu] server: good requests alone done; mixing in non-finite ones", flush=True)
    order = [("g", 0), ("b", 0), ("g", 1), ("g", 2), ("b", 1), ("g", 3), ("g", 4), ("b", 2),
             ("g", 5)]
    tickets = []
    for kind, i in order:
        if kind == "g":
            L, D, K, prec = good[i]
            sites, _ = ising_request(L, D, K)
        else:
            L, D, K, prec, value, where = bad[i]
            sites = bad_sites(L, D, K, value, where)
        tickets.append((kind, i, srv.submit(L, L, sites, D=D, precision=prec)))
    mixed = {}
    for kind, i, t in tickets:
        while True:
            st, res, _ = srv.poll(t)
            if st != tn.TN_PENDING:
                break
            time.sleep(1e-4)
        if kind == "b":
            assert st == tn.TN_ENONFINITE and res.status == tn.TN_ENONFINITE, (bad[i], st)
        else:
            assert st == tn.TN_OK and res.status == 0
            mixed[i] = (res.sign, res.mantissa, res.exp2_sum)
    assert [mixed[i] for i in range(len(good))] == alone
    st = srv.stats()
    assert st["peak_active"] >= 2 and st["active"] == 0 and st["queued"] == 0
    srv.close()


def test_small_requests_overtake_a_running_large_one(tn):
    # three slots: with 4 hardware queues per process (GPU_MAX_HW_QUEUES) and
    # the caller's own stream, more slot streams would share a queue with the
    # large request and wait behind its kernels
    srv = tn.Server(16 * GiB, max_slots=3)
    big_sites, big_want = ising_request(13, 4, 0.44)
    big = srv.submit(13, 13, big_sites, D=4, precision="f64")
    small = []
    for k in range(6):
        s, w = ising_request(5, 2, 0.3 + 0.05 * k)
        small.append((srv.submit(5, 5, s, D=2, precision="f64"), w))
    admit_small, done_small = [], []
    for t, w in small:
        res, times = srv.wait(t)
        assert abs(res.log_abs - w) <= 1e-12
        admit_small.append(times[1])
        done_small.append(times[2])
    res, times_big = srv.wait(big)
    assert abs(res.log_abs - big_want) <= 1e-12
    # continuous batching: every small request was admitted while the large
    # one ran, and they overtook it.  Streams that other code in the process
    # created earlier (a side stream per thread, graph fork streams) take
    # hardware queues for good, and a slot stream that shares a queue with
    # the large request waits behind its kernels: most, not all, finish first
    assert max(admit_small) < times_big[2], (admit_small, times_big)
    assert sum(d < times_big[2] for d in done_small) >= 4, (done_small, times_big)
    srv.close()


def test_admission_by_footprint(tn):
    # room for one 12x12 D=4 FP64 workspace at a time (two would not fit)
    import paper_1908_08553_amd as T
    plan = T.tn_plan_grid(12, 12, 4, order=T.TN_ORDER_HEURISTIC)
    need = plan.info()["workspace_bytes"][0]
    srv = tn.Server(int(need * 1.5), max_slots=4)
    s1, w = ising_request(12, 4, 0.44)
    t1 = srv.submit(12, 12, s1, D=4, precision="f64")
    t2 = srv.submit(12, 12, s1, D=4, precision="f64")
    r1, tm1 = srv.wait(t1)
    r2, tm2 = srv.wait(t2)
    assert tm2[1] >= tm1[2]          # the second was admitted after the first finished
    assert (r1.mantissa, r1.exp2_sum) == (r2.mantissa, r2.exp2_sum)
    st = srv.stats()
    assert st["peak_arena_in_use"] <= st["arena_bytes"] and st["peak_active"] == 1
    srv.close()


def test_error_paths(tn):
    srv = tn.Server(64 << 20, max_slots=1, queue_depth=2)
    sites, _ = ising_request(12, 4, 0.4)
    with pytest.raises(tn.TnError) as e:          # footprint larger than the arena
        srv.submit(12, 12, sites, D=4, precision="f64")
    assert e.value.status == tn.TN_ENOMEM
    small, want = ising_request(4, 2, 0.4)
    t = srv.submit(4, 4, small, D=2)
    res, _ = srv.wait(t)
    assert abs(res.log_abs - want) <= 1e-12
    with pytest.raises(tn.TnError) as e:          # already retired
        srv.poll(t)
    assert e.value.status == tn.TN_ENOTFOUND
    bad = li.uniform(4, 4, 2, 0)
    bad[3] = bad[3].copy()
    bad[3].flat[1] = np.nan
    st, res, _ = (None, None, None)
    tb = srv.submit(4, 4, bad, D=2)
    while True:
        st, res, _ = srv.poll(tb)
        if st != tn.TN_PENDING:
            break
        time.sleep(1e-4)
    assert st == tn.TN_ENONFINITE and res.status == tn.TN_ENONFINITE
    srv.close()


def test_queue_full_returns_busy(tn):
    srv = tn.Server(8 * GiB, max_slots=1, queue_depth=1)
    big, _ = ising_request(13, 4, 0.44)
    tickets = [srv.submit(13, 13, big, D=4, precision="f64")]
    busy = False
    for _ in range(4):
        try:
            tickets.append(srv.submit(13, 13, big, D=4, precision="f64"))
        except tn.TnError as e:
            assert e.status == tn.TN_EBUSY
            busy = True
            break
    assert busy
    for t in tickets:
        srv.wait(t)
    srv.close()

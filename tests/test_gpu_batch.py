"""Batched contraction (one captured hipGraph: one workgroup per lattice plus
lock-step launches for the costliest) vs the CPU oracle and vs single
contractions, through the C ABI."""
import math

import numpy as np
import pytest

import lattice_inputs as li
from oracle import contract as OC

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tn():
    import torch
    assert torch.cuda.is_available()
    import paper_1908_08553_amd as tn
    tn.tn_set_option(tn.TN_OPT_KERNEL_IMPL, 0)
    # single contractions here run one launch per step: the batch kernel's own
    # per-step bodies in the same order of arithmetic, so alone == in the
    # batch bitwise (fused column chunks sum in another order)
    tn.tn_set_option(tn.TN_OPT_FUSE_STEPS, 0)
    yield tn
    tn.tn_set_option(tn.TN_OPT_FUSE_STEPS, 2)


def build(tn, mix):
    plans = [tn.tn_plan_grid(r, c, D, order=tn.TN_ORDER_SWEEP_AUTO) for r, c, D, _ in mix]
    sites = [tn.device_sites(s) for _, _, _, s in mix]
    return plans, sites


@pytest.fixture(scope="module")
def mix48():
    mix = li.batch_mix(48, 7)
    ref = [OC.contract_grid(s, r, c) for r, c, _, s in mix]
    return mix, ref


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_batch_vs_oracle_and_single(tn, mix48, prec):
    mix, ref = mix48
    plans, sites = build(tn, mix)
    print(f"[gpu] batch of {len(mix)} prec={prec}", flush=True)
    b = tn.Batch(plans, prec)
    res = b.run(sites)
    for i, (got, want) in enumerate(zip(res, ref)):
        assert got.status == 0 and got.sign == 1 == want.sign
        tol = 1e-12 if prec == "f64" else 1e-5 * max(1.0, abs(want.log_abs))
        assert abs(got.log_abs - want.log_abs) <= tol, (i, mix[i][:3], got, want)
        single = tn.contract_grid(plans[i], sites[i], prec)
        assert (single.mantissa, single.exp2_sum) == (got.mantissa, got.exp2_sum), i
    b.close()


def test_graph_replays_match_eager(tn, mix48):
    mix, ref = mix48
    plans, sites = build(tn, mix)
    b = tn.Batch(plans, "f32")
    first = b.run(sites)
    for rep in range(3):
        # eager work on the same stream between replays
        for i in (0, 5, 11):
            e = tn.contract_grid(plans[i], sites[i], "f32")
            assert (e.mantissa, e.exp2_sum) == (first[i].mantissa, first[i].exp2_sum)
        again = b.run(sites)
        assert [(r.mantissa, r.exp2_sum) for r in again] == \
               [(r.mantissa, r.exp2_sum) for r in first], rep
    b.close()


def test_changed_site_pointers_rebuild_their_descriptors(tn):
    # the staging descriptors are rebuilt only for lattices whose site
    # pointers changed since the previous run: A, then A with one lattice's
    # sites swapped for new tensors, then A again
    mix = li.batch_mix(10, 31)
    plans, sites_a = build(tn, mix)
    r, c, D, _ = mix[4]
    other = li.uniform(r, c, D, 4321)
    sites_b = list(sites_a)
    sites_b[4] = tn.device_sites(other)
    b = tn.Batch(plans, "f64", split=3)
    first = b.run(sites_a)
    second = b.run(sites_b)
    third = b.run(sites_a)
    assert abs(second[4].log_abs - OC.contract_grid(other, r, c).log_abs) <= 1e-12
    for i in range(10):
        assert (third[i].mantissa, third[i].exp2_sum) == (first[i].mantissa, first[i].exp2_sum)
        if i != 4:
            assert (second[i].mantissa, second[i].exp2_sum) == \
                   (first[i].mantissa, first[i].exp2_sum)
    assert np.array_equal(third.log_abs, first.log_abs) and len(third) == 10
    b.close()


def test_configs_are_bitwise_identical(tn, mix48):
    mix, _ = mix48
    plans, sites = build(tn, mix)
    out = None
    for threads in (256, 512, 1024):
        b = tn.Batch(plans, "bf16x3", threads)
        r = [(x.mantissa, x.exp2_sum) for x in b.run(sites)]
        b.close()
        assert out is None or r == out, threads
        out = r


def test_new_sites_same_batch(tn):
    mix_a = li.batch_mix(12, 100)
    plans, sites_a = build(tn, mix_a)
    # same shapes, different entries: the captured graph is reused
    sites_b = [tn.device_sites(li.uniform(r, c, D, 999 + i)) for i, (r, c, D, _) in enumerate(mix_a)]
    b = tn.Batch(plans, "f64")
    ra = b.run(sites_a)
    rb = b.run(sites_b)
    for i, (r, c, D, s) in enumerate(mix_a):
        assert abs(ra[i].log_abs - OC.contract_grid(s, r, c).log_abs) < 1e-12
        sb = li.uniform(r, c, D, 999 + i)
        assert abs(rb[i].log_abs - OC.contract_grid(sb, r, c).log_abs) < 1e-12
    b.close()


def test_nonfinite_lattice_is_isolated(tn):
    mix = li.batch_mix(10, 3)
    mix[4][3][5] = mix[4][3][5].copy()
    mix[4][3][5].flat[0] = np.inf
    plans, sites = build(tn, mix)
    res = tn.tn_contract_batch(plans, sites, "f32")
    for i, r in enumerate(res):
        if i == 4:
            assert r.status == tn.TN_ENONFINITE
        else:
            rr, cc, _, s = mix[i]
            assert r.status == 0
            assert abs(r.log_abs - OC.contract_grid(s, rr, cc).log_abs) < 1e-5 * max(1, r.log_abs)


def test_thin_and_tiny_lattices_in_a_batch(tn):
    shapes = [(1, 1, 3), (1, 6, 2), (6, 1, 4), (2, 2, 4), (2, 9, 3), (3, 3, 1)]
    mix = [(r, c, D, li.uniform(r, c, D, 50 + k)) for k, (r, c, D) in enumerate(shapes)]
    plans, sites = build(tn, mix)
    for prec in ("f64", "f32"):
        res = tn.Batch(plans, prec).run(sites)
        for (r, c, D, s), got in zip(mix, res):
            want = OC.contract_grid(s, r, c)
            tol = 1e-12 if prec == "f64" else 1e-5 * max(1, abs(want.log_abs))
            assert abs(got.log_abs - want.log_abs) <= tol, (r, c, D)


def test_512_lattice_mix_sampled(tn):
    # the full 512-lattice configuration; the oracle checks a sample
    mix = li.batch_mix(512, 2024)
    plans, sites = build(tn, mix)
    res = tn.Batch(plans, "f32").run(sites)
    assert all(r.status == 0 and r.sign == 1 and math.isfinite(r.log_abs) for r in res)
    for i in range(0, 512, 37):
        r, c, _, s = mix[i]
        want = OC.contract_grid(s, r, c)
        assert abs(res[i].log_abs - want.log_abs) <= 1e-5 * max(1, want.log_abs), i


def test_autotuner_picks_a_config_and_caches_it(tn, tmp_path, monkeypatch):
    from paper_1908_08553_amd import autotune
    monkeypatch.setenv("TN_TUNE_CACHE", str(tmp_path / "cache.json"))
    mix = li.batch_mix(32, 11)
    plans, sites = build(tn, mix)
    out = autotune.tune_batch(plans, sites, "f32", candidates=[256, 512], splits=[0, 4, 32],
                              reps=2)
    assert out["best"] in (256, 512) and out["split"] in (0, 4, 32)
    assert autotune.tuned_config(plans, "f32") == (out["best"], out["split"])
    b = autotune.tuned_batch(plans, "f32")
    assert len(b.run(sites)) == 32


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_lockstep_split_is_bitwise_the_same(tn, mix48, prec):
    # the costliest lattices in lock-step over the GPU, the rest one
    # workgroup each: every split (none, some, all) and workgroup size gives
    # the same bits, and the split lattices match the oracle
    mix, ref = mix48
    plans, sites = build(tn, mix)
    base = None
    for threads, split in [(512, 0), (256, 5), (1024, 17), (512, 48)]:
        print(f"[gpu] batch prec={prec} threads={threads} split={split}", flush=True)
        b = tn.Batch(plans, prec, threads, split=split)
        res = b.run(sites)
        again = b.run(sites)
        b.close()
        bits = [(r.sign, r.mantissa, r.exp2_sum) for r in res]
        assert bits == [(r.sign, r.mantissa, r.exp2_sum) for r in again]
        if base is None:
            base = bits
        assert bits == base, (threads, split)
    for got, want in zip(res, ref):
        tol = 1e-12 if prec == "f64" else 1e-5 * max(1.0, abs(want.log_abs))
        assert abs(got.log_abs - want.log_abs) <= tol


def test_lockstep_nonfinite_lattice_is_flagged(tn):
    mix = li.batch_mix(12, 3)
    plans, sites = build(tn, mix)
    costs = [p.info()["flops"] for p in plans]
    worst = int(np.argmax(costs))
    import torch
    sites[worst][len(sites[worst]) // 2].view(-1)[0] = float("nan")
    b = tn.Batch(plans, "f32", 512, split=3)
    res = b.run(sites)
    b.close()
    assert res[worst].status == tn.TN_ENONFINITE
    assert all(r.status == 0 for i, r in enumerate(res) if i != worst)


def test_quadrant_plan_rejected(tn):
    import torch
    plans = [tn.tn_plan_grid(4, 4, 2, order=tn.TN_ORDER_QUADRANT)]
    with pytest.raises(tn.TnError) as e:
        tn.Batch(plans, "f32")
    assert e.value.status == tn.TN_EINVAL

"""PEPS norm and observables on the GPU (paper §3: <O> = <Psi|O|Psi> /
<Psi|Psi>; §5: one full contraction of O|Psi> against <Psi| per site and per
nearest-neighbour pair), checked against the FP64 oracle:

* tn_double_layer against the oracle's double-layer site, elementwise, for
  ranks 0..4 (corner, edge, bulk and the thin-lattice cases), spin
  dimensions 1..3, mixed bond dimensions, with and without an operator;
* one whole observable evaluation (norm, m^x, m^z, c_ij: 1 + 2 L^2 +
  2 L (L-1) networks in one batch launch) against the oracle's values, FP64.
"""
import numpy as np
import pytest

import lattice_inputs as li
from oracle import contract as OC
from oracle import peps as Q
from oracle import plan as P

pytestmark = pytest.mark.gpu

SX, SZ = li.spin_half()


@pytest.fixture(scope="module")
def tn():
    import torch
    assert torch.cuda.is_available()
    import paper_1908_08553_amd as tn
    tn.tn_set_option(tn.TN_OPT_KERNEL_IMPL, 0)
    return tn


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


@pytest.mark.parametrize("shape", [(2,), (3, 4), (2, 2, 3), (2, 3, 1, 2), (2, 2, 2, 2, 2),
                                   (1, 3, 2, 2, 4), (3, 2, 3, 2, 3)])
@pytest.mark.parametrize("with_op", [False, True])
def test_double_layer_matches_oracle(tn, shape, with_op):
    import torch
    rng = np.random.default_rng(sum(shape) + 7 * with_op)
    A = rng.standard_normal(shape)
    d = shape[0]
    op = rng.standard_normal((d, d)) if with_op else None
    want = Q.double_layer(A, op)
    E = torch.empty(want.shape, dtype=torch.float64, device="cuda")
    print(f"[gpu] double layer {shape} op={with_op}", flush=True)
    tn.tn_double_layer([(dev(A), dev(op) if with_op else None, E)])
    torch.cuda.synchronize()
    got = E.cpu().numpy()
    scale = max(1.0, float(np.max(np.abs(want))))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14 * scale)


def test_double_layer_many_sites_one_call(tn):
    # more sites than one launch holds, different shapes mixed
    import torch
    rng = np.random.default_rng(3)
    shapes = [(2,) + tuple(int(x) for x in rng.integers(1, 4, size=int(rng.integers(0, 5))))
              for _ in range(131)]
    As = [rng.standard_normal(s) for s in shapes]
    ops = [rng.standard_normal((2, 2)) if i % 3 else None for i in range(len(As))]
    Es = [torch.empty(Q.double_layer(A).shape, dtype=torch.float64, device="cuda") for A in As]
    tn.tn_double_layer([(dev(A), dev(o) if o is not None else None, E)
                        for A, o, E in zip(As, ops, Es)])
    torch.cuda.synchronize()
    for A, o, E in zip(As, ops, Es):
        want = Q.double_layer(A, o)
        np.testing.assert_allclose(E.cpu().numpy(), want, rtol=0,
                                   atol=1e-14 * max(1.0, float(np.max(np.abs(want)))))


@pytest.mark.parametrize("rows,cols,chi,seed", [(3, 3, 2, 0), (4, 4, 2, 1), (3, 5, 2, 2),
                                                (6, 6, 2, 3), (4, 4, 3, 4)])
def test_observable_set_matches_oracle(tn, rows, cols, chi, seed):
    from paper_1908_08553_amd.peps import ObservableSet
    peps = li.peps(rows, cols, chi, seed)
    want = Q.expectation_values(peps, rows, cols, SX, SZ, P.COLSWEEP)
    obs = ObservableSet(rows, cols, chi, precision="f64")
    print(f"[gpu] observables {rows}x{cols} chi={chi}: {obs.count} networks", flush=True)
    got = obs.run([dev(A) for A in peps], dev(SX), dev(SZ))
    obs.close()
    norm = got["results"][0]
    assert norm.status == 0 and norm.sign == want["norm"].sign
    assert abs(norm.log_abs - want["norm"].log_abs) <= 1e-12
    for key in ("mx", "mz", "czz"):
        np.testing.assert_allclose(got[key], want[key], rtol=0, atol=1e-11, err_msg=key)


def test_observable_set_repeatable(tn):
    from paper_1908_08553_amd.peps import ObservableSet
    peps = [dev(A) for A in li.peps(5, 5, 2, 9)]
    obs = ObservableSet(5, 5, 2, precision="f64")
    a = obs.run(peps, dev(SX), dev(SZ))
    b = obs.run(peps, dev(SX), dev(SZ))
    obs.close()
    assert a["mx"] == b["mx"] and a["mz"] == b["mz"] and a["czz"] == b["czz"]


def test_observable_set_tuned_matches_default(tn, tmp_path, monkeypatch):
    # the autotuner times 256/512/1024-thread workgroups on these networks and
    # raises if any of them changes a result; the tuned batch must then agree
    # with the default one bit for bit
    from paper_1908_08553_amd.peps import ObservableSet
    monkeypatch.setenv("TN_TUNE_CACHE", str(tmp_path / "tune.json"))
    peps = [dev(A) for A in li.peps(4, 4, 2, 13)]
    obs = ObservableSet(4, 4, 2, precision="f64")
    a = obs.run(peps, dev(SX), dev(SZ))
    report = obs.tune(peps, dev(SX), dev(SZ), reps=2)
    b = obs.run(peps, dev(SX), dev(SZ))
    obs.close()
    assert report["best"] in (256, 512, 1024)
    assert a["mx"] == b["mx"] and a["mz"] == b["mz"] and a["czz"] == b["czz"]


@pytest.mark.parametrize("rows,cols,chi,seed", [(3, 3, 2, 0), (4, 4, 2, 1), (3, 5, 2, 2),
                                                (5, 3, 2, 5), (6, 6, 2, 3), (4, 4, 3, 4)])
def test_observable_set_env_mode_matches_oracle(tn, rows, cols, chi, seed):
    # cached column environments: each observable network absorbs the one or
    # two columns of its operator sites and closes against the right
    # environment; same values as full contractions
    from paper_1908_08553_amd.peps import ObservableSet
    peps = li.peps(rows, cols, chi, seed)
    want = Q.expectation_values(peps, rows, cols, SX, SZ, P.COLSWEEP)
    obs = ObservableSet(rows, cols, chi, precision="f64", mode="env")
    print(f"[gpu] env observables {rows}x{cols} chi={chi}: {obs.count} networks", flush=True)
    got = obs.run([dev(A) for A in peps], dev(SX), dev(SZ))
    again = obs.run([dev(A) for A in peps], dev(SX), dev(SZ))
    obs.close()
    norm = got["results"][0]
    assert norm.status == 0 and norm.sign == want["norm"].sign
    assert abs(norm.log_abs - want["norm"].log_abs) <= 1e-12
    for key in ("mx", "mz", "czz"):
        np.testing.assert_allclose(got[key], want[key], rtol=0, atol=1e-11, err_msg=key)
        assert got[key] == again[key]


def test_auto_mode_choice_and_agreement_8x8(tn):
    # mode "auto" takes the batch for 6 x 6 (boundaries of 4^7 entries) and
    # cached environments (with site environments) for 8 x 8 (4^9); at 8 x 8
    # both modes give the same observables
    from paper_1908_08553_amd.peps import ObservableSet
    small = ObservableSet(6, 6, 2)
    assert small.mode == "batch"
    small.close()
    # the shorter side decides: a 12 x 3 lattice sweeps 4^4-entry boundaries
    # in the batch; a 9 x 8 one takes environments, transposed
    tall = ObservableSet(12, 3, 2)
    assert tall.mode == "batch"
    tall.close()
    big = ObservableSet(9, 8, 2)
    assert big.mode == "env" and big.transposed
    big.close()
    peps = [dev(A) for A in li.peps(8, 8, 2, 17)]
    auto = ObservableSet(8, 8, 2)
    assert auto.mode == "env"
    print("[gpu] 8x8 observables, environments", flush=True)
    a = auto.run(peps, dev(SX), dev(SZ))
    auto.close()
    batch = ObservableSet(8, 8, 2, mode="batch")
    print("[gpu] 8x8 observables, batch", flush=True)
    b = batch.run(peps, dev(SX), dev(SZ))
    batch.close()
    na, nb = a["results"][0], b["results"][0]
    assert na.sign == nb.sign and abs(na.log_abs - nb.log_abs) <= 1e-12
    for key in ("mx", "mz", "czz"):
        np.testing.assert_allclose(a[key], b[key], rtol=0, atol=1e-12, err_msg=key)


@pytest.mark.parametrize("rows,cols", [(7, 3), (6, 4)])
def test_tall_lattice_environments_transposed(tn, rows, cols):
    # environments sweep the transposed lattice (legs laid out by the
    # double-layer kernel's leg permutation); observables against the oracle
    from paper_1908_08553_amd.peps import ObservableSet
    peps = li.peps(rows, cols, 2, rows * cols)
    want = Q.expectation_values(peps, rows, cols, SX, SZ, P.COLSWEEP)
    obs = ObservableSet(rows, cols, 2, precision="f64", mode="env")
    assert obs.transposed
    print(f"[gpu] env observables {rows}x{cols}, transposed", flush=True)
    got = obs.run([dev(A) for A in peps], dev(SX), dev(SZ))
    obs.close()
    norm = got["results"][0]
    assert norm.status == 0 and norm.sign == want["norm"].sign
    assert abs(norm.log_abs - want["norm"].log_abs) <= 1e-12
    for key in ("mx", "mz", "czz"):
        np.testing.assert_allclose(got[key], want[key], rtol=0, atol=1e-11, err_msg=key)

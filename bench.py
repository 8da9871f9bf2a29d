"""Benchmark: exact 12x12 D=4 planar-lattice contraction on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-legs]
                    [--no-batch] [--no-serve] [--leg NAME ...] [--calibrate]
    python bench.py --summarize-stats DIR OUT.txt   (rocprofv3 --stats CSV -> text)
    python bench.py --summarize-traffic FETCH_DIR WRITE_DIR OUT.json
    python bench.py --summarize-mfma DIR OUT.txt   (rocprofv3 --pmc MFMA/CU busy -> text)
                                                    (rocprofv3 --pmc CSVs -> traffic)

One step = one full contraction through the C ABI -- site staging, every
pairwise absorption with its per-column exact rescale, the quadrant ring
products with the closing dot, and the result copy -- of a 12x12, D=4
network with i.i.d. uniform[0,1) entries (seed 0) already resident in HBM,
in the order the paper's heuristic picks (smallest bottleneck: the quadrant
split for even L), in FP64 as the paper computes (DGEMM, §6).  `value` is
the plan's algorithmic flops per second.  Prints ONE JSON line; FP32 and
split BF16x3 on the same network (each with its |d log Z| against the FP64
oracle), the column sweep, the 10x10 configuration, the 512-lattice batch
and the served Poisson stream ride along under "legs".
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# dense peaks; split BF16x3 issues three bf16 products per algorithmic one
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16x3": 2500.0 / 3.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_stats():
    from paper_1908_08553_amd import tn_profile_read
    return tn_profile_read()


def pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(round(q * (len(xs) - 1))))]


def run_leg(tn, torch, rows, cols, D, kind, seed, order, prec, steps, warmup, profile=False):
    import lattice_inputs as li
    # the inputs stay resident; their pointer table is built once, as a C caller would
    sites = tn.prepare_sites(tn.device_sites(li.make(kind, rows, cols, D, seed, K=0.44)))
    plan = tn.tn_plan_grid(rows, cols, D, order=order)
    info = plan.info()
    pidx = {"f64": 0, "f32": 1, "bf16x3": 2}[prec]
    ws = tn.workspace_for(plan, pidx)
    stream = torch.cuda.current_stream()
    res = None
    for _ in range(warmup):
        res = tn.contract_grid(plan, sites, prec, ws, stream)
    # timed pass: no per-launch events
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        res = tn.contract_grid(plan, sites, prec, ws, stream)
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ks = None
    if profile:
        # a second pass of the same steps with every launch bracketed by HIP
        # events on its own stream: per-kernel durations for the roofline
        tn.tn_profile_enable(True)
        for _ in range(steps):
            tn.contract_grid(plan, sites, prec, ws, stream)
        torch.cuda.synchronize()
        ks = kernel_stats()
        tn.tn_profile_enable(False)
    return {"rows": rows, "cols": cols, "D": D, "inputs": kind, "order": info["order"],
            "quad": list(info["quad"]), "precision": prec, "ms": 1e3 * dt / steps,
            "p50_ms": 1e3 * pct(lat, 0.5), "p99_ms": 1e3 * pct(lat, 0.99),
            "gflops": info["flops"] / (dt / steps) / 1e9,
            "contractions_per_s": steps / dt, "flops": info["flops"],
            "peak_entries": info["peak_entries"], "hbm_bytes": info["hbm_bytes"][pidx],
            "log_abs": res.log_abs, "sign": res.sign, "kernels": ks}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_12x12_D4.json")


def measured_traffic(key):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) that
    rocprofv3 recorded for `key` = "<workload>:<kernel>", or None when there is
    no record or a listed kernel source has changed since it was taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)["kernels"].get(key)
    except (OSError, ValueError, KeyError):
        return None
    if not rec:
        return None
    for path, digest in rec["sources_sha256"].items():
        try:
            with open(os.path.join(ROOT, path), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != digest:
                    return None
        except OSError:
            return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def roofline(ks, prec, workload=None):
    """Dominant kernel (most GPU time) of a profiled leg against its bound;
    `traffic` from the committed rocprofv3 counters of that kernel on
    `workload` ("quadrant" / "sweep" of the 12x12 D=4 uniform network)."""
    if not ks:
        return None
    dom = max(ks, key=lambda k: k["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    share = dom["total_ms"] / sum(k["total_ms"] for k in ks)
    traffic = measured_traffic(f"{workload}:{dom['name']}") if workload else None
    alg_bytes = dom["bytes"] / dom["launches"]
    extra = {"launches": dom["launches"], "avg_ms": avg_ms, "share_of_gpu_time": share,
             "algorithmic_bytes_per_launch": alg_bytes}
    # bound: the kernel's algorithmic intensity against the ridge point of its
    # arithmetic (peak flops / 8 TB/s)
    dt = "f64" if dom["name"].endswith("f64") else prec
    peak = PEAK_TFLOPS[dt]
    intensity = dom["flops"] / dom["bytes"] if dom["bytes"] else float("inf")
    extra["flops_per_byte"] = intensity
    if intensity >= peak * 1e12 / (PEAK_HBM_GBS * 1e9):
        ach = dom["flops"] / dom["launches"] / (avg_ms * 1e-3) / 1e12
        return {"kernel": dom["name"], "bound": "mfma", "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "traffic": traffic, **extra}
    ach = alg_bytes / (avg_ms * 1e-3) / 1e9
    return {"kernel": dom["name"], "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": ach / PEAK_HBM_GBS, "traffic": traffic, **extra}


def copy_calibration(torch, mib=256, reps=20):
    """A plain device-to-device copy of `mib` MiB (torch's copy kernel): the
    achievable HBM rate, and the reference dispatch for scaling rocprofv3's
    FETCH_SIZE / WRITE_SIZE counters."""
    n = mib * (1 << 20) // 4
    x = torch.rand(n, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return {"bytes_per_launch": 2 * n * 4, "avg_ms": ms, "gbs": 2 * n * 4 / (ms * 1e-3) / 1e9}


def batch_leg(tn, torch, n=512, seed=2024, reps=20):
    """512 independent lattices (Lh, Lw ~ U{4..8}, D ~ U{2,3,4}, uniform[0,1))
    in one graph-replayed launch, FP32; workgroup size from the autotuner."""
    import lattice_inputs as li
    from paper_1908_08553_amd import autotune
    mix = li.batch_mix(n, seed)
    plans = [tn.tn_plan_grid(r, c, D, order=tn.TN_ORDER_SWEEP_AUTO) for r, c, D, _ in mix]
    sites = [tn.device_sites(s) for _, _, _, s in mix]
    flops = sum(p.info()["flops"] for p in plans)
    tuned = autotune.tune_batch(plans, sites, "f32", reps=5)
    b = autotune.tuned_batch(plans, "f32")
    prep = b.prepare(sites)   # pointer tables of the resident inputs, built once
    b.run(None, prepared=prep)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = b.run(None, prepared=prep)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    b.close()
    # the same lattices one tn_contract_grid call at a time
    ws = torch.empty(max(max(p.info()["workspace_bytes"][1] for p in plans), 256),
                     dtype=torch.uint8, device="cuda")
    psites = [tn.prepare_sites(s) for s in sites]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    single = [tn.contract_grid(p, s, "f32", ws) for p, s in zip(plans, psites)]
    torch.cuda.synchronize()
    dt_seq = time.perf_counter() - t0
    # one launch per step: the batch kernel's own per-step arithmetic, so the
    # results must agree bit for bit (fused column chunks sum in another order)
    tn.tn_set_option(tn.TN_OPT_FUSE_STEPS, 0)
    try:
        plain = [tn.contract_grid(p, s, "f32", ws) for p, s in zip(plans, sites)]
    finally:
        tn.tn_set_option(tn.TN_OPT_FUSE_STEPS, 2)
    same = all((a.mantissa, a.exp2_sum) == (c.mantissa, c.exp2_sum) for a, c in zip(res, plain))
    rel = max(abs(a.log_abs - c.log_abs) / max(1.0, abs(c.log_abs)) for a, c in zip(res, single))
    return {"lattices": n, "precision": "f32", "ms": 1e3 * dt,
            "contractions_per_s": n / dt, "gflops": flops / dt / 1e9,
            "flops_per_batch": flops, "tuned_threads": tuned["best"],
            "tuned_split": tuned["split"],
            "tuning_ms": {str(k): v for k, v in tuned["ms"].items()},
            "sequential_ms": 1e3 * dt_seq, "sequential_contractions_per_s": n / dt_seq,
            "speedup_vs_sequential": dt_seq / dt, "bitwise_equal_to_single_step_launches": same,
            "max_rel_dlogz_vs_fused_single": rel,
            "all_finite": all(r.status == 0 for r in res)}


def peps_leg(tn, torch, rows=6, cols=6, chi=2, seed=3, reps=10):
    """One observable evaluation of a real rows x cols PEPS (bond dimension chi,
    spin 1/2, N(0,1) tensors): the norm, m^x and m^z at every site and c_ij on
    every nearest-neighbour pair, 1 + 2 L^2 + 2 L (L-1) networks of bond
    dimension chi^2, FP64: double-layer sites in one call, all networks in one
    batch launch, ratios in the library."""
    import lattice_inputs as li
    from paper_1908_08553_amd.peps import ObservableSet
    sx, sz = (torch.as_tensor(m, dtype=torch.float64).cuda() for m in li.spin_half())
    peps = [torch.as_tensor(a, dtype=torch.float64).cuda() for a in li.peps(rows, cols, chi, seed)]
    obs = ObservableSet(rows, cols, chi, precision="f64")
    tuned = obs.tune(peps, sx, sz)
    out = obs.run(peps, sx, sz)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = obs.run(peps, sx, sz)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    flops = obs.count * obs.plan.info()["flops"]
    obs.close()
    return {"rows": rows, "cols": cols, "chi": chi, "precision": "f64", "networks": obs.count,
            "ms_per_evaluation": 1e3 * dt, "networks_per_s": obs.count / dt,
            "gflops": flops / dt / 1e9, "tuned_threads": tuned["best"],
            "tuning_ms": {str(k): v for k, v in tuned["ms"].items()},
            "norm_log_abs": out["results"][0].log_abs,
            "mean_mx": sum(out["mx"]) / len(out["mx"]),
            "all_finite": all(r.status == 0 for r in out["results"])}


def peps_env_leg(tn, torch, rows=10, cols=10, chi=2, seed=3, reps=5):
    """The same evaluation on a 10 x 10 PEPS (381 networks of bond dimension
    4, boundaries of 4^11 entries) with cached column environments: the norm
    network's left and right column sweeps once, then each network absorbs
    only the columns of its operator sites and closes against the right
    environment.  Baseline: the same networks as full column sweeps one after
    another (one full sweep timed, times the network count)."""
    import lattice_inputs as li
    from paper_1908_08553_amd.peps import ObservableSet
    sx, sz = (torch.as_tensor(m, dtype=torch.float64).cuda() for m in li.spin_half())
    peps = [torch.as_tensor(a, dtype=torch.float64).cuda() for a in li.peps(rows, cols, chi, seed)]
    obs = ObservableSet(rows, cols, chi, precision="f64", mode="env")
    out = obs.run(peps, sx, sz)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        out = obs.run(peps, sx, sz)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    plan = tn.tn_plan_grid(rows, cols, chi * chi, order=tn.TN_ORDER_COLSWEEP)
    norm_sites = tn.prepare_sites(obs.E[0])
    ws = tn.workspace_for(plan, tn.TN_PREC_F64)
    full = tn.contract_grid(plan, norm_sites, "f64", workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        tn.contract_grid(plan, norm_sites, "f64", workspace=ws)
    torch.cuda.synchronize()
    t_full = (time.perf_counter() - t0) / reps
    n = obs.count
    obs.close()
    return {"rows": rows, "cols": cols, "chi": chi, "precision": "f64", "networks": n,
            "mode": "env", "ms_per_evaluation": 1e3 * dt, "networks_per_s": n / dt,
            "full_sweep_ms": 1e3 * t_full, "sequential_full_sweeps_ms": 1e3 * t_full * n,
            "speedup_vs_full_sweeps": t_full * n / dt,
            "norm_matches_full_sweep": (out["results"][0].mantissa, out["results"][0].exp2_sum)
            == (full.mantissa, full.exp2_sum),
            "all_finite": all(r.status == 0 for r in out["results"])}


def orders_leg(tn, torch, reps=5):
    """The paper's order comparison (§6, Fig. 6: row scheme against quadrant
    scheme, 5 <= L <= 10): FP64 contractions of L x L networks (uniform
    entries, seed 0) in the row scheme, the quadrant order and the column
    sweep, at D = 2 for L = 5..10 and D = 4 for L = 5..8.  A plan is run only
    when its intermediate storage fits the free device memory
    (tn_plan_grid_budget); the row scheme stops fitting first."""
    import lattice_inputs as li
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free) // 8          # float64 entries
    out = {}
    for D, Ls in ((2, range(5, 11)), (4, range(5, 9))):
        for L in Ls:
            row = {}
            sites = None
            for name, order in (("rows", tn.TN_ORDER_ROWS), ("quadrant", tn.TN_ORDER_QUADRANT),
                                ("sweep", tn.TN_ORDER_COLSWEEP)):
                try:
                    plan = tn.tn_plan_grid(L, L, D, order=order, budget=budget)
                except tn.TnError as e:
                    if e.status not in (tn.TN_ENOMEM, tn.TN_EOVERFLOW):
                        raise
                    row[name] = {"fits": False, "peak_entries": None}
                    continue
                if sites is None:
                    sites = tn.prepare_sites(tn.device_sites(li.uniform(L, L, D, 0)))
                info = plan.info()
                ws = tn.workspace_for(plan, tn.TN_PREC_F64)
                r = tn.contract_grid(plan, sites, "f64", ws)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    r = tn.contract_grid(plan, sites, "f64", ws)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / reps
                del ws
                row[name] = {"fits": True, "ms": 1e3 * dt, "gflops": info["flops"] / dt / 1e9,
                             "peak_entries": info["peak_entries"],
                             "buffer_entries": info["buffer_entries"], "log_abs": r.log_abs}
            q = row["quadrant"]
            if row["rows"]["fits"]:
                row["rows_over_quadrant_time"] = row["rows"]["ms"] / q["ms"]
                row["abs_dlogz_rows_vs_quadrant"] = abs(row["rows"]["log_abs"] - q["log_abs"])
            out[f"L{L}_D{D}"] = row
    return out


def ite_leg(tn, torch, steps=10):
    """Imaginary-time evolution (§5) on the paper's Fig. 5 workload: L x L
    lattices, 5 <= L <= 8, chi = 2, Gamma = J = 1, eps = 0.01: milliseconds
    per Trotter step (one-body gates, pair gates with their SVDs, three
    normalisations) and per energy evaluation (1 + 2L^2 + 2L(L-1) networks of
    bond dimension 4), after `steps` warm steps.  Also the 2 x 2 and 3 x 3
    energies of Fig. 4 (chi = 2, tau = 3, 200 steps) next to exact
    diagonalisation, which the CPU leg supplies."""
    out = {}
    for L in range(5, 9):
        ite = tn.Ite(L, L, 2, 1.0, 1.0, 0.01)
        ite.step(0.03, steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ite.step(0.03, steps)
        torch.cuda.synchronize()
        t_step = (time.perf_counter() - t0) / steps
        ite.energy()
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            e = ite.energy()[0]
        t_e = (time.perf_counter() - t0) / reps
        ite.close()
        out[f"L{L}"] = {"ms_per_step": 1e3 * t_step, "ms_per_energy": 1e3 * t_e,
                        "networks_per_energy": 1 + 2 * L * L + 2 * L * (L - 1),
                        "energy_per_site": e / (L * L)}
    fig4 = {}
    for L in (2, 3):
        for G in (0.5, 1.0, 2.0):
            ite = tn.Ite(L, L, 2, 1.0, G, 1e-10)
            t0 = time.perf_counter()
            es = ite.evolve(3.0, 200, energy_every=2)
            torch.cuda.synchronize()
            fig4[f"{L}x{L}_G{G}"] = {"energy_per_site": es[-1][1] / (L * L),
                                     "s_for_200_steps_with_energies": time.perf_counter() - t0}
            ite.close()
    out["fig4"] = fig4
    return out


def served_leg(tn, torch, n=2000, seed=5):
    """Poisson stream: L ~ U{4..13} square Ising lattices, D ~ U{2,4} (D=4 is
    the two-replica network), tag ~ U{FP64, BF16x3}, beta*J ~ U[0.1, 0.8],
    heuristic order.  First the plain FP64 GPU path runs every request back
    to back (rate mu).  Then the server takes every request at once
    (saturation), first all tagged FP64 (results bitwise those of the serial
    path), then as tagged; then the Poisson stream at arrival rates 0.5 mu
    and 0.9 mu.  Accuracy: |d log Z| against the FP64 serial path."""
    import numpy as np
    import lattice_inputs as li
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n):
        L = int(rng.integers(4, 14))
        D = int(rng.choice([2, 4]))
        tag = str(rng.choice(["f64", "bf16x3"]))
        K = float(rng.uniform(0.1, 0.8))
        sites = li.ising(L, L, K) if D == 2 else li.ising_d4(L, L, K)
        reqs.append((L, D, tag, sites))
    plans = [tn.tn_plan_grid(L, L, D, order=tn.TN_ORDER_HEURISTIC) for L, D, _, _ in reqs]
    ws = torch.empty(max(p.info()["workspace_bytes"][0] for p in plans), dtype=torch.uint8,
                     device="cuda")
    tn.contract_grid(plans[0], reqs[0][3], "f64", ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ref = [tn.contract_grid(p, r[3], "f64", ws) for p, r in zip(plans, reqs)]
    t_serial = time.perf_counter() - t0
    del ws
    mu = n / t_serial
    out = {"requests": n, "fp64_serial_s": t_serial, "fp64_serial_contractions_per_s": mu,
           "mean_flops": sum(p.info()["flops"] for p in plans) / n}
    # one slot per hardware queue left beside the caller's stream
    srv = tn.Server(24 << 30, max_slots=3, queue_depth=n + 8)

    def closed_loop(tags):
        """Every request submitted at t = 0 (saturation): contractions/s,
        latency, and |d log Z| per precision against the FP64 serial path."""
        tickets = []
        start = time.perf_counter()
        for (L, D, _, sites), tag in zip(reqs, tags):
            tickets.append(srv.submit(L, L, sites, D=D, precision=tag))
        res = [srv.wait(t) for t in tickets]
        wall = time.perf_counter() - start
        lat = [(tm[2] - tm[0]) * 1e-6 for _, tm in res]
        err = {}
        same = True
        for k, ((r, _), tag) in enumerate(zip(res, tags)):
            err[tag] = max(err.get(tag, 0.0), abs(r.log_abs - ref[k].log_abs))
            if tag == "f64":
                same = same and (r.mantissa, r.exp2_sum) == (ref[k].mantissa, ref[k].exp2_sum)
        return {"contractions_per_s": n / wall, "wall_s": wall, "p50_ms": pct(lat, 0.5),
                "p99_ms": pct(lat, 0.99), "max_abs_dlogz_vs_fp64_serial": err,
                "fp64_results_bitwise_equal_to_serial": same,
                "speedup_vs_fp64_serial": (n / wall) / mu,
                "peak_active": srv.stats()["peak_active"]}

    # the same requests, all FP64: equal (bitwise) accuracy to the serial path
    out["saturation_all_f64"] = closed_loop(["f64"] * n)
    # the mix as tagged (half FP64, half split BF16x3)
    out["saturation_mixed"] = closed_loop([r[2] for r in reqs])
    for frac in (0.5, 0.9):
        lam = frac * mu
        arrivals = np.cumsum(rng.exponential(1.0 / lam, size=n))
        pending = {}
        done = {}
        start = time.perf_counter()
        i = 0
        while len(done) < n:
            now = time.perf_counter() - start
            while i < n and arrivals[i] <= now:
                L, D, tag, sites = reqs[i]
                pending[srv.submit(L, L, sites, D=D, precision=tag)] = i
                i += 1
            for t in list(pending):
                st, res, times = srv.poll(t)
                if st != tn.TN_PENDING:
                    done[pending.pop(t)] = (res, times)
            time.sleep(100e-6)
        lat = [(done[k][1][2] - done[k][1][0]) * 1e-6 for k in range(n)]
        span = (max(done[k][1][2] for k in range(n)) - min(done[k][1][0] for k in range(n))) * 1e-9
        err = {"f64": 0.0, "bf16x3": 0.0}
        for k in range(n):
            d = abs(done[k][0].log_abs - ref[k].log_abs)
            err[reqs[k][2]] = max(err[reqs[k][2]], d)
        out[f"rate_{frac}"] = {"arrival_per_s": lam, "p50_ms": pct(lat, 0.5),
                               "p99_ms": pct(lat, 0.99), "max_ms": max(lat),
                               "contractions_per_s": n / span,
                               "max_abs_dlogz_vs_fp64_serial": err,
                               "peak_active": srv.stats()["peak_active"]}
    srv.close()
    return out


def cpu_baseline():
    """The FP64 oracle, unchanged, contracting the whole headline network
    (12x12, D=4, uniform seed 0, the heuristic's quadrant plan); its log|Z|
    is also the accuracy reference of every leg on that network.  The
    two-replica Ising leg's reference is the oracle's row transfer matrix
    (untimed, milliseconds)."""
    import lattice_inputs as li
    from oracle import contract as OC
    from oracle import network as ON
    from oracle import plan as OP
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    sites = li.uniform(12, 12, 4, 0)
    plan = OP.plan_grid(12, 12, 4, order=OP.HEURISTIC)
    t = time.perf_counter()
    r = OC.contract(sites, plan)
    dt = time.perf_counter() - t
    from oracle import ite as OI
    ed = {f"{L}x{L}_G{G}": OI.ground_energy(L, L, 1.0, G) / (L * L)
          for L in (2, 3) for G in (0.5, 1.0, 2.0)}
    return {"value": plan.flops / dt / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"one complete 12x12 D=4 contraction (quadrant plan, {plan.flops:.3e} "
                      f"flops), FP64 numpy/OpenBLAS, {dt:.1f} s",
            "log_abs": r.log_abs, "sign": r.sign,
            "ising12_d4_log_abs_transfer_matrix": 2 * ON.transfer_log_z(12, 12, 0.44),
            "ed_energy_per_site": ed}


LEGS = [("quad12_f32", 12, 12, 4, "uniform", 1, "f32"),
        ("quad12_bf16x3", 12, 12, 4, "uniform", 1, "bf16x3"),
        ("sweep12_f64", 12, 12, 4, "uniform", 0, "f64"),
        ("sweep12_f32", 12, 12, 4, "uniform", 0, "f32"),
        ("sweep12_bf16x3", 12, 12, 4, "uniform", 0, "bf16x3"),
        ("ising12_d4_quad_f64", 12, 12, 4, "ising", 1, "f64"),
        ("ising12_d4_quad_f32", 12, 12, 4, "ising", 1, "f32"),
        ("ising12_d4_quad_bf16x3", 12, 12, 4, "ising", 1, "bf16x3"),
        ("sweep10_f64_normal", 10, 10, 4, "normal", 0, "f64"),
        ("quad10_f64_normal", 10, 10, 4, "normal", 1, "f64"),
        ("quad10_f32", 10, 10, 4, "uniform", 1, "f32"),
        ("quad10_bf16x3", 10, 10, 4, "uniform", 1, "bf16x3")]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-legs", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--leg", action="append", default=None,
                    help="run only the named leg(s) besides the headline (repeatable)")
    ap.add_argument("--calibrate", action="store_true",
                    help="also time a plain 256 MiB device copy")
    ap.add_argument("--summarize-stats", nargs=2, metavar=("DIR", "OUT"), default=None,
                    help="reduce a rocprofv3 --stats CSV directory to a text summary")
    ap.add_argument("--summarize-traffic", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "OUT"),
                    default=None, help="reduce two rocprofv3 --pmc runs (FETCH_SIZE, "
                    "WRITE_SIZE) with --calibrate to per-launch HBM bytes")
    ap.add_argument("--summarize-mfma", nargs=2, metavar=("DIR", "OUT"), default=None,
                    help="reduce a rocprofv3 --pmc run of SQ_VALU_MFMA_BUSY_CYCLES "
                    "SQ_BUSY_CU_CYCLES GRBM_GUI_ACTIVE to per-kernel busy fractions")
    ap.add_argument("--chunk-schedule", type=int, default=None,
                    help="TN_OPT_CHUNK_SCHEDULE for every contraction of the run")
    ap.add_argument("--command", default="", help="command line recorded in a summary")
    ap.add_argument("--workload", default="quadrant",
                    help="workload key of a traffic record (quadrant / sweep)")
    args = ap.parse_args()
    if args.summarize_stats or args.summarize_traffic or args.summarize_mfma:
        from paper_1908_08553_amd import profsum
        if args.summarize_stats:
            profsum.write_stats(args.summarize_stats[0], args.summarize_stats[1], args.command)
        if args.summarize_mfma:
            profsum.write_mfma(args.summarize_mfma[0], args.summarize_mfma[1], args.command)
        if args.summarize_traffic:
            profsum.write_traffic(*args.summarize_traffic, command=args.command, root=ROOT,
                                  workload=args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU quadrant partition is a design, not part of this build)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1908_08553_amd as tn
    torch.cuda.set_device(0)
    if args.chunk_schedule is not None:
        tn.tn_set_option(tn.TN_OPT_CHUNK_SCHEDULE, args.chunk_schedule)

    calib = copy_calibration(torch) if args.calibrate else None
    head = run_leg(tn, torch, 12, 12, 4, "uniform", 0, tn.TN_ORDER_HEURISTIC, "f64",
                   args.steps, args.warmup, profile=True)
    log(f"headline: {head['ms']:.3f} ms/contraction, {head['gflops']:.1f} GFLOP/s")
    legs = {}
    if not args.no_legs:
        spec = [x for x in LEGS if not args.leg or x[0] in args.leg]
        for name, r, c, D, kind, order, prec in spec:
            leg = run_leg(tn, torch, r, c, D, kind, 0, order, prec, max(3, args.steps // 4),
                          1, profile=True)
            wl = ({0: "sweep", 1: "quadrant"}.get(order) if (r, c, D, kind) == (12, 12, 4, "uniform")
                  else None)
            leg["roofline"] = roofline(leg["kernels"], prec, wl)
            legs[name] = leg
            log(f"{name}: {leg['ms']:.3f} ms, {leg['gflops']:.1f} GFLOP/s, "
                f"log|Z|={leg['log_abs']:.10f}")
    contraction_legs = list(legs.items())
    def want(name):
        return not args.leg or name in args.leg

    if not args.no_legs:
        if not args.no_batch:
            if want("batch512_f32"):
                legs["batch512_f32"] = batch_leg(tn, torch)
                log(f"batch: {legs['batch512_f32']['contractions_per_s']:.0f} contractions/s")
            if want("peps6_observables_f64"):
                legs["peps6_observables_f64"] = peps_leg(tn, torch)
                log(f"peps observables: {json.dumps(legs['peps6_observables_f64'])}")
            if want("peps10_observables_env_f64"):
                legs["peps10_observables_env_f64"] = peps_env_leg(tn, torch)
                log(f"peps observables, cached environments: "
                    f"{json.dumps(legs['peps10_observables_env_f64'])}")
        if want("orders"):
            legs["orders"] = orders_leg(tn, torch)
            log(f"orders: {json.dumps(legs['orders'])}")
        if want("ite"):
            legs["ite"] = ite_leg(tn, torch)
            log(f"ite: {json.dumps(legs['ite'])}")
        if not args.no_serve and want("served"):
            legs["served"] = served_leg(tn, torch)
            log(f"served: {json.dumps(legs['served'])}")
    # the CPU leg after every GPU leg: its BLAS threads keep the host cores
    # busy for a while after it returns, which would slow the launches of a
    # GPU leg that followed it
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline()
        log(f"cpu baseline: {json.dumps(cpu)}")
    # accuracy: |d log Z| (the relative error in Z) of every 12x12 leg against
    # the FP64 oracle (or, without the CPU leg, against the GPU FP64 headline)
    ref_u = cpu["log_abs"] if cpu else head["log_abs"]
    ref_i = (cpu["ising12_d4_log_abs_transfer_matrix"] if cpu
             else legs.get("ising12_d4_quad_f64", {}).get("log_abs"))
    ref_name = "oracle_f64" if cpu else "gpu_f64"
    for name, leg in contraction_legs + [("headline", head)]:
        ref = {"uniform": ref_u, "ising": ref_i}.get(leg["inputs"]) if leg["rows"] == 12 else None
        if ref is not None:
            leg[f"abs_dlogz_vs_{ref_name}"] = abs(leg["log_abs"] - ref)
    if cpu and "ite" in legs:
        for k, v in legs["ite"]["fig4"].items():
            v["ed_energy_per_site"] = cpu["ed_energy_per_site"][k]
            v["rel_error_vs_ed"] = abs(v["energy_per_site"] - v["ed_energy_per_site"]) / \
                abs(v["ed_energy_per_site"])
    head_kernels = head.pop("kernels")
    line = {
        "metric": "exact contraction GFLOP/s + contractions/s, p50/p99 latency; FP64 vs split-prec",
        "value": head["gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: 12x12 lattice, D=4, i.i.d. uniform[0,1) site tensors, seed 0",
        "config": {"workload": "12x12 square-lattice network, bond dimension 4, minimal-bottleneck "
                               "(quadrant) order, FP64 throughout with exact power-of-two "
                               "rescaling",
                   "rows": 12, "cols": 12, "D": 4, "order": "HEURISTIC -> QUADRANT 6,6",
                   "precision": "f64", "parallelism": "single GPU"},
        "contractions_per_s": head["contractions_per_s"],
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
        "log_abs": head["log_abs"],
        "roofline": roofline(head_kernels, "f64", "quadrant"),
        "kernels": head_kernels,
        "legs": legs,
    }
    for k, v in head.items():
        if k.startswith("abs_dlogz_vs_"):
            line[k] = v
    if calib:
        line["copy_calibration"] = calib
    if cpu:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

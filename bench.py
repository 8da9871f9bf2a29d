"""Benchmark: exact 12x12 D=4 lattice contraction on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-legs]

One step = one full contraction through the C ABI (staging, every pairwise
absorption with its per-column rescale, the final float64 reduction and the
result copy) of a 12x12, D=4 network with i.i.d. uniform[0,1) entries
(seed 0) already resident in HBM.  `value` is the plan's algorithmic flops
per second.  Prints ONE JSON line; the extra legs (other orders and
precisions, the 10x10 FP64 configuration) ride along under "legs".
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
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16x3": 2500.0 / 3.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_stats(tn):
    import ctypes as C
    from paper_1908_08553_amd._native import lib

    class KS(C.Structure):
        _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double),
                    ("bytes", C.c_double), ("flops", C.c_double)]
    n = C.c_int32(0)
    arr = (KS * 64)()
    lib.tn_profile_read.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
    lib.tn_profile_read(C.cast(arr, C.c_void_p), 64, C.byref(n))
    return [{"name": arr[i].name.decode(), "launches": arr[i].launches,
             "total_ms": arr[i].total_ms, "bytes": arr[i].bytes, "flops": arr[i].flops}
            for i in range(min(n.value, 64))]


def run_leg(tn, torch, rows, cols, D, kind, seed, order, prec, steps, warmup, profile=False):
    import lattice_inputs as li
    sites = tn.device_sites(li.make(kind, rows, cols, D, seed, K=0.44))
    plan = tn.tn_plan_grid(rows, cols, D, order=order)
    info = plan.info()
    pidx = {"f64": 0, "f32": 1, "bf16x3": 2}[prec]
    ws = tn.workspace_for(plan, pidx)
    stream = torch.cuda.current_stream()
    res = None
    for _ in range(warmup):
        res = tn.contract_grid(plan, sites, prec, ws, stream)
    torch.cuda.synchronize()
    if profile:
        tn.lib.tn_profile_enable(1)
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        res = tn.contract_grid(plan, sites, prec, ws, stream)
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ks = kernel_stats(tn) if profile else None
    if profile:
        tn.lib.tn_profile_enable(0)
    lat.sort()
    return {"rows": rows, "cols": cols, "D": D, "inputs": kind, "order": info["order"],
            "quad": list(info["quad"]), "precision": prec, "ms": 1e3 * dt / steps,
            "p50_ms": 1e3 * lat[len(lat) // 2], "p99_ms": 1e3 * lat[min(len(lat) - 1, int(0.99 * len(lat)))],
            "gflops": info["flops"] / (dt / steps) / 1e9,
            "contractions_per_s": steps / dt, "flops": info["flops"],
            "peak_entries": info["peak_entries"], "hbm_bytes": info["hbm_bytes"][pidx],
            "log_abs": res.log_abs, "sign": res.sign, "kernels": ks}


def roofline(ks, prec):
    if not ks:
        return None
    dom = max(ks, key=lambda k: k["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    if dom["name"].startswith("ring_mfma") or dom["name"].startswith("ring_valu"):
        ach = dom["flops"] / dom["launches"] / (avg_ms * 1e-3) / 1e12
        peak = PEAK_TFLOPS[prec]
        return {"kernel": dom["name"], "bound": "mfma", "achieved": ach, "peak": peak,
                "unit": "TFLOP/s", "frac": ach / peak, "traffic": None,
                "launches": dom["launches"], "avg_ms": avg_ms,
                "share_of_gpu_time": dom["total_ms"] / sum(k["total_ms"] for k in ks)}
    ach = dom["bytes"] / dom["launches"] / (avg_ms * 1e-3) / 1e9
    return {"kernel": dom["name"], "bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": ach / PEAK_HBM_GBS, "traffic": None,
            "launches": dom["launches"], "avg_ms": avg_ms,
            "share_of_gpu_time": dom["total_ms"] / sum(k["total_ms"] for k in ks)}


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


def cpu_baseline():
    """The FP64 oracle, unchanged, on the first two columns (24 steps) of the
    same 12x12 D=4 column sweep; GFLOP/s from the plan's flops."""
    import lattice_inputs as li
    from oracle import contract as OC
    from oracle import plan as OP
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    sites = li.uniform(12, 12, 4, 0)
    plan = OP.plan_grid(12, 12, 4)
    t = time.perf_counter()
    flops = OC.run_prefix(sites, plan, 24)
    dt = time.perf_counter() - t
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"first 24 of 144 steps (columns 0-1, {flops:.3e} flops) of the 12x12 D=4 "
                      f"column sweep, FP64 numpy/OpenBLAS, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-legs", action="store_true")
    ap.add_argument("--calibrate", action="store_true",
                    help="also time a plain 256 MiB device copy")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU quadrant partition is a design, not part of this build)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1908_08553_amd as tn
    torch.cuda.set_device(0)

    calib = copy_calibration(torch) if args.calibrate else None
    head = run_leg(tn, torch, 12, 12, 4, "uniform", 0, tn.TN_ORDER_COLSWEEP, "f32",
                   args.steps, args.warmup, profile=True)
    log(f"headline: {head['ms']:.3f} ms/contraction, {head['gflops']:.1f} GFLOP/s")
    legs = {}
    if not args.no_legs:
        spec = [("sweep12_bf16x3", 12, 12, 4, "uniform", 0, "f32"),
                ("sweep12_f64", 12, 12, 4, "uniform", 0, "f64"),
                ("quad12_f32", 12, 12, 4, "uniform", 1, "f32"),
                ("quad12_bf16x3", 12, 12, 4, "uniform", 1, "bf16x3"),
                ("quad12_f64", 12, 12, 4, "uniform", 1, "f64"),
                ("sweep10_f64_normal", 10, 10, 4, "normal", 0, "f64"),
                ("quad10_f64_normal", 10, 10, 4, "normal", 1, "f64")]
        spec[0] = ("sweep12_bf16x3", 12, 12, 4, "uniform", 0, "bf16x3")
        for name, r, c, D, kind, order, prec in spec:
            leg = run_leg(tn, torch, r, c, D, kind, 0, order, prec, max(3, args.steps // 4),
                          1, profile=True)
            leg["roofline"] = roofline(leg["kernels"], prec)
            legs[name] = leg
            log(f"{name}: {leg['ms']:.3f} ms, {leg['gflops']:.1f} GFLOP/s, log|Z|={leg['log_abs']:.10f}")
        ref = legs["sweep12_f64"]["log_abs"]
        for name, leg in legs.items():
            if leg["rows"] == 12:
                leg["dlogz_vs_gpu_f64_sweep"] = abs(leg["log_abs"] - ref)
    head_kernels = head.pop("kernels")
    line = {
        "metric": "exact contraction GFLOP/s (12x12 D=4 column sweep)",
        "value": head["gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: 12x12 lattice, D=4, i.i.d. uniform[0,1) site tensors, seed 0",
        "config": {"workload": "12x12 square lattice, bond dim 4, column sweep, FP32 boundary "
                               "with FP64 rescale exponents and FP64 last column",
                   "rows": 12, "cols": 12, "D": 4, "order": "COLSWEEP", "precision": "f32",
                   "parallelism": "single GPU"},
        "contractions_per_s": head["contractions_per_s"],
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
        "log_abs": head["log_abs"],
        "roofline": roofline(head_kernels, "f32"),
        "kernels": head_kernels,
        "legs": legs,
    }
    if calib:
        line["copy_calibration"] = calib
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

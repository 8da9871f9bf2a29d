"""Autotuner for the batched launch graph.

Two launch-shape knobs: the workgroup size of the one-workgroup-per-lattice
path (how many waves sweep one lattice together: more finish a large lattice
sooner, fewer leave room for more lattices per compute unit), and the split,
how many of the costliest lattices instead advance in lock-step with every
step spread over the GPU (each lock-step launch costs a graph node; the
costliest lattices otherwise set the batch's time on one compute unit).
``tune_batch`` times every pair on the caller's own batch (replaying the
captured graph), checks that every candidate returns bit-identical results,
and caches the fastest under a signature of the workload (device name,
precision, sorted lattice shapes and plan costs) in a JSON file:
$TN_TUNE_CACHE, else ``tune_cache.json`` beside this module.
``tuned_batch`` builds a Batch with the cached choice (library defaults when
the workload has not been tuned).
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

from . import _native as N

CANDIDATES: List[int] = [256, 512, 1024]
SPLITS: List[int] = [0, 16, 32, 64, 128, 256, 512]


def cache_path() -> str:
    return os.environ.get("TN_TUNE_CACHE",
                          os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                       "tune_cache.json"))


def signature(plans: Sequence[N.Plan], precision) -> str:
    import torch
    if isinstance(precision, str):
        precision = N._PRECS[precision]
    shapes = sorted((p.info()["peak_entries"], p.info()["flops"], p.info()["n_steps"])
                    for p in plans)
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    h = hashlib.sha1(json.dumps([dev, precision, shapes]).encode()).hexdigest()
    return f"batch:{precision}:{len(plans)}:{h[:16]}"


def _load() -> Dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(d: Dict) -> None:
    path = cache_path()
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned_config(plans, precision) -> Optional[Tuple[int, int]]:
    e = _load().get(signature(plans, precision))
    return (e["threads"], e.get("split", 0)) if e else None


def tune_batch(plans, site_lists, precision="f32", candidates=CANDIDATES, splits=SPLITS,
               reps=5, warmup=1, save=True) -> Dict:
    """Time each (workgroup size, split) pair; returns {"best": threads,
    "split": split, "ms": {"threads/split": median ms}, "signature": ...}."""
    import torch
    timings = {}
    ref = None
    pairs = [(t, s) for s in splits if s <= len(plans) for t in candidates]
    for threads, split in pairs:
        b = N.Batch(plans, precision, threads, split=split)
        prep = b.prepare(site_lists)
        for _ in range(warmup):
            res = b.run(None, prepared=prep)
        if ref is None:
            ref = [(r.mantissa, r.exp2_sum) for r in res]
        elif [(r.mantissa, r.exp2_sum) for r in res] != ref:
            raise RuntimeError(f"workgroup size {threads}, split {split} changed the results")
        ms = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            z = torch.cuda.Event(enable_timing=True)
            a.record()
            b.run(None, prepared=prep)
            z.record()
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(z))
        ms.sort()
        timings[(threads, split)] = ms[len(ms) // 2]
        b.close()
    best = min(timings, key=timings.get)
    sig = signature(plans, precision)
    if save:
        d = _load()
        d[sig] = {"threads": best[0], "split": best[1], "ms": timings[best]}
        _save(d)
    return {"best": best[0], "split": best[1],
            "ms": {f"{t}/{s}": v for (t, s), v in timings.items()}, "signature": sig}


def tuned_batch(plans, precision="f32") -> N.Batch:
    cfg = tuned_config(plans, precision)
    threads, split = cfg if cfg else (0, 0)
    return N.Batch(plans, precision, threads, split=split)

"""Reduce rocprofv3 CSV output to the summaries kept under ``profiles/``.

Measurement tooling, not part of the contraction path: it reads what
``rocprofv3 --kernel-trace --stats --output-format csv`` and
``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` wrote and prints the
per-kernel figures ``bench.py`` uses (``python bench.py --summarize-stats`` /
``--summarize-traffic``).

HBM bytes: FETCH_SIZE and WRITE_SIZE count KiB per dispatch.  Each is scaled
by what the same counter reads for the 256 MiB device copy that
``bench.py --calibrate`` times in the same run (it reads and writes 256 MiB),
so the figures are bytes that crossed the HBM interface per launch.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
from collections import OrderedDict

# library kernel name (the name tn_profile_read reports) -> rocprofv3 kernel
# name pattern, and the sources whose change invalidates a traffic record
KERNELS = OrderedDict([
    ("ring_mfma_f64", (r"ring_mfma<double>", ["paper_1908_08553_amd/csrc/ring_mfma.hip"])),
    ("ring_mfma_f32", (r"ring_mfma_f32_big|ring_mfma<float>",
                       ["paper_1908_08553_amd/csrc/ring_mfma.hip"])),
    ("ring_mfma_bf16x3", (r"ring_bf16x3_nt", ["paper_1908_08553_amd/csrc/ring_mfma.hip"])),
    ("absorb_chunk_reg_f64", (r"absorb_chunk_reg<double, 1,",
                              ["paper_1908_08553_amd/csrc/absorb_chunk_reg.hip",
                               "paper_1908_08553_amd/csrc/absorb_device.hpp"])),
    ("absorb_chunk_reg_f32", (r"absorb_chunk_reg<float, 0,",
                              ["paper_1908_08553_amd/csrc/absorb_chunk_reg.hip",
                               "paper_1908_08553_amd/csrc/absorb_device.hpp"])),
    ("absorb_chunk_reg_bf16x3", (r"absorb_chunk_reg<float, 2,",
                                 ["paper_1908_08553_amd/csrc/absorb_chunk_reg.hip",
                                  "paper_1908_08553_amd/csrc/absorb_device.hpp"])),
    ("absorb_chunk_reg_stream_f64", (r"absorb_chunk_reg_stream<double, 1,",
                                     ["paper_1908_08553_amd/csrc/absorb_chunk_reg.hip",
                                      "paper_1908_08553_amd/csrc/absorb_device.hpp"])),
    ("absorb_chunk_reg_stream_f32", (r"absorb_chunk_reg_stream<float, 0,",
                                     ["paper_1908_08553_amd/csrc/absorb_chunk_reg.hip",
                                      "paper_1908_08553_amd/csrc/absorb_device.hpp"])),
    ("absorb_chunk_reg_stream_bf16x3", (r"absorb_chunk_reg_stream<float, 2,",
                                        ["paper_1908_08553_amd/csrc/absorb_chunk_reg.hip",
                                         "paper_1908_08553_amd/csrc/absorb_device.hpp"])),
    ("absorb_edge_f64", (r"absorb_edge<(double|float), double",
                         ["paper_1908_08553_amd/csrc/absorb_edge.hip",
                          "paper_1908_08553_amd/csrc/absorb_device.hpp"])),
    ("absorb_edge_f32", (r"absorb_edge<float, float",
                         ["paper_1908_08553_amd/csrc/absorb_edge.hip",
                          "paper_1908_08553_amd/csrc/absorb_device.hpp"])),
    ("absorb_chunk_f64", (r"absorb_chunk<double, 1>",
                          ["paper_1908_08553_amd/csrc/absorb_chunk.hip",
                           "paper_1908_08553_amd/csrc/absorb_device.hpp"])),
    ("absorb_chunk_f32", (r"absorb_chunk<float, 0>",
                          ["paper_1908_08553_amd/csrc/absorb_chunk.hip",
                           "paper_1908_08553_amd/csrc/absorb_device.hpp"])),
    ("absorb_chunk_bf16x3", (r"absorb_chunk<float, 2>",
                             ["paper_1908_08553_amd/csrc/absorb_chunk.hip",
                              "paper_1908_08553_amd/csrc/absorb_device.hpp"])),
])
COPY_KERNEL = "__amd_rocclr_copyBuffer"
CALIB_BYTES = 256 << 20


def _find(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits


def _short(name: str) -> str:
    """Kernel name without return type, namespaces and argument list."""
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    name = name.replace("(anonymous namespace)::", "")
    if name.startswith("tn::"):
        name = name[4:]
    cut = name.find("(")
    return name[:cut] if cut > 0 else name


def read_stats(d):
    """[(kernel, calls, total_us, avg_us, pct)] from a kernel_stats CSV."""
    rows = []
    for path in _find(d, "kernel_stats.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                rows.append((_short(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
                             float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    rows.sort(key=lambda x: -x[2])
    return rows


def write_stats(d, out, command=""):
    rows = read_stats(d)
    lines = ["# rocprofv3 kernel statistics", ""]
    if command:
        lines += ["Command (repository root on an MI355X, ROCm 7.2):", "    " + command, ""]
    lines.append(f"{'kernel':60s} {'calls':>7s} {'total_us':>12s} {'avg_us':>10s} {'pct':>6s}")
    for k, n, tot, avg, pct in rows:
        lines.append(f"{k[:60]:60s} {n:7d} {tot:12.1f} {avg:10.2f} {pct:6.2f}")
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    return rows


def read_counter(d, counter):
    """{dispatch id: (kernel, KiB)} for one counter of a --pmc run (values of
    one dispatch summed over the rows it was reported in)."""
    out = {}
    for path in _find(d, "counter_collection.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                key = (path, int(r["Dispatch_Id"]))
                name = _short(r["Kernel_Name"])
                prev = out.get(key, (name, 0.0))[1]
                out[key] = (name, prev + float(r["Counter_Value"]))
    return out


def _scale(vals):
    """bytes per counter unit from the calibration copies (the largest
    copyBuffer dispatches: the 256 MiB copies of --calibrate)."""
    copies = sorted(v for k, v in vals.values() if k.startswith(COPY_KERNEL))
    big = [v for v in copies if v * 1024 > CALIB_BYTES / 8]
    if not big:
        raise ValueError("no 256 MiB calibration copy in the run (use bench.py --calibrate)")
    med = big[len(big) // 2]
    return CALIB_BYTES / (med * 1024.0)


def traffic(fetch_dir, write_dir):
    fetch = read_counter(fetch_dir, "FETCH_SIZE")
    write = read_counter(write_dir, "WRITE_SIZE")
    fs, ws = _scale(fetch), _scale(write)
    res = {"fetch_scale": fs, "write_scale": ws, "kernels": {}}
    for lib, (pat, _) in KERNELS.items():
        rx = re.compile(pat)
        fv = [v for k, v in fetch.values() if rx.search(k)]
        wv = [v for k, v in write.values() if rx.search(k)]
        if fv and wv:
            res["kernels"][lib] = {
                "launches_sampled": min(len(fv), len(wv)),
                "fetch_bytes_per_launch": int(round(sum(fv) / len(fv) * 1024 * fs)),
                "write_bytes_per_launch": int(round(sum(wv) / len(wv) * 1024 * ws))}
    return res


def _sha(root, rel):
    with open(os.path.join(root, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_table(fetch_dir, write_dir):
    """Mean MiB fetched and written per launch of every kernel in the runs."""
    fetch = read_counter(fetch_dir, "FETCH_SIZE")
    write = read_counter(write_dir, "WRITE_SIZE")
    fs, ws = _scale(fetch), _scale(write)
    rows = OrderedDict()
    for k, v in fetch.values():
        rows.setdefault(k, [[], []])[0].append(v * 1024 * fs / 2**20)
    for k, v in write.values():
        rows.setdefault(k, [[], []])[1].append(v * 1024 * ws / 2**20)
    lines = [f"{'kernel':44s} {'n':>5s} {'fetch MiB':>11s} {'write MiB':>11s}"]
    for k, (fv, wv) in rows.items():
        if not fv or not wv:
            continue
        lines.append(f"{k[:44]:44s} {len(fv):5d} {sum(fv) / len(fv):11.2f} {sum(wv) / len(wv):11.2f}")
    return fs, ws, "\n".join(lines) + "\n"


def write_traffic(fetch_dir, write_dir, out, command="", root=".", workload="quadrant"):
    """Merge this run's per-launch bytes into the JSON record ``out`` under
    "<workload>:<kernel>" keys, with the SHA-256 of each kernel's sources;
    print the per-kernel table."""
    fs, ws, table = traffic_table(fetch_dir, write_dir)
    head = (f"# HBM traffic per launch, workload '{workload}' (rocprofv3 FETCH_SIZE and WRITE_SIZE,"
            f" one counter per run)\n\nCommands (repository root on an MI355X, ROCm 7.2):\n"
            f"    {command}\n\nScale: a 256 MiB device copy timed in the same runs reads"
            f" FETCH_SIZE x{fs:.3f} and WRITE_SIZE x{ws:.3f} KiB per counted KiB.\n"
            f"Mean per launch:\n")
    txt = os.path.splitext(out)[0] + f"_{workload}.txt"
    with open(txt, "w") as f:
        f.write(head + table)
    print(head + table, end="")
    t = traffic(fetch_dir, write_dir)
    try:
        with open(out) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {"kernels": {}}
    rec["about"] = ("HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE (two runs), "
                    "each scaled by what the counter reads for a 256 MiB device copy in the same "
                    f"run (FETCH_SIZE x{t['fetch_scale']:.3f}, WRITE_SIZE x{t['write_scale']:.3f}). "
                    "Valid only while the listed kernel sources are unchanged.")
    if command:
        rec.setdefault("commands", [])
        if command not in rec["commands"]:
            rec["commands"].append(command)
    for lib, v in t["kernels"].items():
        v["sources_sha256"] = {p: _sha(root, p) for p in KERNELS[lib][1]}
        rec["kernels"][f"{workload}:{lib}"] = v
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return t


MFMA_COUNTERS = ("SQ_VALU_MFMA_BUSY_CYCLES", "SQ_BUSY_CU_CYCLES", "GRBM_GUI_ACTIVE")


def write_mfma(d, out, command="", min_us=20.0):
    """Matrix-core and CU busy fractions and the shader clock per kernel, from
    one ``rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES SQ_BUSY_CU_CYCLES
    GRBM_GUI_ACTIVE --kernel-trace`` run: cycles = GRBM_GUI_ACTIVE / 8 (the
    counter sums the 8 XCDs), MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (1024
    SIMDs x cycles), CU busy = SQ_BUSY_CU_CYCLES / (256 CUs x cycles), clock =
    cycles / kernel duration.  Kernels averaging under ``min_us`` are left out."""
    per = {}
    for path in _find(d, "counter_collection.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                key = (path, int(r["Dispatch_Id"]))
                e = per.setdefault(key, {"name": _short(r["Kernel_Name"]),
                                         "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"]),
                                         "c": {}})
                e["c"][r["Counter_Name"]] = e["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    agg = OrderedDict()
    for e in per.values():
        a = agg.setdefault(e["name"], [0, 0.0, 0.0, 0.0, 0.0])
        a[0] += 1
        a[1] += e["ns"]
        for i, c in enumerate(MFMA_COUNTERS):
            a[2 + i] += e["c"].get(c, 0.0)
    lines = ["# MFMA utilisation per kernel (rocprofv3 counters)", ""]
    if command:
        lines += ["Command (repository root on an MI355X, ROCm 7.2):", "    " + command, ""]
    lines += ["MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x cycles), CU busy = "
              "SQ_BUSY_CU_CYCLES /",
              "(256 CUs x cycles), cycles = GRBM_GUI_ACTIVE / 8 (the counter sums the 8 XCDs), "
              "clock = cycles",
              "per ns of the kernel-trace duration.  Every dispatch also counts a fixed window "
              "around the",
              "kernel, which lowers both fractions for kernels much shorter than a millisecond; "
              "the counters",
              f"slow the kernels a little.  Kernels of at least {min_us:g} us:", ""]
    rows = []
    for name, (n, ns, mf, cu, gr) in agg.items():
        if n == 0 or ns / n / 1e3 < min_us or gr <= 0:
            continue
        cyc = gr / 8.0
        rows.append((ns, f"{name[:44]:44s} n={n:5d} avg={ns / n / 1e3:9.1f} us  MFMA busy "
                         f"{100 * mf / (1024 * cyc):5.1f} %  CU busy {100 * cu / (256 * cyc):5.1f} %  "
                         f"clock {cyc / ns:4.2f} GHz"))
    rows.sort(key=lambda x: -x[0])
    lines += [r for _, r in rows]
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    print(text, end="")
    return rows

#!/usr/bin/env python3
"""Benchmark: gates/s and fraction of the HBM roofline on the 30-qubit,
depth-40 random circuit (6x5 grid, 10% controlled-U3), fused complex64 path
against the plain complex128 per-gate path, on one MI355X.

A step is one full pass of the simulation over the circuit: re-initialise the
state to |0...0>, apply every gate (the whole circuit), then the FP64 norm
and a PMEASURE over three qubits.  Inputs (the circuit, the state buffer)
are resident before the timed region starts.

Prints one JSON line.  `python bench.py --steps K --warmup W`.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 matrix-core peak
METRIC = "gates/s and % of HBM roofline, 30q depth-40 circuit; fused c64 vs plain c128"

KERNEL_SYMBOL = {  # library kernel class -> kernel function name in rocprof traces
    "dense1": "k_dense1", "dense2": "k_dense_small", "dense3": "k_dense_small",
    "denseN": "k_denseN", "phase": "k_phase", "fused": "k_fused", "tile": "k_tile",
    "reduce": "k_probs", "init": "k_init",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="rqc30_d40")
    p.add_argument("--paths", default="fused_c64,plain_c128")
    p.add_argument("--kmax", type=int, default=0, help="fused block width (0 = library default)")
    p.add_argument("--tile-qubits", type=int, default=0, help="qubits per LDS tile (0 = library default)")
    p.add_argument("--plan", default="greedy", choices=["greedy", "learned", "autotune"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--trajectories", type=int, default=512,
                   help="noisy trajectories in the batched-trajectory measurement (0 = skip)")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-extras", action="store_true",
                   help="skip the partial-amplitude and qubit-remap measurements that follow the main paths")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 4 GiB device-to-device copy (5 times), the reference "
                        "for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE")
    p.add_argument("--no-by-target", action="store_true",
                   help="skip the per-target / per-control bandwidth sweep of single gates")
    p.add_argument("--remap", action="store_true",
                   help="bandwidth of the qubit-remap pack / unpack on a 30-qubit shard (one JSON line)")
    p.add_argument("--partial", action="store_true",
                   help="partial-amplitude mode on a 40-qubit depth-8 circuit (one JSON line)")
    p.add_argument("--traj", action="store_true",
                   help="only the batched-trajectory measurement (512 trajectories, one JSON line)")
    p.add_argument("--single", action="store_true",
                   help="single-amplitude mode on a 60-qubit depth-14 circuit (one JSON line)")
    p.add_argument("--config5", action="store_true",
                   help="34-qubit learned-planner comparison: complex128 reference on 2^20 sampled "
                        "indices, then complex64 learned vs greedy vs unfused")
    p.add_argument("--summarize-profiles", metavar="DIR", default="",
                   help="CPU only: read the rocprofv3 CSV output under DIR (the runs in PROFILE_RUNS) "
                        "and write profiles/traffic.json plus the text summaries")
    return p.parse_args()


# The device sources of the kernels whose counters bench.py reports: the
# tile sweeps and the per-gate kernels of the fused and plain paths.
PROFILED_SOURCES = ("qs_fused.hip", "qs_kernels.hip")


def _code_only(text: bytes) -> bytes:
    """C/C++ source without comments, each run of white space one blank."""
    import re
    t = re.sub(rb"/\*.*?\*/", b" ", text, flags=re.S)
    t = re.sub(rb"//[^\n]*", b" ", t)
    return b" ".join(t.split())


def source_hash(sources=PROFILED_SOURCES, root=None):
    """Hash of the device code of the profiled paths: their .hip sources and
    the headers those include (transitively), comments and layout left out,
    so host-only changes, comment edits and changes to other kernels keep
    stored counter readings valid."""
    import re
    root = root or ROOT
    csrc = os.path.join(root, "paper_2008_07140_amd", "csrc")
    files, todo = set(), [os.path.join(csrc, f) for f in sources]
    while todo:
        f = os.path.normpath(todo.pop())
        if f in files or not os.path.exists(f):
            continue
        files.add(f)
        with open(f) as fh:
            for inc in re.findall(r'#include\s+"([^"]+)"', fh.read()):
                todo.append(os.path.join(os.path.dirname(f), inc))
    h = hashlib.sha256()
    for f in sorted(files):
        h.update(os.path.relpath(f, root).encode())
        with open(f, "rb") as fh:
            h.update(_code_only(fh.read()))
    return h.hexdigest()[:16]


def traffic_key(workload: str, n: int, path_name: str, kernel_class: str) -> str:
    return "%s/n%d/%s/%s" % (workload, n, path_name, kernel_class)


def traffic_for(workload: str, n: int, path_name: str, kernel_class: str, plan: str = "greedy"):
    """HBM bytes per launch measured by rocprofv3 counters for this kernel class
    on this path of this workload, if the counters were taken on the current
    kernel sources (and, for fused paths, under the same plan); None when no
    reading matches exactly."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get(traffic_key(workload, n, path_name, kernel_class))
    if not rec or rec.get("source_hash") != source_hash():
        return None
    if path_name.startswith("fused") and rec.get("plan", "greedy") != plan:
        return None
    return rec.get("bytes_per_launch")


# --- rocprofv3 summaries ------------------------------------------------------
# The counter passes, each a run of its own (rocprofv3 does not split counters
# over passes), from the repository root on the GPU machine:
PROFILE_DIR = "rocprof_out"  # where the runs below write their CSVs and logs
PROFILE_RUNS = [
    ("ktrace", "--kernel-trace --stats",
     "--steps 2 --warmup 1 --no-cpu-baseline --trajectories 0 --no-by-target --no-extras"),
    ("pmc_fetch_fused_c64", "--pmc FETCH_SIZE",
     "--steps 1 --warmup 0 --no-cpu-baseline --trajectories 0 --no-by-target --no-extras --paths fused_c64"),
    ("pmc_write_fused_c64", "--pmc WRITE_SIZE",
     "--steps 1 --warmup 0 --no-cpu-baseline --trajectories 0 --no-by-target --no-extras --paths fused_c64"),
    ("pmc_fetch_plain_c128", "--pmc FETCH_SIZE",
     "--steps 1 --warmup 0 --no-cpu-baseline --trajectories 0 --no-by-target --no-extras --paths plain_c128"),
    ("pmc_write_plain_c128", "--pmc WRITE_SIZE",
     "--steps 1 --warmup 0 --no-cpu-baseline --trajectories 0 --no-by-target --no-extras --paths plain_c128"),
    ("pmc_sq1_fused_c64", "--pmc GRBM_GUI_ACTIVE SQ_VALU_MFMA_BUSY_CYCLES SQ_ACTIVE_INST_VALU SQ_LDS_IDX_ACTIVE "
     "SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_LDS SQ_BUSY_CU_CYCLES SQ_WAVE_CYCLES SQ_WAVES",
     "--steps 1 --warmup 0 --no-cpu-baseline --trajectories 0 --no-by-target --no-extras --paths fused_c64"),
    ("pmc_sq2_fused_c64", "--pmc GRBM_GUI_ACTIVE SQ_INSTS_VALU SQ_INSTS_MFMA SQ_INSTS_LDS SQ_INSTS_VMEM_RD "
     "SQ_INSTS_VMEM_WR SQ_INSTS_SALU SQ_INSTS_VALU_MFMA_MOPS_BF16 SQ_WAIT_INST_LDS",
     "--steps 1 --warmup 0 --no-cpu-baseline --trajectories 0 --no-by-target --no-extras --paths fused_c64"),
    ("remap", "--kernel-trace --stats", "--remap"),
    ("traj", "--kernel-trace --stats", "--traj"),
    ("single", "--kernel-trace --stats", "--single"),
    ("partial", "--kernel-trace --stats", "--partial"),
    ("pmc_fetch_copy", "--pmc FETCH_SIZE", "--copy-calibration"),
    ("pmc_write_copy", "--pmc WRITE_SIZE", "--copy-calibration"),
]


def profile_command(sub, flags, bench_args):
    return ("rocprofv3 %s -f csv -d %s/%s -o run -- python3 bench.py %s > %s/%s.log"
            % (flags, PROFILE_DIR, sub, bench_args, PROFILE_DIR, sub))


def kernel_class_of(name: str):
    """Library kernel class of a rocprofv3 kernel name (None for other kernels)."""
    import re
    m = re.search(r"::(k_[A-Za-z0-9_]+)", name)
    if not m:
        return None
    f = m.group(1)
    if f == "k_tile":
        return "tile"
    if f.startswith("k_dense1"):
        return "dense1"
    if f.startswith("k_phase"):
        return "phase"
    table = {"k_dense_small": "dense_small", "k_denseN": "denseN", "k_phase": "phase", "k_init": "init",
             "k_scale": "other"}
    if f in table:
        return table[f]
    if f.startswith(("k_probs", "k_sum", "k_gather", "k_rdm", "k_zsum")):
        return "reduce"
    return None


def short_kernel(name: str):
    import re
    m = re.search(r"::(k_[A-Za-z0-9_]+(<[^()]*>)?)\(", name)
    return m.group(1) if m else name[:60]


def _csv_rows(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _counter_means(d, sub):
    """{kernel name: (dispatches, mean counter value in KiB)} of one --pmc pass."""
    import glob
    files = glob.glob(os.path.join(d, sub, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit("no counter CSV under %s" % os.path.join(d, sub))
    acc = {}
    for r in _csv_rows(files[0]):
        k = r["Kernel_Name"]
        v = float(r["Counter_Value"])
        c, t = acc.get(k, (0, 0.0))
        acc[k] = (c + 1, t + v)
    return {k: (c, t / c) for k, (c, t) in acc.items()}


def _counters_by_name(d, sub, kernel_class):
    """{counter: mean value per dispatch} over the dispatches of one kernel
    class in a --pmc pass with several counters (one CSV row per dispatch and
    counter)."""
    import glob
    files = glob.glob(os.path.join(d, sub, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        return None
    acc = {}
    for r in _csv_rows(files[0]):
        if kernel_class_of(r["Kernel_Name"]) != kernel_class:
            continue
        c, t = acc.get(r["Counter_Name"], (0, 0.0))
        acc[r["Counter_Name"]] = (c + 1, t + float(r["Counter_Value"]))
    return {k: t / c for k, (c, t) in acc.items()}


def summarize_sq(d, cmds, src, cu=256, simd=1024, xcd=8):
    """profiles/counters_k_tile_rqc30_d40.md: instruction mix and unit
    activity of the tile kernel from two --pmc passes of SQ counters, with
    rocprofv3's own formulas for the derived ratios (CU_NUM = 256,
    SIMD_NUM = 1024 on MI355X).  The counter CSV sums each counter over its
    hardware instances; the formulas take the maximum of GRBM_GUI_ACTIVE over
    the eight XCDs, which run the whole dispatch, so the sum / 8 stands in
    for it."""
    a = _counters_by_name(d, "pmc_sq1_fused_c64", "tile")
    b = _counters_by_name(d, "pmc_sq2_fused_c64", "tile")
    if not a or not b:
        return
    g = a.get("GRBM_GUI_ACTIVE", 0.0) / xcd
    lines = ["# Tile kernel counters, 30-qubit depth-40 circuit (rqc30_d40), fused complex64 path", "",
             "Two `rocprofv3 --pmc` passes over one step (28 `k_tile` dispatches: 4-qubit blocks on the",
             "matrix cores, split-bf16); mean per dispatch, each counter summed over its hardware",
             "instances.  Derived ratios use rocprofv3's formulas, with GRBM_GUI_ACTIVE / 8 (its sum",
             "over the eight XCDs) for the maximum over XCDs (the dispatch's active cycles).", "",
             "| counter | mean per dispatch |", "|---|---|"]
    for k in sorted(set(a) | set(b)):
        lines.append("| %s | %.4g |" % (k, a.get(k, b.get(k))))
    lines += ["", "| derived | value | formula |", "|---|---|---|"]
    if g:
        lines.append("| active cycles per dispatch (one XCD) | %.4g (%.2f ms at 2.4 GHz) | GRBM_GUI_ACTIVE / 8 |"
                     % (g, g / 2.4e6))
        lines.append("| MFMA busy %% | %.1f | 100 SQ_VALU_MFMA_BUSY_CYCLES / (active cycles x %d SIMDs) |"
                     % (100 * a["SQ_VALU_MFMA_BUSY_CYCLES"] / (g * simd), simd))
        lines.append("| VALU busy %% | %.1f | 100 SQ_ACTIVE_INST_VALU / %d CUs / active cycles |"
                     % (100 * a["SQ_ACTIVE_INST_VALU"] / cu / g, cu))
        lines.append("| LDS active %% | %.1f | 100 SQ_LDS_IDX_ACTIVE / (active cycles x %d CUs) |"
                     % (100 * a["SQ_LDS_IDX_ACTIVE"] / (g * cu), cu))
    if a.get("SQ_LDS_IDX_ACTIVE", 0) > a.get("SQ_LDS_BANK_CONFLICT", 0):
        lines.append("| LDS bank-conflict cycles / conflict-free LDS cycles | %.3f | SQ_LDS_BANK_CONFLICT / "
                     "(SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT) |"
                     % (a["SQ_LDS_BANK_CONFLICT"] / (a["SQ_LDS_IDX_ACTIVE"] - a["SQ_LDS_BANK_CONFLICT"])))
    if a.get("SQ_WAVES"):
        w = a["SQ_WAVES"]
        lines.append("| waves per dispatch | %.0f | SQ_WAVES |" % w)
        for k in ("SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
                  "SQ_INSTS_SALU"):
            if k in b:
                lines.append("| %s per wave | %.1f | %s / SQ_WAVES |" % (k[9:], b[k] / w, k))
    if "SQ_INSTS_VALU_MFMA_MOPS_BF16" in b:
        lines.append("| bf16 matrix-core flops per dispatch | %.4g | 512 SQ_INSTS_VALU_MFMA_MOPS_BF16 |"
                     % (512 * b["SQ_INSTS_VALU_MFMA_MOPS_BF16"]))
    lines += ["", "Commands (from the repository root, each pass its own process):", "", "```",
              cmds["pmc_sq1_fused_c64"], cmds["pmc_sq2_fused_c64"],
              "python3 bench.py --summarize-profiles %s" % PROFILE_DIR, "```", "", "Kernel sources hash: %s" % src]
    with open(os.path.join(ROOT, "profiles", "counters_k_tile_rqc30_d40.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print("wrote profiles/counters_k_tile_rqc30_d40.md")


def _last_json(path):
    if not os.path.exists(path):
        return None
    last = None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("{") and '"metric"' in line:
                last = json.loads(line)
    return last


def remap_label(name: str):
    """k_remap<unit, shift, pack, walk-the-shard> with readable vector types."""
    import re
    m = re.search(r"k_remap<(.*?)>\(", name)
    if not m:
        return name[:60]
    args = re.sub(r"(double|float) __vector\((\d)\)", r"\1\2", m.group(1))
    return "`k_remap<%s>`" % args


def summarize_remap(d, cmd, src):
    """profiles/kernel_stats_remap_l30.md from the kernel trace of bench.py
    --remap: per case and direction, the average of its timed dispatches (each
    case runs one untimed and three timed calls per direction, in the order of
    the run's JSON line) beside the run's own event timing."""
    import glob
    prof = os.path.join(ROOT, "profiles")
    line = _last_json(os.path.join(d, "remap.log"))
    tr = glob.glob(os.path.join(d, "remap", "**", "*kernel_trace.csv"), recursive=True)
    if not line or not tr:
        return
    rows = sorted((r for r in _csv_rows(tr[0]) if "k_remap" in r["Kernel_Name"]),
                  key=lambda r: int(r["Start_Timestamp"]))
    L = line["shard_qubits"]
    kl = ["# Kernel time, qubit-remap pack / unpack on a %d-qubit shard (g = %d)" % (L, line["g"]), "",
          "`rocprofv3 --kernel-trace` of `bench.py --remap`; per case and direction the average of the",
          "three timed dispatches. Algorithmic bytes per call: 2 * 2^%d * sizeof(amplitude) (34.36 GB for" % L,
          "complex128, 17.18 GB for complex64).", "",
          "| dtype | lq | direction | kernel | average us | GB/s (trace) | GB/s (HIP events, same run) |",
          "|---|---|---|---|---|---|---|"]
    per = 4
    for ci, res in enumerate(line["results"]):
        amp = 16 if res["dtype"] == "c128" else 8
        nbytes = 2.0 * (1 << L) * amp
        for di, name in enumerate(("pack", "unpack")):
            grp = rows[(2 * ci + di) * per:(2 * ci + di + 1) * per]
            if len(grp) < per:
                continue
            durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in grp[1:]]
            avg = sum(durs) / len(durs)
            kl.append("| %s | %s | %s | %s | %.1f | %.0f | %.0f |"
                      % (res["dtype"], res["lq"], name, remap_label(grp[0]["Kernel_Name"]), avg / 1e3,
                         nbytes / avg, res[name + "_GBps"]))
    kl += ["", "Command (from the repository root):", "", "```", cmd, "python3 bench.py --summarize-profiles %s"
           % PROFILE_DIR, "```", "", "Kernel sources hash: %s" % src]
    with open(os.path.join(prof, "kernel_stats_remap_l30.md"), "w") as f:
        f.write("\n".join(kl) + "\n")
    print("wrote profiles/kernel_stats_remap_l30.md")


def summarize_traj(d, cmd, src):
    """profiles/kernel_stats_trajectories.md: where a 512-trajectory batch
    spends its device time (kernel trace of bench.py --traj), beside the
    wall time and device time the library reports for the same calls."""
    import glob
    line = _last_json(os.path.join(d, "traj.log"))
    st = glob.glob(os.path.join(d, "traj", "**", "*kernel_stats.csv"), recursive=True)
    if not line or not st:
        return
    rows = _csv_rows(st[0])
    calls = len(line.get("autotune_calls", [])) + 3 + 1  # tuning calls, timed calls, the direct-launch call
    kl = ["# Kernel time, batched noisy trajectories (512 trajectories, 14-22 qubits, depth 24)", "",
          "`rocprofv3 --kernel-trace --stats` of `bench.py --traj`: %d calls of the 512-trajectory batch" % calls,
          "(the autotuner's candidates, three timed calls, one with direct launches) and the 4096-trajectory",
          "accuracy batch at n = 10.", "",
          "| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for r in rows[:12]:
        kl.append("| %s | %s | %.1f | %.1f | %s |" % (short_kernel(r["Name"]), r["Calls"],
                                                       float(r["TotalDurationNs"]) / 1e6,
                                                       float(r["AverageNs"]) / 1e3, r["Percentage"]))
    kl += ["", "The fastest timed call of the same run (library statistics): %.3f s wall, %.3f s device time "
           "(HIP events around each job), %.3f s of host planning, program build and upload, %d passes, "
           "%d jumps, %d kernel launches in %s; %.0f trajectories/s."
           % (line["seconds"], line["device_s"], line["host_s"], line["passes"], line["jumps"], line["launches"],
              "captured HIP graphs" if line.get("graph") else "direct launches", line["traj_per_s"]),
           "", "Command (from the repository root):", "", "```", cmd, "```", "",
           "Kernel sources hash (qs_fused.hip, qs_traj.hip and their headers): %s" % src]
    with open(os.path.join(ROOT, "profiles", "kernel_stats_trajectories.md"), "w") as f:
        f.write("\n".join(kl) + "\n")
    print("wrote profiles/kernel_stats_trajectories.md")


def summarize_single(d, cmd, src):
    """profiles/kernel_stats_single_c60.md: where the single-amplitude mode
    spends its device time (kernel trace of bench.py --single), beside the
    figures of the same run."""
    import glob
    line = _last_json(os.path.join(d, "single.log"))
    st = glob.glob(os.path.join(d, "single", "**", "*kernel_stats.csv"), recursive=True)
    if not line or not st:
        return
    rows = _csv_rows(st[0])
    kl = ["# Kernel time, single-amplitude mode (60-qubit 6x10 grid circuit, depth 14)", "",
          "`rocprofv3 --kernel-trace --stats` of `bench.py --single`: one warm-up bitstring, then %d bitstrings"
          % line["bitstrings"],
          "in chunks of %d, every merge of the plan per chunk." % line["batch"], "",
          "| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for r in rows[:12]:
        kl.append("| %s | %s | %.1f | %.1f | %s |" % (short_kernel(r["Name"]), r["Calls"],
                                                       float(r["TotalDurationNs"]) / 1e6,
                                                       float(r["AverageNs"]) / 1e3, r["Percentage"]))
    kl += ["", "The same run: %d amplitudes in %.3f s (%.1f /s), %.2f TFLOP/s FP64 on the plan's algorithmic "
           "flops (%.3g per amplitude), %d merges, largest merged tensor %d indices; planning %.2f s, once "
           "per circuit, outside the timed calls."
           % (line["bitstrings"], line["seconds"], line["value"], line["roofline"]["achieved"],
              line["flops_per_amplitude"], line["merges"], line["max_rank"], line["planning_s"]),
           "", "Command (from the repository root):", "", "```", cmd, "```", "",
           "Kernel sources hash (qs_single.hip and its headers): %s" % src]
    with open(os.path.join(ROOT, "profiles", "kernel_stats_single_c60.md"), "w") as f:
        f.write("\n".join(kl) + "\n")
    print("wrote profiles/kernel_stats_single_c60.md")


def summarize_partial(d, cmd, src):
    """profiles/kernel_stats_partial_40q.md: device time of the partial-amplitude
    mode (kernel trace of bench.py --partial), beside the figures of the same run."""
    import glob
    line = _last_json(os.path.join(d, "partial.log"))
    st = glob.glob(os.path.join(d, "partial", "**", "*kernel_stats.csv"), recursive=True)
    if not line or not st:
        return
    rows = _csv_rows(st[0])
    kl = ["# Kernel time, partial-amplitude mode (%s)" % line["workload"], "",
          "`rocprofv3 --kernel-trace --stats` of `bench.py --partial`: the circuit divided into parts of %s qubits "
          "by %d cut gates (Eq. 4), %d sub-circuits, %d sampled amplitudes, once unfused and once with greedy "
          "complex128 blocks." % (" and ".join(str(x) for x in line["parts"]), line["cuts"], line["sub_circuits"],
                                  line["amplitudes"]), "",
          "| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for r in rows[:12]:
        kl.append("| %s | %s | %.1f | %.1f | %s |" % (short_kernel(r["Name"]), r["Calls"],
                                                       float(r["TotalDurationNs"]) / 1e6,
                                                       float(r["AverageNs"]) / 1e3, r["Percentage"]))
    kl += ["", "The same run (wall time of each whole call): " + "; ".join(
        "%s %.3f s, %.0f amplitudes/s" % (r["path"], r["seconds"], r["amplitudes_per_s"]) for r in line["runs"]) + ".",
        "", "Command (from the repository root):", "", "```", cmd, "```", "",
        "Kernel sources hash: %s" % src]
    with open(os.path.join(ROOT, "profiles", "kernel_stats_partial_40q.md"), "w") as f:
        f.write("\n".join(kl) + "\n")
    print("wrote profiles/kernel_stats_partial_40q.md")


def summarize_profiles(d):
    """Write profiles/traffic.json and the text summaries from rocprofv3 CSVs."""
    import glob
    prof = os.path.join(ROOT, "profiles")
    os.makedirs(prof, exist_ok=True)
    cmds = {sub: profile_command(sub, fl, ba) for sub, fl, ba in PROFILE_RUNS}
    # copy calibration: a plain 4 GiB device copy reads and writes 4 GiB
    copy_kib = float(4 << 30) / 1024.0
    cf = [v for k, v in _counter_means(d, "pmc_fetch_copy").items() if "copyBuffer" in k or "copy" in k.lower()]
    cw = [v for k, v in _counter_means(d, "pmc_write_copy").items() if "copyBuffer" in k or "copy" in k.lower()]
    cf = max(cf, key=lambda x: x[1])
    cw = max(cw, key=lambda x: x[1])
    fetch_scale, write_scale = copy_kib / cf[1], copy_kib / cw[1]
    src = source_hash()
    bench_line = _last_json(os.path.join(d, "ktrace.log"))
    traffic = {"_calibration": {"copy_bytes": 4 << 30, "fetch_kib": cf[1], "write_kib": cw[1],
                                "fetch_scale": fetch_scale, "write_scale": write_scale,
                                "commands": [cmds["pmc_fetch_copy"], cmds["pmc_write_copy"]]}}
    lines = ["# HBM traffic per dispatch, 30-qubit depth-40 circuit (rqc30_d40)", "",
             "FETCH_SIZE and WRITE_SIZE (KiB per dispatch, rocprofv3 `--pmc`, one counter per run),",
             "scaled by what the same counters read for a plain 4 GiB device copy:",
             "", "| copy counter | KiB per dispatch | true KiB | scale |", "|---|---|---|---|",
             "| FETCH_SIZE | %.1f | %.1f | %.4f |" % (cf[1], copy_kib, fetch_scale),
             "| WRITE_SIZE | %.1f | %.1f | %.4f |" % (cw[1], copy_kib, write_scale), "",
             "| path | kernel | dispatches | FETCH KiB | WRITE KiB | scaled HBM bytes / dispatch | "
             "algorithmic bytes / launch | ratio |", "|---|---|---|---|---|---|---|---|"]
    for path in ("fused_c64", "plain_c128"):
        fm = _counter_means(d, "pmc_fetch_%s" % path)
        wm = _counter_means(d, "pmc_write_%s" % path)
        alg = None
        if bench_line and path in bench_line.get("paths", {}):
            alg = bench_line["paths"][path]
        by_class = {}
        for k in fm:
            cls = kernel_class_of(k)
            if cls is None or k not in wm:
                continue
            nf, vf = fm[k]
            nw, vw = wm[k]
            b = (vf * fetch_scale + vw * write_scale) * 1024.0
            c = by_class.setdefault(cls, [0, 0.0, 0.0, 0.0])
            c[0] += nf
            c[1] += vf * nf
            c[2] += vw * nf
            c[3] += b * nf
            lines.append("| %s | %s | %d | %.0f | %.0f | %.4g | | |" % (path, short_kernel(k), nf, vf, vw, b))
        for cls, (cnt, tf, tw, tb) in sorted(by_class.items()):
            rec = {"source_hash": src, "plan": "greedy", "dispatches": cnt, "fetch_kib_per_launch": tf / cnt,
                   "write_kib_per_launch": tw / cnt, "bytes_per_launch": tb / cnt,
                   "commands": [cmds["pmc_fetch_%s" % path], cmds["pmc_write_%s" % path]]}
            ab = None
            if alg and alg.get("dominant") == cls:
                ab = alg["roofline"]["alg_bytes_per_launch"]
                rec["alg_bytes_per_launch"] = ab
                rec["ratio_to_algorithmic"] = rec["bytes_per_launch"] / ab
            traffic[traffic_key("rqc30_d40", 30, path, cls)] = rec
            lines.append("| %s | **class %s** | %d | %.0f | %.0f | %.4g | %s | %s |"
                         % (path, cls, cnt, tf / cnt, tw / cnt, tb / cnt,
                            "%.4g" % ab if ab else "", "%.3f" % (tb / cnt / ab) if ab else ""))
    lines += ["", "Commands (from the repository root, after `cd /tmp && export TMPDIR=/tmp` and with",
              "paths taken from the root; each pass is its own process):", "", "```"]
    lines += [cmds[k] for k in cmds if k.startswith(("pmc_fetch", "pmc_write"))]
    lines += ["python3 bench.py --summarize-profiles %s" % PROFILE_DIR, "```", "",
              "Kernel sources hash: %s" % src]
    with open(os.path.join(prof, "hbm_traffic_rqc30_d40.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.join(prof, "traffic.json"), "w") as f:
        json.dump(traffic, f, indent=1, sort_keys=True)
        f.write("\n")
    # kernel trace statistics
    files = glob.glob(os.path.join(d, "ktrace", "**", "*kernel_stats.csv"), recursive=True)
    rows = _csv_rows(files[0])
    kl = ["# Kernel time, 30-qubit depth-40 circuit (rqc30_d40), fused c64 and plain c128 paths", "",
          "`rocprofv3 --kernel-trace --stats` over the warm-up runs (plain c128: 1; fused c64: 5, four of"
          " which time the candidate tile orders) and 2 timed steps of each path.", "",
          "| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for r in rows[:20]:
        kl.append("| %s | %s | %.1f | %.1f | %s |" % (short_kernel(r["Name"]), r["Calls"],
                                                       float(r["TotalDurationNs"]) / 1e6,
                                                       float(r["AverageNs"]) / 1e3, r["Percentage"]))
    if bench_line:
        kl += ["", "The same run's bench line measured, with HIP events on the state's stream:", ""]
        for path, pr in bench_line.get("paths", {}).items():
            rf = pr["roofline"]
            kl.append("- %s: %.1f gates/s; dominant kernel class `%s` (%s), average launch %.1f us, "
                      "%.0f GB/s on %.4g algorithmic bytes per launch"
                      % (path, pr["gates_per_s"], pr["dominant"], rf["kernel"], rf["avg_launch_ms"] * 1e3,
                         rf["achieved"], rf["alg_bytes_per_launch"]))
    # the same trace per dispatch: the dominant kernel of each path over the
    # timed steps only (the last steps x launches-per-step dispatches of its
    # class), to set beside the bench line's event timing
    tr = glob.glob(os.path.join(d, "ktrace", "**", "*kernel_trace.csv"), recursive=True)
    if tr and bench_line:
        trows = sorted(_csv_rows(tr[0]), key=lambda r: int(r["Start_Timestamp"]))
        kl += ["", "Per dispatch (kernel trace), timed steps only:", ""]
        for path, pr in bench_line.get("paths", {}).items():
            dom = pr["dominant"]
            nl = pr["kernels"][dom]["launches"] * bench_line.get("steps", 0)
            durs = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in trows
                    if kernel_class_of(r["Kernel_Name"]) == dom][-nl:] if nl else []
            if durs:
                kl.append("- %s: class `%s`, last %d dispatches, average %.1f us (HIP events: %.1f us)"
                          % (path, dom, len(durs), sum(durs) / len(durs) / 1e3,
                             pr["roofline"]["avg_launch_ms"] * 1e3))
    kl += ["", "Command (from the repository root):", "", "```", cmds["ktrace"], "```", "",
           "Kernel sources hash: %s" % src]
    with open(os.path.join(prof, "kernel_stats_rqc30_d40.md"), "w") as f:
        f.write("\n".join(kl) + "\n")
    if os.path.isdir(os.path.join(d, "remap")):
        summarize_remap(d, cmds["remap"], src)
    if os.path.isdir(os.path.join(d, "pmc_sq1_fused_c64")):
        summarize_sq(d, cmds, src)
    if os.path.isdir(os.path.join(d, "traj")):
        summarize_traj(d, cmds["traj"], source_hash(("qs_fused.hip", "qs_traj.hip")))
    if os.path.isdir(os.path.join(d, "partial")):
        summarize_partial(d, cmds["partial"], src)
    if os.path.isdir(os.path.join(d, "single")):
        summarize_single(d, cmds["single"], source_hash(("qs_single.hip",)))
    print("wrote profiles/traffic.json, profiles/hbm_traffic_rqc30_d40.md, profiles/kernel_stats_rqc30_d40.md")


def run_path(qs, torch, cg, name, n, circuit, gates, steps, warmup, kmax, plan, tile_qubits=0,
             workload="rqc30_d40"):
    dt = qs.C64 if name.endswith("c64") else qs.C128
    fused = name.startswith("fused")
    tdt = torch.complex64 if dt == qs.C64 else torch.complex128
    buf = torch.empty(1 << n, dtype=tdt, device="cuda")
    stream = torch.cuda.Stream()
    st = qs.State(n, dt, buffer=buf, stream=stream.cuda_stream)
    plan_id = ({"learned": qs.PLAN_LEARNED, "autotune": qs.PLAN_AUTOTUNE}.get(plan, qs.PLAN_GREEDY)
               if fused else qs.PLAN_UNFUSED)
    if fused and dt == qs.C64:
        # the first runs of a plan time each candidate tile order per sweep
        # (RunOpts.tile_order = 0): they are plan preparation, untimed
        warmup = max(warmup, qs.TILE_ORDERS + 1)
    if plan_id == qs.PLAN_AUTOTUNE:  # every candidate runs once before the timed steps
        warmup = max(warmup, circuit.autotune_result(n, dt)[1] + qs.TILE_ORDERS + 1)
    pm = [n - 1, n // 2, 0]

    def step():
        st.reset()
        st.run(circuit, plan=plan_id, k_max=kmax, tile_qubits=tile_qubits if fused else 0)
        nrm = st.norm()
        pr = st.probabilities(pm)
        return nrm, pr

    for w in range(warmup):
        t0 = time.perf_counter()
        step()
        log("%s warmup %d: %.3f s" % (name, w, time.perf_counter() - t0))
    torch.cuda.synchronize()
    st.profile(True)
    st.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        nrm, pr = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kern = {}
    for kid, kname in enumerate(qs.KERNEL_NAMES):
        r = st.profile_query(kid)
        if r["launches"]:
            kern[kname] = r
    st.profile(False)
    tot_bytes = sum(r["bytes"] for r in kern.values())
    dom = max(kern, key=lambda k: kern[k]["ms"])
    d = kern[dom]
    achieved = (d["bytes"] / d["launches"]) / (d["ms"] / d["launches"] * 1e-3) / 1e9
    res = {
        "gates_per_s": gates * steps / el,
        "ms_per_step": el / steps * 1e3,
        "hbm_frac_path": tot_bytes / el / 1e9 / HBM_PEAK_GBPS,
        "kernels": {k: {"launches": v["launches"] // steps, "ms_per_step": v["ms"] / steps,
                        "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] else 0.0}
                    for k, v in kern.items()},
        "norm": nrm,
        "dominant": dom,
        "roofline": {"bound": "hbm", "kernel": KERNEL_SYMBOL.get(dom, dom),
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "alg_bytes_per_launch": d["bytes"] / d["launches"],
                     "avg_launch_ms": d["ms"] / d["launches"],
                     "traffic": traffic_for(workload, n, name, dom, plan)},
    }
    if dom == "tile" and d["flops"]:
        # the same launches seen from the matrix cores: the fused blocks'
        # algorithmic flops (8 * 2^k per amplitude, the real-form GEMM count)
        # executed three times as split-bf16 products, against the dense
        # bf16 peak
        alg_tf = (d["flops"] / d["launches"]) / (d["ms"] / d["launches"] * 1e-3) / 1e12
        res["roofline_mfma"] = {"bound": "mfma", "kernel": KERNEL_SYMBOL.get(dom, dom),
                                "achieved": 3 * alg_tf, "algorithmic": alg_tf, "peak": MFMA_BF16_PEAK_TFLOPS,
                                "unit": "TFLOP/s", "frac": 3 * alg_tf / MFMA_BF16_PEAK_TFLOPS,
                                "alg_flops_per_launch": d["flops"] / d["launches"]}
    if plan_id == qs.PLAN_AUTOTUNE:
        tr, nc, tq, km, sec = circuit.autotune_result(n, dt)
        res["autotune"] = {"tried": tr, "candidates": nc, "tile_qubits": tq, "k_max": km, "seconds": sec}
    log("%s: %.1f gates/s, %.1f ms/step, path HBM fraction %.3f, dominant %s at %.0f GB/s"
        % (name, res["gates_per_s"], res["ms_per_step"], res["hbm_frac_path"], dom, achieved))
    return res, st, buf, stream


def gate_bandwidth_sweep(qs, torch, cg, st, stream, n, amp_bytes, reps=3):
    """Effective GB/s of single gates on the resident state: a dense U3 on each
    target bit k, and a controlled U3 for each control bit (target n-1, or 0
    when the control is n-1).  Algorithmic bytes: 2 * 2^n * amp (dense),
    2 * 2^(n-1) * amp (one control).  Timed with events on the state's stream."""
    u = cg.u3(1.1, 0.7, -0.4)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(targets, controls, nbytes):
        st.apply_gate(targets, controls, u)  # first touch / warm
        ev0.record(stream)
        for _ in range(reps):
            st.apply_gate(targets, controls, u)
        ev1.record(stream)
        ev1.synchronize()
        return nbytes * reps / (ev0.elapsed_time(ev1) * 1e-3) / 1e9

    dense = [timed([k], [], 2.0 * (1 << n) * amp_bytes) for k in range(n)]
    ctrl = [timed([n - 1 if c != n - 1 else 0], [c], 2.0 * (1 << (n - 1)) * amp_bytes) for c in range(n)]
    log("single gates: dense U3 %.0f..%.0f GB/s over targets, CU3 %.0f..%.0f GB/s over controls"
        % (min(dense), max(dense), min(ctrl), max(ctrl)))
    return {"dense_u3_GBps_by_target": [round(x, 1) for x in dense],
            "cu3_GBps_by_control": [round(x, 1) for x in ctrl]}


def copy_ceiling(torch, nbytes=4 << 30, reps=5):
    """Device copy bandwidth (read + write bytes / time) as a measured HBM
    ceiling beside the nominal peak: the runtime's blit copy and an
    elementwise copy kernel; the better of the two is reported."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for name, fn in (("blit", lambda: b.copy_(a)), ("elementwise", lambda: torch.mul(a, 1.0, out=b))):
        fn()
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        ev1.synchronize()
        res[name] = 2.0 * nbytes * reps / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    log("device copy: %.0f GB/s blit, %.0f GB/s elementwise (read + write)" % (res["blit"], res["elementwise"]))
    return max(res.values()), res


def remap_bench(qs, torch, L=30, g=3, reps=3, emit=True):
    """Pack and unpack of the qubit-remap exchange (qs_remap_pack / _unpack) on
    one shard at its real shape (L local qubits), for several local-qubit
    sets: algorithmic bytes 2 * 2^L * amp per call (every amplitude read and
    written once) / the average call time, from HIP events on the shard's
    stream.  The all-to-all between the calls needs more than one GPU and is
    not run."""
    cases = [("c128", [L - 3, L - 2, L - 1]), ("c128", [20, 21, 22]), ("c128", [4, 5, 6]),
             ("c128", [0, 13, L - 1]), ("c64", [4, 5, 6]), ("c64", [0, 13, L - 1])]
    out = []
    stream = torch.cuda.Stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for dtype, lq in cases:
        lq = lq[:g]
        dt = qs.C128 if dtype == "c128" else qs.C64
        tdt = torch.complex128 if dt == qs.C128 else torch.complex64
        t = torch.empty(1 << L, dtype=tdt, device="cuda")
        buf = torch.empty_like(t)
        st = qs.State(L, dt, buffer=t, stream=stream.cuda_stream)
        nbytes = 2.0 * (1 << L) * t.element_size()
        res = {"dtype": dtype, "lq": lq}
        for name, fn in (("pack", lambda: st.remap_pack(lq, buf)), ("unpack", lambda: st.remap_unpack(lq, buf))):
            fn()
            ev0.record(stream)
            for _ in range(reps):
                fn()
            ev1.record(stream)
            ev1.synchronize()
            res[name + "_GBps"] = round(nbytes * reps / (ev0.elapsed_time(ev1) * 1e-3) / 1e9, 1)
        log("remap %s L=%d lq=%s: pack %.0f GB/s, unpack %.0f GB/s"
            % (dtype, L, lq, res["pack_GBps"], res["unpack_GBps"]))
        out.append(res)
        st.close()
        del t, buf
        torch.cuda.empty_cache()
    rec = {"metric": "qubit-remap pack / unpack bandwidth", "unit": "GB/s", "shard_qubits": L, "g": g,
           "bytes": "2 * 2^L * sizeof(amplitude) per call", "results": out}
    if emit:
        print(json.dumps(rec))
    return rec


def partial_bench(qs, cg, rows=8, cols=5, depth=8, top_rows=4, m=1 << 20, seed=6001, emit=True):
    """Partial-amplitude mode (qs_partial_amplitudes) on a circuit no full state
    of which fits one GPU: an 8 x 5 grid (40 qubits, 16 TiB as complex128) at
    depth 8, divided between rows 3 and 4 (two 20-qubit parts, 10 CZ cut),
    2^20 sampled output amplitudes.  Wall time of the whole call (cut
    planning, 2^c branch words x 2 sub-circuits on the device, FP64
    recombination)."""
    import numpy as np
    n = rows * cols
    ops = cg.random_circuit(rows, cols, depth, seed=seed)
    c = qs.Circuit(ops)
    part_a = (1 << (top_rows * cols)) - 1
    idx = np.random.default_rng(seed + 1).integers(0, 1 << n, size=m, dtype=np.uint64)
    cuts = c.partial_cuts(n, part_a)
    runs = []
    ref = None
    for name, dt, plan in (("c128_unfused", qs.C128, qs.PLAN_UNFUSED), ("c128_greedy", qs.C128, qs.PLAN_GREEDY),
                           ("c64_greedy", qs.C64, qs.PLAN_GREEDY)):
        t0 = time.perf_counter()
        amps, _ = c.partial_amplitudes(n, part_a, idx, dtype=dt, plan=plan)
        sec = time.perf_counter() - t0
        p = np.abs(amps) ** 2
        rec_run = {"path": name, "seconds": round(sec, 3), "amplitudes_per_s": round(m / sec, 1),
                   "mean_prob_times_2n": round(float(p.mean() * 2.0 ** n), 4)}
        extra = ""
        if ref is None:
            ref = amps
        else:
            # agreement with the unfused complex128 run on the same indices
            d = amps - ref
            rec_run["max_abs_diff_vs_c128_unfused"] = float(np.max(np.abs(d)))
            rec_run["rel_l2_vs_c128_unfused"] = float(np.linalg.norm(d) / np.linalg.norm(ref))
            extra = "; vs c128 unfused: max|d| %.2e, rel l2 %.2e" % (rec_run["max_abs_diff_vs_c128_unfused"],
                                                                    rec_run["rel_l2_vs_c128_unfused"])
        log("partial %s: %d qubits, %d cuts, %d sub-circuits, %d amplitudes in %.2f s (%.0f amplitudes/s); "
            "mean |amp|^2 * 2^n = %.3f%s" % (name, n, cuts, 2 << cuts, m, sec, m / sec, p.mean() * 2.0 ** n, extra))
        runs.append(rec_run)
    rec = {"metric": "partial-amplitude mode: sampled amplitudes per second", "unit": "amplitudes/s",
           "value": max(r["amplitudes_per_s"] for r in runs),
           "workload": "%dx%d grid random circuit, %d qubits, depth %d, %d gates" % (rows, cols, n, depth,
                                                                                   cg.count_gates(ops)),
           "parts": [top_rows * cols, n - top_rows * cols], "cuts": cuts, "sub_circuits": 2 << cuts,
           "amplitudes": m, "runs": runs}
    if emit:
        print(json.dumps(rec))
    return rec


FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 (vector and matrix alike)


def single_bench(qs, cg, rows=6, cols=10, depth=14, words=32, seed=6201, emit=True):
    """Single-amplitude mode (qs_single_amplitudes) on a circuit far wider than
    any state vector: a 6 x 10 grid (60 qubits) at depth 14, `words` random
    bitstrings per call.  The graph, slices and elimination order are made
    once per circuit and kept with it (planning_s, timed apart); the timed
    call places the gate tensors and contracts every bitstring on the
    device.  The merges' algorithmic FP64 flops (8 per complex
    multiply-add) over the call's wall time, against the FP64 peak."""
    import numpy as np
    n = rows * cols
    ops = cg.random_circuit(rows, cols, depth, seed=seed)
    c = qs.Circuit(ops)
    bits = np.random.default_rng(seed + 1).integers(0, 1 << n, size=words, dtype=np.uint64)
    t0 = time.perf_counter()
    plan = c.single_plan(n)  # graph, slices and elimination order, kept with the circuit
    plan_s = time.perf_counter() - t0
    c.single_amplitudes(n, bits[:1])  # warm-up (first launches of the kernels)
    t0 = time.perf_counter()
    amps, info = c.single_amplitudes(n, bits)
    sec = time.perf_counter() - t0
    tf = plan["flops"] * words / sec / 1e12
    rec = {"metric": "single-amplitude mode: amplitudes per second", "unit": "amplitudes/s",
           "value": round(words / sec, 2),
           "workload": "%dx%d grid random circuit, %d qubits, depth %d, %d gates" % (rows, cols, n, depth,
                                                                                   cg.count_gates(ops)),
           "bitstrings": words, "seconds": round(sec, 4), "planning_s": round(plan_s, 3),
           "vertices": plan["vertices"], "merges": plan["merges"],
           "max_rank": plan["max_rank"], "flops_per_amplitude": plan["flops"],
           "peak_bytes_per_bitstring": plan["peak_bytes"], "batch": info["batch"],
           "roofline": {"bound": "fp64", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": tf / FP64_PEAK_TFLOPS},
           "mean_prob_times_2n": float(np.mean(np.abs(amps) ** 2) * 2.0 ** n)}
    log("single-amplitude: %d qubits depth %d, %d amplitudes in %.3f s (%.1f /s), %.2f TFLOP/s FP64, "
        "max rank %d" % (n, depth, words, sec, words / sec, tf, plan["max_rank"]))
    if emit:
        print(json.dumps(rec))
    return rec


def trajectory_bench(qs, cg, count, seed=4001, reps=3):
    """Batched noisy trajectories: widths n ~ U{14..22}, depth 24, depolarizing
    1e-3 / 1e-2 (two-qubit, Kronecker form) and amplitude damping 5e-4 per
    layer, complex64 states, one batch per call.  The autotuner's calls (one
    per candidate width set) run first as warm-up; the timed calls use the
    fastest.  Also: the mean <Z_q> of 4096 trajectories of the 10-qubit
    depth-24 circuit at the same rates against the exact density-matrix
    values (tests/golden/dm_n10_d24_workload_rates.txt, written by the
    oracle)."""
    import numpy as np
    t0 = time.perf_counter()
    batch = cg.trajectory_batch(count, seed=seed)
    circs = [qs.Circuit(ops) for _, ops in batch]
    widths = [n for n, _ in batch]
    gen = time.perf_counter() - t0
    tuning = []
    for _ in range(16):
        _, info = qs.run_trajectories(circs, widths, dtype=qs.C64, seed=seed, plan=qs.PLAN_AUTOTUNE)
        tuning.append({"tile_qubits": info["tile_qubits"], "k_max": info["k_max"], "max_outer": info["max_outer"],
                       "seconds": round(info["seconds"], 4)})
        if info["autotune_tried"] >= info["autotune_candidates"]:
            break
    runs = []
    for _ in range(reps):
        _, info = qs.run_trajectories(circs, widths, dtype=qs.C64, seed=seed, plan=qs.PLAN_AUTOTUNE)
        runs.append(info)
    best = min(runs, key=lambda r: r["seconds"])
    _, direct = qs.run_trajectories(circs, widths, dtype=qs.C64, seed=seed, plan=qs.PLAN_AUTOTUNE,
                                    direct_launch=True)
    sites = sum(sum(1 for o in ops if o.kind == "noise") for _, ops in batch)
    gates = sum(cg.count_gates(ops) for _, ops in batch)
    res = {"count": count, "seconds": best["seconds"], "traj_per_s": count / best["seconds"],
           "widths": [min(widths), max(widths)], "mean_width": sum(widths) / count,
           "logical_gates": gates, "noise_sites": sites, "generation_s": gen,
           "dtype": "c64 state, FP64 run sums and branch weights, Kraus branches drawn on the device",
           "passes": best["passes"], "jumps": best["jumps"], "launches": best["launches"],
           "graph": bool(best["graph"]), "host_s": best["host_seconds"], "device_s": best["device_seconds"],
           "widths_chosen": {"tile_qubits": best["tile_qubits"], "k_max": best["k_max"],
                             "max_outer": best["max_outer"]},
           "autotune_calls": tuning, "direct_launch_s": direct["seconds"]}
    log("trajectories: %d in %.3f s -> %.1f traj/s (%d passes, %d jumps, device %.3f s, host %.3f s; "
        "widths %s; direct launches %.3f s)" % (count, best["seconds"], count / best["seconds"], best["passes"],
                                               best["jumps"], best["device_seconds"], best["host_seconds"],
                                               res["widths_chosen"], direct["seconds"]))
    # accuracy of the trajectory mean at n = 10 against the exact density matrix
    n, T = 10, 4096
    ops = cg.random_circuit(2, 5, 24, seed=4010, dep1=1e-3, dep2=1e-2, damping=5e-4)
    zdm = np.loadtxt(os.path.join(ROOT, "tests", "golden", "dm_n10_d24_workload_rates.txt"))
    z, _ = qs.run_trajectories([qs.Circuit(ops)] * T, [n] * T, dtype=qs.C64, seed=78)
    zs = z.reshape(T, n)
    dev = np.abs(zs.mean(axis=0) - zdm)
    se = zs.std(axis=0) / math.sqrt(T)
    res["dm_check_n10"] = {"trajectories": T, "max_abs_dev_mean_z": float(dev.max()),
                           "max_dev_in_std_errors": float((dev / np.maximum(se, 1e-12)).max()),
                           "reference": "exact density matrix (FP64 oracle), tests/golden/dm_n10_d24_workload_rates.txt"}
    log("trajectory mean at n=10: max |<Z> - rho| = %.2e (%.2f standard errors)"
        % (dev.max(), res["dm_check_n10"]["max_dev_in_std_errors"]))
    return res


def train_cost_model(qs, cg, n=28, circuits=8, log_fn=None, ns=None):
    """Train the planner's cost network on sweep timings that the simulator
    records itself: random circuits on n-qubit complex64 states (each size in
    ns, default n alone), run under every candidate tile shape, each sweep's
    features and measured time per amplitude a sample; Adam on the GPU with
    the library's kernels."""
    import numpy as np
    Xs, ys = [], []
    for nn in (ns or (n,)):
        s = qs.State(nn, qs.C64)
        s.profile(True)
        shapes = [(r, nn // r) for r in range(2, nn // 2 + 1) if nn % r == 0]
        for i in range(circuits):
            rows, cols = shapes[i % len(shapes)]
            c = qs.Circuit(cg.random_circuit(rows, cols, 12, seed=9000 + i, cu3_prob=0.1))
            for m in (11, 12, 13):
                for k in (4, 5):
                    s.reset()
                    s.run(c, plan=qs.PLAN_GREEDY, k_max=k, tile_qubits=m)
        X, y = s.profile_samples()
        s.profile(False)
        s.close()
        Xs.append(X)
        ys.append(y)
    X, y = np.concatenate(Xs), np.concatenate(ys)
    p, loss = qs.mlp_train(qs.mlp_init(4), X, y, steps=3000, batch=256, lr=2e-3, seed=7)
    if log_fn:
        log_fn("cost model: %d sweep samples at %s qubits, final loss %.4f"
               % (X.shape[0], "/".join(str(v) for v in (ns or (n,))), loss))
    return p, int(X.shape[0])


def config5(qs, cg, torch):
    """34 qubits, 17 x 2 grid, depth 24: end-to-end gates/s of the complex64
    path under the learned, greedy and unfused plans, and agreement with the
    complex128 greedy-fused path (validated against the FP64 oracle at 30
    qubits) on 2^20 indices sampled without replacement (seed 5002)."""
    import numpy as np
    n, ops = cg.workload("rqc34_d24")
    gates = cg.count_gates(ops)
    circuit = qs.Circuit(ops)
    rng = np.random.default_rng(5002)
    cand = np.unique(rng.integers(0, 1 << n, size=(1 << 20) + (1 << 16), dtype=np.uint64))
    idx = np.sort(rng.permutation(cand)[: 1 << 20])
    out = {"workload": "rqc34_d24: 34-qubit random circuit, 17 x 2 grid, depth 24, %d logical gates" % gates,
           "sampled_indices": int(idx.size)}
    log("config 5: complex128 reference (256 GiB) ...")
    t0 = time.perf_counter()
    ref = qs.State(n, qs.C128)
    ref.run(circuit, plan=qs.PLAN_GREEDY, k_max=3)
    ref.synchronize()
    ref_s = time.perf_counter() - t0
    a = ref.amplitudes(idx)
    ref.close()
    del ref
    out["c128_greedy_k3"] = {"seconds": ref_s, "gates_per_s": gates / ref_s}
    log("c128 reference: %.1f s" % ref_s)
    p, nsamp = train_cost_model(qs, cg, log_fn=log)
    out["cost_model_samples"] = nsamp
    st = qs.State(n, qs.C64)
    for name, plan in (("learned", qs.PLAN_LEARNED), ("greedy", qs.PLAN_GREEDY), ("unfused", qs.PLAN_UNFUSED)):
        qs.cost_model_set(p if plan == qs.PLAN_LEARNED else None)
        # fused plans: the first runs of a plan time its candidate tile orders
        reps = 1 if plan == qs.PLAN_UNFUSED else qs.TILE_ORDERS + 2
        best = 1e30
        for r in range(reps):
            st.reset()
            st.synchronize()
            t0 = time.perf_counter()
            st.run(circuit, plan=plan)
            st.norm()
            best = min(best, time.perf_counter() - t0)
        b = st.amplitudes(idx)
        ov = abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)
        info = circuit.plan_info(n, qs.C64, plan)
        out[name] = {"seconds": best, "gates_per_s": gates / best, "sweeps": info["sweeps"],
                     "blocks": info["blocks"], "max_abs_diff": float(np.max(np.abs(a - b))),
                     "rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(a)),
                     "infidelity_sampled": float(1 - ov)}
        log("%s: %.1f gates/s, max|d| %.2e" % (name, gates / best, out[name]["max_abs_diff"]))
    qs.cost_model_set(None)
    st.close()
    out["learned_vs_greedy"] = out["greedy"]["seconds"] / out["learned"]["seconds"]
    out["learned_vs_unfused"] = out["unfused"]["seconds"] / out["learned"]["seconds"]
    print(json.dumps({"config5": out}), flush=True)


def _host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cg, n, ops, seconds, seconds_1t=12.0):
    """The FP64 oracle on the host, as it stands, on the full 2^n complex128
    state: a sample of the circuit's own gates taken evenly over the whole
    circuit (bit-reversed order of the gate index, so any prefix mixes
    one-qubit gates, CU3 and CZ in about their proportions), applied for
    about `seconds` with every host thread and for about `seconds_1t` with
    one.  Gates/s of each; state initialisation excluded."""
    import oracle
    gl = [o for o in ops if o.kind == "gate"]
    bits = max(1, (len(gl) - 1).bit_length())
    order = sorted(range(len(gl)), key=lambda i: int(format(i, "0%db" % bits)[::-1], 2))
    full = oracle.num_threads()
    psi = oracle.zero_state(n)

    def timed(budget, threads, start):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        done = 0
        kinds = {}
        while start + done < len(order) and (time.perf_counter() - t0 < budget or done < 2):
            g = gl[order[start + done]]
            oracle.apply(psi, g.targets, g.controls, g.matrix)
            kinds[g.name] = kinds.get(g.name, 0) + 1
            done += 1
        return done / (time.perf_counter() - t0), done, kinds

    rate, done, kinds = timed(seconds, full, 0)
    rate1, done1, _ = timed(seconds_1t, 1, done)
    oracle.set_threads(full)
    del psi
    mix = {"cz": kinds.get("cz", 0), "cu3": kinds.get("cu3", 0),
           "one_qubit": sum(v for k, v in kinds.items() if k not in ("cz", "cu3"))}
    circ = {"cz": sum(1 for g in gl if g.name == "cz"), "cu3": sum(1 for g in gl if g.name == "cu3")}
    circ["one_qubit"] = len(gl) - circ["cz"] - circ["cu3"]
    return {"value": rate, "unit": "gates/s", "cores": full, "kind": "oracle",
            "value_1_thread": rate1, "cpu_model": _host_cpu_model(),
            "sample": "%d gates of the %d-qubit circuit spread over all of it (one-qubit %d, CU3 %d, CZ %d; "
                      "circuit: %d / %d / %d) on the full 2^%d complex128 state, FP64, %d threads; then %d more "
                      "gates on 1 thread" % (done, n, mix["one_qubit"], mix["cu3"], mix["cz"], circ["one_qubit"],
                                             circ["cu3"], circ["cz"], n, full, done1)}


def main():
    args = parse()
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU: the state-vector path here is single-GPU "
              "(multi-GPU sharding is described, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        a = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": 4 << 30, "copy_bytes_written_per_launch": 4 << 30,
                          "launches": 5}))
        return

    from paper_2008_07140_amd import circuits as cg
    from paper_2008_07140_amd import qs

    if args.config5:
        config5(qs, cg, torch)
        return
    if args.remap:
        remap_bench(qs, torch)
        return
    if args.partial:
        partial_bench(qs, cg)
        return
    if args.single:
        single_bench(qs, cg)
        return
    if args.traj:
        rec = trajectory_bench(qs, cg, args.trajectories or 512)
        rec["metric"] = "batched noisy trajectories per second"
        print(json.dumps(rec))
        return
    if args.plan == "learned":
        p, _ = train_cost_model(qs, cg, log_fn=log)
        qs.cost_model_set(p)
    n, ops = cg.workload(args.workload)
    gates = cg.count_gates(ops)
    circuit = qs.Circuit(ops)
    log("workload %s: %d qubits, %d gates" % (args.workload, n, gates))
    paths = [p for p in args.paths.split(",") if p]
    out = {}
    states = {}
    sweep_state = None
    copy_gbps, copy_detail = copy_ceiling(torch)
    for p in paths:
        res, st, buf, stream = run_path(qs, torch, cg, p, n, circuit, gates, args.steps, args.warmup,
                                        args.kmax, args.plan, args.tile_qubits, args.workload)
        out[p] = res
        states[p] = (st, buf)
        if p == "plain_c128" and not args.no_by_target:
            sweep_state = (st, stream)
    learned = None
    if "fused_c64" in out and args.plan == "greedy" and not args.no_extras:
        # the learned planner on the same circuit (spec comparison):
        # the cost network trained on the simulator's own sweep timings
        t0 = time.perf_counter()
        p, nsamp = train_cost_model(qs, cg, log_fn=log)
        train_s = time.perf_counter() - t0
        qs.cost_model_set(p)
        try:
            res_l, st_l, _, _ = run_path(qs, torch, cg, "fused_c64", n, circuit, gates, args.steps, args.warmup,
                                         args.kmax, "learned", args.tile_qubits, args.workload)
            st_l.close()
            info_l = circuit.plan_info(n, qs.C64, qs.PLAN_LEARNED, k_max=args.kmax, tile_qubits=args.tile_qubits)
        finally:
            qs.cost_model_set(None)
        info_g = circuit.plan_info(n, qs.C64, qs.PLAN_GREEDY, k_max=args.kmax, tile_qubits=args.tile_qubits)
        learned = {"gates_per_s": res_l["gates_per_s"], "ms_per_step": res_l["ms_per_step"],
                   "sweeps": info_l["sweeps"], "blocks": info_l["blocks"],
                   "greedy_sweeps": info_g["sweeps"], "greedy_blocks": info_g["blocks"],
                   "same_plan_as_greedy": info_l == info_g,
                   "learned_over_greedy": res_l["gates_per_s"] / out["fused_c64"]["gates_per_s"],
                   "training_samples": nsamp, "training_s": train_s}
        if "plain_c128" in out:
            learned["learned_over_plain_c128"] = res_l["gates_per_s"] / out["plain_c128"]["gates_per_s"]
        log("learned plan: %.1f gates/s (%d sweeps, %d blocks; greedy %d / %d), learned/greedy %.3f"
            % (res_l["gates_per_s"], info_l["sweeps"], info_l["blocks"], info_g["sweeps"], info_g["blocks"],
               learned["learned_over_greedy"]))
    acc = None
    if "fused_c64" in states and "plain_c128" in states:
        rng = np.random.default_rng(12345)
        idx = np.unique(rng.integers(0, 1 << n, size=1 << 20, dtype=np.uint64))
        a = states["plain_c128"][0].amplitudes(idx)
        b = states["fused_c64"][0].amplitudes(idx)
        ov = abs(np.vdot(a, b)) ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)
        acc = {"sampled_indices": int(idx.size), "infidelity_c64_vs_c128": float(1 - ov),
               "max_abs_diff": float(np.max(np.abs(a - b))),
               "rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(a))}
        log("accuracy c64 vs c128 on %d sampled amplitudes: infidelity %.3e, max|d| %.3e"
            % (idx.size, acc["infidelity_c64_vs_c128"], acc["max_abs_diff"]))
    by_target = None
    if sweep_state is not None:
        by_target = gate_bandwidth_sweep(qs, torch, cg, sweep_state[0], sweep_state[1], n, 16)
        sweep_state = None
    for st, buf in states.values():
        st.close()
    del states
    torch.cuda.empty_cache()
    traj = trajectory_bench(qs, cg, args.trajectories) if args.trajectories > 0 else None
    # the widened paths, measured after (and apart from) the timed steps
    extras = {}
    if not args.no_extras:
        for key, fn in (("partial_mode", lambda: partial_bench(qs, cg, emit=False)),
                        ("single_amplitude_mode", lambda: single_bench(qs, cg, emit=False)),
                        ("remap", lambda: remap_bench(qs, torch, emit=False))):
            try:
                extras[key] = fn()
            except Exception as e:  # reported, never fatal to the headline
                log("%s measurement failed: %s" % (key, e))
                extras[key] = {"error": str(e)}
    primary = "fused_c64" if "fused_c64" in out else paths[0]
    prim = out[primary]
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        cpu = cpu_baseline(cg, n, ops, args.cpu_seconds)
        log("cpu baseline: %.3f gates/s on %d threads" % (cpu["value"], cpu["cores"]))
    line = {
        "metric": METRIC,
        "value": prim["gates_per_s"],
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": prim["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16x3" if primary.endswith("c64") else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %d-qubit random circuit, depth %d, %d logical gates"
                               % (args.workload, n, cg.WORKLOADS[args.workload][2], gates),
                   "path": primary, "plan": args.plan,
                   "k_max": (args.kmax or 4) if primary.endswith("c64") else (args.kmax or 0),
                   "tile_qubits": (args.tile_qubits or min(13, n)) if primary.endswith("c64") else 0,
                   "arithmetic": "complex64 state (FP32); fused blocks on the matrix cores as split-bf16 "
                                 "products (hi*hi + hi*lo + lo*hi, about 16 significant bits per block) with "
                                 "FP32 accumulation; FP64 norm and probability reductions"
                   if primary.endswith("c64") else "complex128 (FP64) per-gate kernels"},
        "roofline": prim["roofline"],
        "hbm_frac_path": prim["hbm_frac_path"],
        "copy_GBps": copy_gbps,
        "copy_detail_GBps": copy_detail,
        "paths": out,
        "single_gates_c128": by_target,
        "accuracy": acc,
        "trajectories": traj,
        "learned_plan": learned,
        "cpu_baseline": cpu,
    }
    line.update(extras)
    if "roofline_mfma" in prim:
        line["roofline_mfma"] = prim["roofline_mfma"]
    if "plain_c128" in out and primary != "plain_c128":
        line["speedup_vs_plain_c128"] = prim["gates_per_s"] / out["plain_c128"]["gates_per_s"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

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
    p.add_argument("--plan", default="greedy", choices=["greedy", "learned"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--trajectories", type=int, default=512,
                   help="noisy trajectories in the batched-trajectory measurement (0 = skip)")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 4 GiB device-to-device copy (5 times), the reference "
                        "for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE")
    return p.parse_args()


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2008_07140_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel_class: str):
    """HBM bytes per launch measured by rocprofv3 counters for this kernel, if
    the counters were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get(kernel_class)
    if not rec or rec.get("source_hash") != source_hash():
        return None
    return rec.get("bytes_per_launch")


def run_path(qs, torch, cg, name, n, circuit, gates, steps, warmup, kmax, plan, tile_qubits=0):
    dt = qs.C64 if name.endswith("c64") else qs.C128
    fused = name.startswith("fused")
    tdt = torch.complex64 if dt == qs.C64 else torch.complex128
    buf = torch.empty(1 << n, dtype=tdt, device="cuda")
    stream = torch.cuda.Stream()
    st = qs.State(n, dt, buffer=buf, stream=stream.cuda_stream)
    plan_id = (qs.PLAN_LEARNED if plan == "learned" else qs.PLAN_GREEDY) if fused else qs.PLAN_UNFUSED
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
                     "traffic": traffic_for(dom)},
    }
    log("%s: %.1f gates/s, %.1f ms/step, path HBM fraction %.3f, dominant %s at %.0f GB/s"
        % (name, res["gates_per_s"], res["ms_per_step"], res["hbm_frac_path"], dom, achieved))
    return res, st, buf


def trajectory_bench(qs, cg, count, seed=4001):
    """Batched noisy trajectories: widths n ~ U{14..22}, depth 24, depolarizing
    1e-3 / 1e-2 (two-qubit, Kronecker form) and amplitude damping 5e-4 per
    layer, complex64 states, one batch."""
    t0 = time.perf_counter()
    batch = cg.trajectory_batch(count, seed=seed)
    circs = [qs.Circuit(ops) for _, ops in batch]
    widths = [n for n, _ in batch]
    gen = time.perf_counter() - t0
    qs.run_trajectories(circs[:8], widths[:8], dtype=qs.C64, seed=seed)  # warm-up
    z, sec = qs.run_trajectories(circs, widths, dtype=qs.C64, seed=seed)
    sites = sum(sum(1 for o in ops if o.kind == "noise") for _, ops in batch)
    gates = sum(cg.count_gates(ops) for _, ops in batch)
    res = {"count": count, "seconds": sec, "traj_per_s": count / sec,
           "widths": [min(widths), max(widths)], "mean_width": sum(widths) / count,
           "logical_gates": gates, "noise_sites": sites, "generation_s": gen,
           "dtype": "c64 state, FP64 branch weights"}
    log("trajectories: %d in %.3f s -> %.1f traj/s" % (count, sec, count / sec))
    return res


def cpu_baseline(cg, n, ops, seconds):
    """The FP64 oracle on the host, on the first gates of the same circuit
    applied to the full 2^n state, for about `seconds` of gate work."""
    import numpy as np

    import oracle
    psi = oracle.zero_state(n)
    gl = [o for o in ops if o.kind == "gate"]
    t0 = time.perf_counter()
    done = 0
    while done < len(gl) and (time.perf_counter() - t0 < seconds or done < 2):
        g = gl[done]
        oracle.apply(psi, g.targets, g.controls, g.matrix)
        done += 1
    el = time.perf_counter() - t0
    del psi
    return {"value": done / el, "unit": "gates/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "first %d gates of the %d-qubit circuit on the full 2^%d complex128 state "
                      "(FP64, OpenMP over the amplitude loop), %.1f s; state initialisation "
                      "excluded" % (done, n, n, el)}


def main():
    args = parse()
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

    n, ops = cg.workload(args.workload)
    gates = cg.count_gates(ops)
    circuit = qs.Circuit(ops)
    log("workload %s: %d qubits, %d gates" % (args.workload, n, gates))
    paths = [p for p in args.paths.split(",") if p]
    out = {}
    states = {}
    for p in paths:
        res, st, buf = run_path(qs, torch, cg, p, n, circuit, gates, args.steps, args.warmup,
                                args.kmax, args.plan, args.tile_qubits)
        out[p] = res
        states[p] = (st, buf)
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
    for st, buf in states.values():
        st.close()
    del states
    torch.cuda.empty_cache()
    traj = trajectory_bench(qs, cg, args.trajectories) if args.trajectories > 0 else None
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
        "dtype": "f32" if primary.endswith("c64") else "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %d-qubit random circuit, depth %d, %d logical gates"
                               % (args.workload, n, cg.WORKLOADS[args.workload][2], gates),
                   "path": primary, "plan": args.plan, "k_max": args.kmax,
                   "tile_qubits": args.tile_qubits,
                   "state": "complex64 (FP32), FP64 reductions" if primary.endswith("c64")
                   else "complex128 (FP64)"},
        "roofline": prim["roofline"],
        "hbm_frac_path": prim["hbm_frac_path"],
        "paths": out,
        "accuracy": acc,
        "trajectories": traj,
        "cpu_baseline": cpu,
    }
    if "plain_c128" in out and primary != "plain_c128":
        line["speedup_vs_plain_c128"] = prim["gates_per_s"] / out["plain_c128"]["gates_per_s"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

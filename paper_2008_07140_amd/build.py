"""Build libqs.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2008_07140_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libqs.so")

SOURCES = ["qs_kernels.hip", "qs_fused.hip", "qs_traj.hip", "qs_mlp.hip", "qs_remap.hip", "qs_single.hip",
           "qs_noalloc.hip",
           "qs_api.cpp", "qs_plan.cpp", "qs_script.cpp", "qs_single.cpp"]
HEADERS = ["qs_internal.h", "qs_plan.h", "qs_philox.h", "qs_tile.h", "qs_traj.h", "qs_mlp.h", "qs_single.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops"]
HOST_FLAGS = ["-D__HIP_PLATFORM_AMD__", "-I", os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include")]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result", "-Wno-unused-value",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose: bool = True, jobs: int = 8, incremental: bool = False) -> str:
    """Compile every source to an object in _build/ and link libqs.so.
    With `incremental`, objects newer than their source and every header are
    kept."""
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs, procs = [], []
    hdr = max([os.path.getmtime(os.path.join(CSRC, h)) for h in HEADERS
               if os.path.exists(os.path.join(CSRC, h))]
              + [os.path.getmtime(os.path.join(ROOT, "include", "qs.h")), os.path.getmtime(__file__)])
    for src in sources():
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        objs.append(obj)
        if incremental and os.path.exists(obj) and os.path.getmtime(obj) > max(hdr, os.path.getmtime(src)):
            continue
        if src.endswith(".hip"):
            cmd = [HIPCC] + COMMON + DEVICE_FLAGS + ["-x", "hip", "-c", src, "-o", obj]
        else:  # host-only C++ against the HIP runtime API
            cmd = [HIPCC] + COMMON + HOST_FLAGS + ["-x", "c++", "-c", src, "-o", obj]
        procs.append((src, cmd))
    t0 = time.time()
    running = []
    for src, cmd in procs:
        while len(running) >= jobs:
            _wait_one(running)
        if verbose:
            print("[build] hipcc", os.path.basename(src), flush=True)
        running.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    while running:
        _wait_one(running)
    tmp = LIB + ".tmp%d" % os.getpid()
    link = [HIPCC] + DEVICE_FLAGS + ["-shared", "-fPIC", "-o", tmp] + objs
    out = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if out.returncode:
        raise RuntimeError("link failed:\n" + out.stdout)
    os.replace(tmp, LIB)
    if verbose:
        print("[build] libqs.so linked in %.1fs" % (time.time() - t0), flush=True)
    return LIB


def _wait_one(running):
    src, p = running.pop(0)
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l]
    if p.returncode:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, "\n".join(lines)))
    if lines and any("warning" in l for l in lines):
        sys.stdout.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv[1:])

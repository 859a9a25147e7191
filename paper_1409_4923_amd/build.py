"""Build libbmotor.so in-tree with hipcc for gfx950.

Usage: python -m paper_1409_4923_amd.build   (or build_library() from Python)
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbmotor.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 instructions are disabled for every HIP translation unit.
COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + INCLUDE, "-I" + CSRC]

# Translation units and their extra flags.  The reduction / host code keeps
# error-free transformations intact, so FMA contraction is off there.
SOURCES = [
    ("abi.hip", ["-ffp-contract=off"]),
    ("paths_f32_od.hip", []),
    ("paths_f32_in.hip", []),
    ("paths_f64_od.hip", []),
    ("paths_f64_in.hip", []),
    ("scan.hip", ["-ffp-contract=off"]),
    ("scan_f32_od.hip", []),
    ("scan_f32_in.hip", []),
    ("scan_f64_od.hip", []),
    ("scan_f64_in.hip", []),
    ("mlp.hip", []),
]

# The vector-ALU issue-rate probe (a measurement aid of the benchmark, not part of
# the method) is a library of its own.
PROBE_SRC = "probe.hip"
PROBE_LIB = os.path.join(HERE, "libbmprobe.so")


def sources() -> list[str]:
    return [os.path.join(CSRC, s) for s, _ in SOURCES]


def build_library(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every translation unit (in parallel), link libbmotor.so and the
    benchmark's libbmprobe.so."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    objs, procs = [], []
    pending = list(SOURCES) + [(PROBE_SRC, [])]
    while pending or procs:
        while pending and len(procs) < jobs:
            src, extra = pending.pop(0)
            obj = os.path.join(BUILD_DIR, src.replace(".hip", ".o"))
            cmd = [HIPCC] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
        src, p = procs.pop(0)
        out, _ = p.communicate()
        if p.returncode != 0:
            for _, q in procs:
                q.wait()
            raise RuntimeError("hipcc failed on %s:\n%s" % (src, out.decode(errors="replace")))
        if verbose and out:
            print(out.decode(errors="replace"), flush=True)
    probe_obj = os.path.join(BUILD_DIR, PROBE_SRC.replace(".hip", ".o"))
    for lib, parts in ((LIB, [o for o in objs if o != probe_obj]), (PROBE_LIB, [probe_obj])):
        tmp = lib + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + parts
        subprocess.check_call(cmd)
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))

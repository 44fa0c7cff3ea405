"""Build libns.so (the HIP library behind include/ns.h) for gfx950, in-tree.

    python -m paper_2509_24949_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libns.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in (
    "ns_api.hip", "ns_server.hip", "ns_kernels.hip", "ns_slice_d1.hip", "ns_slice_d2.hip", "ns_slice_d3.hip",
    "ns_slice_m1.hip", "ns_slice_m2.hip", "ns_slice_m3.hip", "ns_slice_p64.hip", "ns_slice_p128.hip", "ns_walk.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
RATES_SRC = os.path.join(HERE, "csrc", "unit_rates.hip")
RATES = os.path.join(HERE, "unit_rates")

COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]
# device pass only: no packed FP32 instructions anywhere in the device code
DEVICE_ONLY = ["--cuda-device-only", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _objects(src: str, objdir: str) -> tuple[list[str], list[str], str]:
    """The two compile commands of one source: the device pass writes the
    code-object bundle, the host pass embeds it in the host object."""
    base = os.path.join(objdir, os.path.basename(src))
    fatbin, obj = base + ".hipfb", base + ".o"
    dev = [HIPCC, *COMMON, *DEVICE_ONLY, "-c", "-o", fatbin, src]
    host = [HIPCC, *COMMON, "--cuda-host-only", "-Xclang", "-fcuda-include-gpubinary", "-Xclang", fatbin,
            "-c", "-o", obj, src]
    return dev, host, obj


def build(verbose: bool = False) -> str:
    """Compile each source (device pass, then host pass) in parallel, then
    link the library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    jobs = [_objects(src, objdir) for src in SOURCES]

    def run_all(cmds):
        procs = []
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd))
        for p in procs:
            if p.wait() != 0:
                raise subprocess.CalledProcessError(p.returncode, "hipcc")

    run_all([dev for dev, _, _ in jobs])
    run_all([host for _, host, _ in jobs])
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[obj for _, _, obj in jobs],
           "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    # the vector-unit rate probe the benchmark's peaks rest on (bench.py --unit-rates)
    dev, host, obj = _objects(RATES_SRC, objdir)
    run_all([dev])
    run_all([host])
    cmd = [HIPCC, "--offload-arch=gfx950", "-o", RATES + ".tmp", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(RATES + ".tmp", RATES)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

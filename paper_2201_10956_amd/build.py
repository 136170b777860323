"""Builds libepi3.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libepi3.so")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off (vector float code is scalar FP32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def build(out: str = LIB, extra=(), verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out_lines = [l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        sys.stderr.write("\n".join(out_lines) + "\n")
        raise RuntimeError("hipcc failed")
    if out_lines and verbose:
        print("\n".join(out_lines))
    os.replace(tmp, out)
    return out


PEAK_SRC = os.path.join(PKG, "peak", "peak.hip")
PEAK_LIB = os.path.join(PKG, "peak", "libepi3_peak.so")


def build_peak(out: str = PEAK_LIB) -> str:
    """The peak-rate microbenchmarks (matrix-core and vector-ALU chains)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *FLAGS, PEAK_SRC, "-o", tmp]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("hipcc failed (peak microbenchmarks)")
    os.replace(tmp, out)
    return out


HOST_SRC = os.path.join(PKG, "host", "epi3_host.c")
HOST_LIB = os.path.join(PKG, "host", "libepi3_host.so")


def build_host(out: str = HOST_LIB) -> str:
    """The host-CPU scan (a baseline beside the GPU library): gcc, OpenMP;
    the vector loops carry their own target attributes and are chosen at run
    time from the CPU's features, so the library runs on any x86-64 host."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra",
           "-I", os.path.join(ROOT, "include"), HOST_SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_host())
    print(build_peak())

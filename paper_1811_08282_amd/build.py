"""Build step of the HIP library: compiles ``csrc/`` into ``libswept.so``.

Run as ``python -m paper_1811_08282_amd.build``.  Every source is compiled
for gfx950 with contraction off (the swept and classic kernels and the oracle
must see the same IEEE operation sequence), without fast-math (Kahan
compensation and the NaN-aware limiter depend on it), and with packed FP32
instructions disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libswept.so")
SOURCES = ["api.cpp", "tune_batch.cpp", "host_share.cpp", "heat.hip", "euler.hip", "euler_flat.hip",
           "ks.hip", "batch.hip"]

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError("hipcc failed building libswept.so")
    noise = [ln for ln in proc.stderr.splitlines()
             if ln.strip() and "packed-fp32-ops" not in ln and "is not a recognized feature" not in ln]
    if verbose and noise:
        sys.stderr.write("\n".join(noise) + "\n")
    os.replace(tmp, LIB)
    return LIB


def build_test_helpers(verbose: bool = False) -> None:
    """tests/librn_check.so: the kernel tests/test_gpu_rn_ops.py runs the
    rounded-to-nearest sequences of the Euler tiles with; tests/lds_probe:
    the LDS throughput probe whose rates bench.py's LDS roofline uses."""
    exe_flags = [f for f in HIP_FLAGS if f not in ("-fPIC", "-shared")]
    for src, out, flags in (("rn_check.hip", "librn_check.so", HIP_FLAGS),
                            ("lds_probe.hip", "lds_probe", exe_flags)):
        src = os.path.join(ROOT, "tests", src)
        out = os.path.join(ROOT, "tests", out)
        cmd = [hipcc(), *flags, "-o", out + ".tmp", src]
        if verbose:
            print(" ".join(cmd), flush=True)
        proc = subprocess.run(cmd, capture_output=True, text=True)
        if proc.returncode != 0:
            sys.stderr.write(proc.stdout + proc.stderr)
            raise RuntimeError(f"hipcc failed building {out}")
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)

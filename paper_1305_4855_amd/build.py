"""Build step of the HIP library: hipcc for gfx950 into the package directory.

    python -m paper_1305_4855_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "hough.hip")]
OUT = os.path.join(HERE, "libhough.so")
# roofline micro-benchmarks (LDS atomic / read / write rates, HBM copy): a library of their own
PROBE_SOURCES = [os.path.join(HERE, "csrc", "roofline_probe.hip")]
PROBE_OUT = os.path.join(HERE, "libroofline_probe.so")
ARCH = os.environ.get("HOUGH_OFFLOAD_ARCH", "gfx950")

# -ffp-contract=off keeps the host-side table in plain IEEE double (no fused
# multiply-add); packed FP32 instructions are disabled for all device code.
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")]


def _hipcc(sources, out, verbose):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *FLAGS, "-o", tmp, *sources]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    _hipcc(PROBE_SOURCES, PROBE_OUT, verbose)
    return _hipcc(SOURCES, OUT, verbose)


if __name__ == "__main__":
    print(build(verbose=True))

"""Build libmd.so in-tree with hipcc for gfx950.

    python -m paper_2109_10876_amd.build
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# -packed-fp32-ops: keep the compiler from forming packed FP32 VALU ops.
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall",
]


def sources():
    return sorted(glob.glob(os.path.join(_HERE, "csrc", "*.hip")))


def build_library(verbose=False):
    """Compile every csrc/*.hip into paper_2109_10876_amd/libmd.so."""
    out = os.path.join(_HERE, "libmd.so")
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(_ROOT, "include"), *sources(), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops' is not a recognized feature"
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if noise not in l]
    if verbose or r.returncode != 0:
        print("\n".join(msgs), file=sys.stderr)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode})")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))

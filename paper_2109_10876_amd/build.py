"""Build libmd.so in-tree with hipcc for gfx950.

    python -m paper_2109_10876_amd.build

Each csrc/*.hip is compiled to an object of its own (in parallel), then the
objects are linked into paper_2109_10876_amd/libmd.so.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# -packed-fp32-ops: keep the compiler from forming packed FP32 VALU ops.
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall",
]
_NOISE = "packed-fp32-ops' is not a recognized feature"


def sources():
    return sorted(glob.glob(os.path.join(_HERE, "csrc", "*.hip")))


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if _NOISE not in l]
    return r.returncode, "\n".join(msgs)


def build_library(verbose=False, jobs=None):
    """Compile every csrc/*.hip and link paper_2109_10876_amd/libmd.so."""
    out = os.path.join(_HERE, "libmd.so")
    tmp = out + ".tmp"
    inc = ["-I", os.path.join(_ROOT, "include")]
    jobs = jobs or min(16, os.cpu_count() or 1)
    with tempfile.TemporaryDirectory(prefix="libmd_build_") as od:
        srcs = sources()
        objs = [os.path.join(od, os.path.basename(f) + ".o") for f in srcs]
        cmds = [[HIPCC, *FLAGS, *inc, "-c", f, "-o", o] for f, o in zip(srcs, objs)]
        with ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(_run, cmds))
        bad = [(f, m) for f, (rc, m) in zip(srcs, results) if rc != 0]
        for f, (rc, m) in zip(srcs, results):
            if m and (verbose or rc != 0):
                print(f"{os.path.basename(f)}:\n{m}", file=sys.stderr)
        if bad:
            raise RuntimeError("hipcc failed on " + ", ".join(os.path.basename(f) for f, _ in bad))
        rc, m = _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
        if m and (verbose or rc != 0):
            print(m, file=sys.stderr)
        if rc != 0:
            raise RuntimeError(f"link failed ({rc})")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))

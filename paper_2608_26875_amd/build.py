"""Build the HIP shared library libems.so in-tree for gfx950.

Every HIP and C++ source under csrc/ is compiled by hipcc into one shared
object next to this file.  Packed FP32 instructions are disabled for the
device code (plain FP32/FP64 arithmetic only).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libems.so")
ARCH = os.environ.get("EMS_OFFLOAD_ARCH", "gfx950")


def sources():
    src = sorted(glob.glob(os.path.join(HERE, "csrc", "*.cpp")) +
                 glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    return src


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object in parallel, then link libems.so."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    flags = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument", "-I", os.path.join(HERE, "..", "include")]
    procs = []
    objs = []
    for s in sources():
        o = os.path.join(objdir, os.path.basename(s) + ".o")
        objs.append(o)
        cmd = [hipcc, *flags, "-x", "hip", "-c", s, "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _drain(procs)
    _drain(procs)
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode())
    os.replace(tmp, LIB)
    return LIB


def _drain(procs):
    errs = []
    while procs:
        s, p = procs.pop(0)
        out, _ = p.communicate()
        if p.returncode != 0:
            errs.append(f"{os.path.basename(s)}:\n{out.decode()}")
        else:
            msg = out.decode()
            # hipcc's host pass does not know the packed-fp32 feature flag
            lines = [ln for ln in msg.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
            if lines and os.environ.get("EMS_BUILD_VERBOSE"):
                print("\n".join(lines), file=sys.stderr)
    if errs:
        raise RuntimeError("compile failed:\n" + "\n".join(errs))


if __name__ == "__main__":
    print(build(verbose=True))

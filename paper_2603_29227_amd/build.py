"""Build libksdf.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libksdf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["api.hip", "fit.hip", "index.hip", "query.hip", "query_fast.hip", "query_split64_wave.hip",
           "query_split64_lane.hip", "query_split256_wave.hip", "query_split256_lane.hip",
           "query_pairs.hip", "fused.hip", "backward.hip", "bhm.hip", "noalloc.hip"]
HOST_SOURCES = ["cells_host.cpp"]

# Packed FP32 VALU forms are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-munsafe-fp-atomics"]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES + HOST_SOURCES]


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every translation unit and link libksdf.so (always recompiles)."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for s in SOURCES:
        o = os.path.join(objdir, os.path.basename(s) + ".o")
        cmd = [HIPCC, *DEVICE_FLAGS, "-c", os.path.join(CSRC, s), "-o", o]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(o)
    for s in HOST_SOURCES:
        o = os.path.join(objdir, os.path.basename(s) + ".o")
        cmd = [HIPCC, "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-x", "c++", "-c",
               os.path.join(CSRC, s), "-o", o]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(o)
    failed = False
    for cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed = True
            sys.stderr.write(" ".join(cmd) + "\n" + text)
        elif verbose and text.strip():
            sys.stderr.write(text)
    if failed:
        raise RuntimeError("libksdf build failed")
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
                           "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

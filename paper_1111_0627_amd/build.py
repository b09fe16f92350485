"""Builds the HIP library ``libocm.so`` (gfx950) in-tree with hipcc."""

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libocm.so")
SOURCES = ["kernels.hip", "solver.hip", "batch.hip", "general.hip", "multichain.hip"]
ARCH = os.environ.get("OCM_OFFLOAD_ARCH", "gfx950")

# Packed-FP32 instructions are switched off for all device code.
HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False, jobs: int = 4) -> str:
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = ["hipcc", *HIPFLAGS, "-I", INCLUDE, "-I", CSRC, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), cmd))
        objs.append(obj)
    for p, cmd in procs:
        _, err = p.communicate()
        err = "\n".join(l for l in err.splitlines()
                        if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed: {' '.join(cmd)}\n{err}")
        if verbose and err.strip():
            print(err, flush=True)
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs,
           "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build the HIP library libsanns.so in-tree for gfx950 with hipcc.

Each source is compiled to an object file in its own hipcc process (in
parallel), then the objects are linked into the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsanns.so")
SOURCES = ["kernels.hip", "mfma.hip", "kmeans.hip", "sanns_api.hip", "params.cpp"]
ARCH = os.environ.get("SANNS_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    with tempfile.TemporaryDirectory(prefix="sanns_build_") as tmpdir:
        objs, procs = [], []
        for s in SOURCES:
            obj = os.path.join(tmpdir, os.path.splitext(s)[0] + ".o")
            cmd = [hipcc] + FLAGS + ["-c", os.path.join(CSRC, s), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((s, subprocess.Popen(cmd)))
            objs.append(obj)
        failed = [s for s, p in procs if p.wait() != 0]
        if failed:
            raise subprocess.CalledProcessError(1, "hipcc -c " + " ".join(failed))
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

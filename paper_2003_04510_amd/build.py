"""Build the HIP library (gfx950) in-tree: paper_2003_04510_amd/libhe_mi355x.so.

Every source compiles to an object of its own, in parallel (the stage
kernels are split by word type and ring degree over the launch_*.hip
units), then the objects are linked."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhe_mi355x.so")
SOURCES = ["he_lib.hip", "launch_u64_n16.hip", "launch_u64_n16b.hip", "launch_u64_n16r.hip", "launch_w32_n16.hip",
           "launch_w32.hip", "launch_u64_n17.hip", "launch_u64_small.hip", "host_math.cpp", "server.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=off", "-fno-strict-aliasing",
         "-Wall", "-Wno-unused-function"]


def _jobs() -> int:
    n = int(os.environ.get("MAX_JOBS", "0") or 0) or (os.cpu_count() or 4)
    return max(1, min(n, 16, len(SOURCES)))


def build(verbose: bool = False) -> str:
    with tempfile.TemporaryDirectory(prefix="he_build_") as tmpd:
        def compile_one(src):
            obj = os.path.join(tmpd, os.path.splitext(src)[0] + ".o")
            r = subprocess.run([HIPCC] + FLAGS + ["-c", "-o", obj, os.path.join(CSRC, src)], capture_output=True,
                               text=True)
            return src, obj, r
        with cf.ThreadPoolExecutor(_jobs()) as ex:
            results = list(ex.map(compile_one, SOURCES))
        for src, _, r in results:
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError("hipcc failed on %s" % src)
            if verbose:
                sys.stderr.write(r.stderr)
        tmp = LIB + ".tmp%d" % os.getpid()
        r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for _, o, _ in results],
                           capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking %s" % LIB)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

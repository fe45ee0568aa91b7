"""Build ``libsgml.so`` (the HIP library behind include/sgml.h) for gfx950.

Compiles in-tree with hipcc, one object per source in parallel, then links;
the library lands next to this file so that the binding (and the round-trip
to a GPU host) finds it without any install step.  Objects go to a
temporary directory, so every call compiles from source.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsgml.so")
SOURCES = ["sgml_visit2d_f32.hip", "sgml_visit2d_f64.hip", "sgml_visit2d_f32r.hip", "sgml_visit2d_f64r.hip",
           "sgml_kernels.hip", "sgml_sweep3d.hip", "sgml_plan.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC,
]
LDFLAGS = ["--offload-arch=gfx950", "-fPIC", "-shared"]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False) -> str:
    with tempfile.TemporaryDirectory(prefix="sgml_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in sources()]

        def compile_one(pair):
            src, obj = pair
            cmd = [HIPCC] + CFLAGS + ["-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)

        jobs = min(len(objs), max(1, min(8, os.cpu_count() or 1)))
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            list(ex.map(compile_one, zip(sources(), objs)))
        tmp = LIB + ".tmp"
        cmd = [HIPCC] + LDFLAGS + ["-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

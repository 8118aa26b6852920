"""Build libheat.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2307_01117_amd.build
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libheat.so")
SOURCES = ["kernels.hip", "kernels_xchg.hip", "kernels_xchg2.hip", "kernels_resident.hip",
           "kernels_f32.hip",
           "kernels_f32c.hip",
           "batch_kernels.hip", "runtime.hip", "batch.hip", "server.hip", "tune.hip"]

# Per-source additions: the binary32 kernels are scheduled for instruction-
# level parallelism (their per-cell operation chains pair better when
# neighbouring cells interleave); the order changes no result.  Binary64
# instructions do not pair, so its kernels keep the default schedule.
SOURCE_FLAGS = {
    "kernels_f32.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
    "kernels_f32c.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
}

def source_digest() -> str:
    """sha256 over the library's sources: every file under csrc/, the public
    header and this build script (its flags), each preceded by its name, in
    name order.  It is compiled into the library (heat_version) and compared
    by the binding at load time, so a library built from other sources is
    refused instead of silently run."""
    h = hashlib.sha256()
    files = [os.path.join("csrc", f) for f in sorted(os.listdir(CSRC))
             if f.endswith((".hip", ".h"))]
    paths = [(f, os.path.join(HERE, f)) for f in files]
    paths.append(("include/heat.h", os.path.join(ROOT, "include", "heat.h")))
    paths.append(("build.py", os.path.abspath(__file__)))
    for name, path in paths:
        h.update(name.encode() + b"\0")
        with open(path, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    return h.hexdigest()


HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # binary64 bit-parity: no contraction beyond the explicit fma in the kernels
    "-ffp-contract=off",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-pthread",
]


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link the shared
    library; always compiles from scratch."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmpdir = tempfile.mkdtemp(prefix="heat_build_")
    try:
        inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
               f"-DHEAT_SOURCE_SHA256=\"{source_digest()}\""]
        objs = [os.path.join(tmpdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[hipcc, *HIPCC_FLAGS, *SOURCE_FLAGS.get(s, []), *inc, "-c", os.path.join(CSRC, s),
                 "-o", o] for s, o in zip(SOURCES, objs)]

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)

        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "0")) or os.cpu_count() or 1, 8))
        with ThreadPoolExecutor(jobs) as ex:
            list(ex.map(run, cmds))
        tmp = LIB + ".tmp"
        run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", *objs,
             "-L/opt/rocm/lib", "-lhsa-runtime64", "-o", tmp])
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build the gfx950 HIP library (libpisco.so) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpisco.so")
# translation units of libpisco.so (valu_probe.hip is a separate program)
SOURCES = ["conv_kernel.hip", "mlp_kernels.hip", "map_kernel.hip", "order_kernel.hip", "sht_kernel.hip",
           "sidelobe_kernel.hip", "runtime.cpp", "mlp_runtime.cpp", "sht_runtime.cpp", "map_runtime.cpp",
           "sidelobe_runtime.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Every HIP translation unit: gfx950 only, -O3, and no packed FP32 instructions.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose: bool = False) -> str:
    """Compile every translation unit (in parallel) and link libpisco.so."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    jobs = []
    for src in sources():
        obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
        jobs.append((obj, [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", src, "-o", obj]))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))

    def compile_one(job):
        obj, cmd = job
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(compile_one, jobs))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    # the vector-ALU issue-rate probe the benchmark runs beside the roofline
    probe = os.path.join(HERE, "valu_probe")
    subprocess.check_call([HIPCC, *[f for f in FLAGS if f != "-fPIC"], os.path.join(CSRC, "valu_probe.hip"), "-o",
                           probe + ".tmp"])
    os.replace(probe + ".tmp", probe)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build the gfx950 shared library libsce.so in-tree with hipcc.

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection turned off (-Xclang -target-feature -Xclang -packed-fp32-ops), and
linked into ``paper_1508_07344_amd/libsce.so`` next to this file.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsce.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["kernels.hip", "kernels_mfma.hip", "kernels_serve.hip", "kernels_tent.hip",
           "kernels_small.hip", "sce_api.hip", "sce_server.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))
    # surface warnings other than the host pass's note about the packed-fp32 feature
    for line in (r.stderr or "").splitlines():
        if "packed-fp32-ops" in line or not line.strip():
            continue
        if "warning" in line:
            sys.stderr.write(line + "\n")


PEAK_SOURCE = "peak_probe.hip"
PEAK_LIB = os.path.join(HERE, "libsce_peak.so")


def build(verbose: bool = False) -> str:
    """Compile every source and link libsce.so and the throughput probes'
    libsce_peak.so (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
        cmds.append([HIPCC, *COMMON_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
        if verbose:
            print(" ".join(cmds[-1]))
    ptmp = PEAK_LIB + ".tmp%d" % os.getpid()
    cmds.append([HIPCC, *COMMON_FLAGS, "-shared", os.path.join(CSRC, PEAK_SOURCE), "-o", ptmp])
    # one hipcc per source, in parallel (each is single-threaded)
    jobs = max(1, min(len(cmds), os.cpu_count() or 1, 16))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, c) for c in cmds]:
            f.result()
    os.replace(ptmp, PEAK_LIB)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    _run(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the HIP library libstf.so for gfx950 in-tree (next to this file).

The translation units compile in parallel into objects in a temporary
directory (the forward kernels of each filter are one unit, the rest of the
library another, the footprint generator a third) and are then linked."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libstf.so")
SOURCES = [os.path.join(CSRC, name) for name in
           ("stf_forward_bicubic.hip", "stf_forward_bilinear.hip", "stf.hip", "footprints.hip")]

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay disabled in all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core accumulators in ordinary VGPRs: the decoder's ReLU and BF16
    # packing read them directly instead of copying them out of AGPRs
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libstf.so")
    return path


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}: {' '.join(cmd[-3:])}")


def build(verbose: bool = False) -> str:
    """Compile libstf.so (always recompiles). Returns its path."""
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="stf_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in SOURCES]
        jobs = [[cc, *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", "-o", obj, src] for src, obj in zip(SOURCES, objs)]
        with ThreadPoolExecutor(max_workers=min(len(jobs), max(1, os.cpu_count() or 1))) as pool:
            for f in [pool.submit(_run, j, verbose) for j in jobs]:
                f.result()
        tmp = LIB + ".tmp"
        _run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build libttc.so (all HIP kernels and the host runtime) for gfx950 with hipcc.

Every call recompiles every source.  Usage: python paper_2109_00626_amd/build.py
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libttc.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions in generated GPU code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


# Per-source extra flags.  The LDS-resident sweep keeps its accumulators in
# ordinary vector registers (MFMA results in VGPRs rather than accumulation
# registers), which avoids copies between the two register files when every
# operand buffer is live.
EXTRA = {
    "batched_lds.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "pair_lds.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def _compile(src: str, build_dir: str = BUILD, defines=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + [f"-D{d}" for d in defines] + EXTRA.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = True, out: str = LIB, build_dir: str = BUILD, defines=()) -> str:
    """Compile every source and link `out` (defines: extra -D macros, for
    variant builds compared by timing)."""
    os.makedirs(build_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, build_dir, defines), srcs))
    LIB_OUT = out
    tmp = LIB_OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB_OUT)
    if verbose:
        print(f"built {LIB_OUT} from {len(srcs)} sources")
    return LIB_OUT


if __name__ == "__main__":
    build()
    sys.exit(0)

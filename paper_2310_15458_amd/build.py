"""Build librss.so in-tree with hipcc for gfx950.

    python -m paper_2310_15458_amd.build

Objects go to paper_2310_15458_amd/_build/, the library to
paper_2310_15458_amd/librss.so.  Every call rebuilds.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "librss.so")
BUILD = os.path.join(HERE, "_build")

SOURCES = ["rss_kernels.hip", "rss_id.hip", "rss_residual.hip", "rss_fft.hip", "rss_host.cpp", "rss_server.cpp"]

FLAGS = [
    "-O3", "-fPIC", "-std=c++17", "--offload-arch=gfx950",
    # keep packed FP32 instructions out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


# per-source additions: the residual's matrix-core accumulators stay in
# ordinary vector registers (the accumulation registers would be copied to and
# from on every iteration of its branchy source loop)
EXTRA_FLAGS = {"rss_residual.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
               # double-double arithmetic: each operation rounded on its own
               "rss_id.hip": ["-ffp-contract=off"]}


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [hipcc(), "-c", *FLAGS, *EXTRA_FLAGS.get(src, []), "-I", os.path.join(os.path.dirname(HERE), "include"), "-x", "hip",
           os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

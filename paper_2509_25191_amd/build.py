"""Compile the vggtx HIP library for gfx950 into ``libvggtx.so`` (in-tree).

Usage: python -m paper_2509_25191_amd.build   (or call ``build()``).
Every source is compiled each time; objects go to ``_build/`` beside the
package and are linked into the shared library next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libvggtx.so")
BUILD_DIR = os.path.join(os.path.dirname(PKG), "_build")
SOURCES = ["attention.hip", "gemm.hip", "elementwise.hip", "embed.hip", "ga.hip", "runtime.hip"]
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 VALU instructions stay disabled (see the library notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the vggtx library needs ROCm's hipcc to build")


# Per-file additions for attention.hip:
#  * no float operation there sees a NaN (masked scores are -inf; the FP8
#    kernel's overflow NaN is tested on its bits), so max() needs no NaN
#    quieting of the MFMA results; infinities stay honoured;
#  * machine sinking off: it would move the FP8 kernel's MFMAs of the next
#    query block (and the P V MFMAs of the previous one) below the overflow
#    branch, out of the exponentials they are scheduled between.
FILE_FLAGS = {"attention.hip": ["-fno-honor-nans", "-mllvm", "-disable-machine-sink"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, *FILE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

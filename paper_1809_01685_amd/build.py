"""Build libtnslq.so (HIP, gfx950) in-tree.

    python -m paper_1809_01685_amd.build [--jobs N]

Compiles every ``csrc/*.hip`` translation unit with hipcc for gfx950 and links
them into ``paper_1809_01685_amd/libtnslq.so``, and ``peak/peak.hip`` (the
achievable-peak loops the measurements report against) into
``paper_1809_01685_amd/libtnslq_peak.so``.  Packed-FP32 instructions are
disabled for all device code.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libtnslq.so")
PEAK_SRC = os.path.join(PKG, "peak", "peak.hip")
PEAK_OUT = os.path.join(PKG, "libtnslq_peak.so")
# sources built with the matrix instructions' VGPR form (see _compile)
VGPR_FORM = ("peak.hip", "mps.hip", "entropy.hip", "mlp.hip")
BUILD = os.path.join(PKG, "_build")

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-command-line-argument",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    # loops that carry matrix-instruction accumulators from one iteration to
    # the next: in the accumulator-register form the compiler copied them
    # between register files every iteration
    extra = ["-mllvm", "-amdgpu-mfma-vgpr-form=1"] if os.path.basename(src) in VGPR_FORM else []
    cmd = [hipcc(), *FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    # hipcc's host pass warns about the device-only target feature; drop it
    err = "\n".join(line for line in r.stderr.splitlines() if "packed-fp32-ops" not in line and line.strip())
    if err:
        sys.stderr.write(err + "\n")
    return obj


def _link(objs, out: str, extra=()) -> None:
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, *extra]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)


def build(jobs: int = 8, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + [PEAK_SRC]
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(_compile, srcs))
    # roctx ranges mark the phases of an estimate for rocprofv3 --marker-trace
    _link(objs[:-1], OUT, ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"])
    _link(objs[-1:], PEAK_OUT)
    if verbose:
        print(f"built {OUT}")
        print(f"built {PEAK_OUT}")
    return OUT


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    a = ap.parse_args()
    build(a.jobs)

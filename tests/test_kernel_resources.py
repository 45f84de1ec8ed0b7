"""The contraction kernels must keep their staging and accumulators in
registers: a kernel that falls back to per-lane scratch memory runs several
times slower without any change in its results, so only this check sees it."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1809_01685_amd", "csrc")


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_contraction_kernels_use_no_scratch(tmp_path):
    cmd = [_hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "--cuda-device-only", "-c",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-Rpass-analysis=kernel-resource-usage",
           os.path.join(CSRC, "gemm_mfma.hip"), "-o", str(tmp_path / "g.o")]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    usage, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            usage[name] = int(m.group(1))
    gemms = {k: v for k, v in usage.items() if "k_cgemm_nt_mfma" in k}
    assert len(gemms) == 3, usage
    assert all(v == 0 for v in gemms.values()), gemms

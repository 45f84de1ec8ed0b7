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
    gemms = {k: v for k, v in usage.items() if "k_cgemm_" in k}
    assert len(gemms) == 4, usage
    assert all(v == 0 for v in gemms.values()), gemms


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
@pytest.mark.parametrize("src,instrs", [("mps.hip", ("v_mfma_f64_16x16x4", "v_mfma_f32_16x16x4")),
                                        ("entropy.hip", ("v_mfma_f64_16x16x4",)),
                                        ("mlp.hip", ("v_mfma_f32_16x16x32_bf16",))])
def test_matrix_loops_keep_accumulators_in_vgprs(tmp_path, src, instrs):
    # the MPS complex products, the entropy's eight-vector column MAC and the
    # surrogate network's products carry matrix-instruction accumulators
    # across their reduction loops; built as
    # the library builds them (VGPR form) they use no accumulation registers,
    # hence no copies between register files, and no scratch
    from paper_1809_01685_amd import build as b
    out = tmp_path / "m.s"
    cmd = [_hipcc(), *[f for f in b.FLAGS if f != "-fPIC"], "-mllvm", "-amdgpu-mfma-vgpr-form=1",
           "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    asm = out.read_text()
    assert all(i in asm for i in instrs)
    assert "v_accvgpr" not in asm
    spills = [int(x) for x in re.findall(r"\.(?:vgpr|sgpr)_spill_count:\s+(\d+)", asm)]
    assert spills and max(spills) == 0
    scratch = [int(x) for x in re.findall(r"\.private_segment_fixed_size:\s+(\d+)", asm)]
    assert scratch and max(scratch) == 0
    # and the build applies that form to this file
    assert src in b.VGPR_FORM


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_quadrature_and_fit_use_no_scratch(tmp_path):
    # the quadrature keeps each thread's tridiagonal and first-row arrays in
    # LDS (per-lane scratch made it 1.7x slower), and the fit's per-lane state
    # stays in registers
    from paper_1809_01685_amd import build as b
    cmd = [_hipcc(), *[f for f in b.FLAGS if f != "-fPIC"], "--cuda-device-only", "-c",
           "-Rpass-analysis=kernel-resource-usage", os.path.join(CSRC, "lanczos.hip"), "-o", str(tmp_path / "l.o")]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    usage, lds, name = {}, {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            usage[name] = int(m.group(1))
        m = re.search(r"LDS Size \[bytes/block\]: (\d+)", line)
        if m and name:
            lds[name] = int(m.group(1))
    quad = [k for k in usage if "k_quadrature" in k]
    fit = [k for k in usage if re.search(r"5k_fitE", k)]
    assert len(quad) == 1 and len(fit) == 1, usage
    assert usage[quad[0]] == 0 and usage[fit[0]] == 0
    assert 0 < lds[quad[0]] <= 160 * 1024


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_one_read_kernel_keeps_partial_y_in_registers(tmp_path):
    # the one-read matvec holds its rows of the partial Y, of the probe and of
    # the slabs in flight in registers across every slab it streams; a spill
    # would put them in per-lane scratch memory, i.e. back in HBM
    from paper_1809_01685_amd import build as b
    cmd = [_hipcc(), *[f for f in b.FLAGS if f != "-fPIC"], "--cuda-device-only", "-c",
           "-Rpass-analysis=kernel-resource-usage", os.path.join(CSRC, "fused.hip"), "-o", str(tmp_path / "f.o")]
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
    fused = {k: v for k, v in usage.items() if "k_pt_rows" in k}
    assert len(fused) == 2, usage
    assert all(v == 0 for v in fused.values()), fused

"""Host-side logic of bench.py: the counter summary and its staleness check."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write(path, sha):
    path.write_text("# comment = ignored\n"
                    f"kernel_source_sha256 = {sha}\n"
                    "kernel_sources = paper_1809_01685_amd/csrc/gemm_mfma.hip paper_1809_01685_amd/csrc/operands.h\n"
                    "contraction2_hbm_bytes = 1.5e+11\n"
                    "contraction2_mfma_busy_frac = 0.7\n"
                    "contraction2_avg_clock_ghz = 2.0\n")


def test_counter_summary_parses_and_checks_kernel_sources(tmp_path, monkeypatch):
    srcs = ["paper_1809_01685_amd/csrc/gemm_mfma.hip", "paper_1809_01685_amd/csrc/operands.h"]
    p = tmp_path / "c.txt"
    _write(p, bench.kernel_source_sha256(srcs))
    monkeypatch.setattr(bench, "COUNTERS", str(p))
    c = bench.read_counters(str(p))
    assert "comment" not in c and c["contraction2_hbm_bytes"] == "1.5e+11"
    f = bench.counter_figures("haar30", "bf16x3", "contraction2")
    assert f == {"hbm_bytes": 1.5e11, "mfma_busy_frac": 0.7, "avg_clock_ghz": 2.0}
    # other workload, other precision, a contraction without figures
    assert bench.counter_figures("haar26", "bf16x3", "contraction2") is None
    assert bench.counter_figures("haar30", "fp32", "contraction2") is None
    assert bench.counter_figures("haar30", "bf16x3", "contraction1") is None
    # counters taken on other kernel sources are stale
    _write(p, "0" * 64)
    assert bench.counter_figures("haar30", "bf16x3", "contraction2") is None


def test_committed_counter_summary_is_well_formed():
    c = bench.read_counters()
    for k in ("kernel_source_sha256", "fetch_scale", "write_scale", "contraction1_hbm_bytes",
              "contraction2_hbm_bytes"):
        assert k in c
    assert float(c["fetch_scale"]) > 0 and float(c["write_scale"]) > 0

"""Host logic of bench.py (no GPU): the one-GPU guard and the hash-guarded
reading of the committed rocprofv3 counter summary."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counter_summary_fields():
    if bench.measured_traffic("k_pair_vjp") is None:
        pytest.skip("the counter summary was taken on other pair-kernel code")
    for k in ("k_pair_force", "k_pair_vjp"):
        b = bench.measured_traffic(k)
        assert isinstance(b, int) and b > 0
        c = bench.measured_counters(k, 10.0)
        assert set(c) == {"valu_busy", "valu_lane_utilisation",
                          "lds_bank_conflict_frac", "waves_per_simd", "hbm_tb_per_s"}
        assert 0.0 < c["valu_busy"] <= 1.0 and 0.0 < c["valu_lane_utilisation"] <= 1.0
        assert c["hbm_tb_per_s"] == pytest.approx(b / 1e-2 / 1e12, rel=1e-3)
    assert bench.measured_traffic("k_unknown") is None


def test_counters_are_withheld_for_other_sources(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic("k_pair_vjp") is None
    assert bench.measured_counters("k_pair_vjp", 10.0) is None


def test_source_hash_ignores_comments_and_blank_lines(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1211_4864_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in bench.KERNEL_SOURCES:
        src = open(os.path.join(ROOT, "paper_1211_4864_amd", "csrc", name)).read()
        (csrc / name).write_text(src)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    pair = csrc / "pair.hip"
    pair.write_text("// a new comment\n\n" + pair.read_text().replace(
        "namespace hsr {", "namespace hsr {  // trailing comment", 1))
    assert bench.kernel_source_hash() == h0
    pair.write_text(pair.read_text().replace("namespace hsr {", "namespace hsr { ", 1)
                    + "\nint changed_code;\n")
    assert bench.kernel_source_hash() != h0

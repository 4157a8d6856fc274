"""Host-side checks of bench.py (no GPU): the multi-GPU refusal, the
algorithmic bytes per update, and the rule that stored counter figures are
used only while the kernel sources they were taken on are unchanged."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_update():
    # 8 link reads and 1 write per update of an 18-real SU(3) matrix: 9 x 18 reals
    assert bench.bytes_per_update(64) == 9 * 18 * 8 == 1296
    assert bench.bytes_per_update(32) == 648
    # the bytes this library must move: the same 9 transfers of the stored rows 0 and 1 (12 reals)
    assert bench.stored_bytes_per_update(64) == 9 * 12 * 8 == 864
    assert bench.stored_bytes_per_update(32) == 432


def test_chain_deviation_onset():
    p64 = [0.5, 0.5, 0.5, 0.5]
    d = bench.chain_deviation([0.5, 0.5 * (1 + 2e-6), 0.5 * (1 + 3e-5), 0.5], p64)
    assert d["onset_sweep"] == 3
    assert abs(d["max_rel_err_before_onset"] - 2e-6) < 1e-12
    assert bench.chain_deviation(p64, p64)["onset_sweep"] is None


def test_host_cpu_reports_model_and_counts():
    h = bench.host_cpu()
    assert h["model"] and h["nproc"] >= 1 and h["omp_threads"] >= 1


@pytest.fixture
def sources(tmp_path, monkeypatch):
    a, b = tmp_path / "k.hip", tmp_path / "d.h"
    a.write_text("// header\nint f(int x) { return x + 1; }  // add one\n\n/* block\n comment */\n")
    b.write_text("#define N 4\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(a), str(b)])
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    return a, b


def test_source_hash_ignores_comments_only(sources):
    a, _ = sources
    h0 = bench.kernel_source_hash()
    a.write_text("// another header\nint f(int x) { return x + 1; }\n/* other */\n")
    assert bench.kernel_source_hash() == h0
    a.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_hash() != h0


def test_stored_traffic_only_for_the_current_sources(sources, tmp_path):
    a, _ = sources
    prof = tmp_path / "k_update_test_traffic.txt"
    prof.write_text(f"# header: ignored\nkernel_source_sha256_16: {bench.kernel_source_hash()}\n"
                    "hbm_bytes_per_launch: 123456\n")
    assert bench.stored_traffic("k_update_test_traffic.txt") == 123456.0
    a.write_text("int f(int x) { return x - 1; }\n")
    assert bench.stored_traffic("k_update_test_traffic.txt") is None
    assert bench.stored_traffic("missing.txt") is None

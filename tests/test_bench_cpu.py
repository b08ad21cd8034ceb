"""Host logic of bench.py (CPU only): the HBM traffic of the dominant kernel is reported only
while the kernel source matches the hash recorded with the counters, and more than one GPU
is refused before anything touches a device."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _layout(tmp_path, source_text, recorded_hash):
    (tmp_path / "profiles").mkdir()
    src = tmp_path / "k.hip"
    src.write_text(source_text)
    (tmp_path / "profiles" / "hbm_bytes_x.md").write_text(
        "# summary\n\n"
        f"traffic k_block_fused bytes_per_launch=12345 source=k.hip sha256_16={recorded_hash}\n")
    return src


def test_traffic_reported_while_source_unchanged(tmp_path, monkeypatch):
    text = "__global__ void k() {}\n"
    digest = hashlib.sha256(text.encode()).hexdigest()[:16]
    src = _layout(tmp_path, text, digest)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_block_fused") == (12345, os.path.join("profiles", "hbm_bytes_x.md"))
    assert bench.measured_traffic("k_other") is None
    src.write_text(text + "// changed\n")
    assert bench.measured_traffic("k_block_fused") is None


def test_committed_traffic_line_matches_the_source():
    # the committed summaries belong to the committed block kernels
    got = bench.measured_traffic("k_block_fused")
    assert got is not None and got[0] > 2_000_000_000
    got = bench.measured_traffic("k_big_block")
    assert got is not None and got[0] > 3_328_000_000  # at least the dual blocks read and written
    for kernel in ("k_block_fused", "k_big_block"):
        busy = bench.measured_counter("mfma_busy_frac", kernel)
        assert busy is not None and 0.0 < busy[0] < 1.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_counter_figure_reported_while_source_unchanged(tmp_path, monkeypatch):
    text = "__global__ void k() {}\n"
    digest = hashlib.sha256(text.encode()).hexdigest()[:16]
    (tmp_path / "profiles").mkdir()
    src = tmp_path / "k.hip"
    src.write_text(text)
    (tmp_path / "profiles" / "sq_x.md").write_text(
        f"mfma_busy_frac k_block_fused value=0.25 source=k.hip sha256_16={digest}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_counter("mfma_busy_frac", "k_block_fused") == (
        0.25, os.path.join("profiles", "sq_x.md"))
    assert bench.measured_counter("mfma_busy_frac", "k_other") is None
    src.write_text(text + "// changed\n")
    assert bench.measured_counter("mfma_busy_frac", "k_block_fused") is None


def test_block_pass_byte_counts():
    # steps 9-10 read and write every dual block once: 16 K N3 bytes per block
    assert bench.block_pass_algorithmic_bytes(256, 256, 128, 4, 4) == 16 * 16 * 128 * 65536
    assert bench.block_pass_design_bytes(256, 256, 128, 4, 4) > bench.block_pass_algorithmic_bytes(
        256, 256, 128, 4, 4)
    assert bench.gram_flops(256, 256, 128, 4, 4) == 131072 * 65536

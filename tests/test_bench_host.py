"""Host-side logic of bench.py (no GPU): the multi-GPU refusal and the
reading of committed HBM counter summaries."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_measured_traffic_reads_calibrated_summary(tmp_path, monkeypatch):
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    (tmp_path / "paper_2104_10039_amd" / "csrc").mkdir(parents=True)
    for rel in bench.KERNEL_SOURCES:
        (tmp_path / rel).write_text("kernel source v1\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    sha = bench.kernel_source_sha()
    (prof / "k_x_w_pmc.txt").write_text(
        "# summary\n\nsource_sha256: %s\nkernel_FETCH_SIZE_KiB: 500.0\nkernel_WRITE_SIZE_KiB: 100.0\n"
        "copy_bytes: 1048576\ncopy_FETCH_SIZE_KiB: 512.0\ncopy_WRITE_SIZE_KiB: 1024.0\n" % sha)
    # fetch counter reads half the bytes moved, write counter all of them
    assert bench.measured_traffic("k_x", "w") == int(round((1000.0 + 100.0) * 1024))
    assert bench.measured_traffic("k_missing", "w") is None
    # a changed kernel source invalidates the summary
    for rel in bench.KERNEL_SOURCES:
        (tmp_path / rel).write_text("kernel source v2\n")
    assert bench.measured_traffic("k_x", "w") is None

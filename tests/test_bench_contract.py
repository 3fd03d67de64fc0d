"""Host-side parts of the benchmark's contract: more than one GPU is refused
before anything touches a device, and the HBM traffic of a committed
counter record is used only while the kernel sources it was taken from are
unchanged."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_record_is_keyed_by_the_kernel_sources(tmp_path):
    sha = bench.kernel_source_sha()
    assert len(sha) == 16
    good = tmp_path / "good.txt"
    good.write_text(f"kernel k_step<double\nkernel_source_sha {sha}\nfetch_bytes 1\n"
                    f"write_bytes 2\nbytes_per_launch 93227772999\n")
    assert bench.traffic_bytes(str(good)) == 93227772999.0
    stale = tmp_path / "stale.txt"
    stale.write_text("kernel_source_sha 0000000000000000\nbytes_per_launch 5\n")
    assert bench.traffic_bytes(str(stale)) is None
    assert bench.traffic_bytes(str(tmp_path / "missing.txt")) is None

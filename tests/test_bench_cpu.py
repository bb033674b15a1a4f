"""Host-side checks of bench.py that need no GPU: it refuses more than one
GPU before touching any device, and the HBM traffic it reports for the
default engine belongs to the kernel sources as they are now (a changed
kernel must be measured again rather than inherit an old figure)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_default_engine_traffic_matches_sources():
    key = ("mfma_fp4", bench.kernel_source_hash("mfma_fp4"))
    assert key in bench.MEASURED_TRAFFIC, key
    # the figure is bytes per launch of the large workload: between the
    # library read once (2 GB) and every pair's bytes read (7e10 x 2 KiB)
    assert 2e9 < bench.MEASURED_TRAFFIC[key] < 1.5e14

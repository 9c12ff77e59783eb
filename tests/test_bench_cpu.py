"""The benchmark's command-line contract, checked without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    """The step runs on one GPU; asking for more exits with status 2 and a
    message, before any device work."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bench_roofline_constants():
    """Peaks the roofline objects are priced against: 8 TB/s of HBM and one
    wave64 VALU instruction per SIMD every 4 cycles on 1024 SIMDs at 2.4 GHz;
    algorithmic bytes per update: a read and a write of each distribution."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.HBM_PEAK_GBS == 8000.0
    assert bench.VALU_PEAK == 1024 * 2.4e9 / 4
    assert bench.B_ALG == {(2, "f64"): 32, (2, "f32"): 16, (3, "f64"): 16, (3, "f32"): 8}

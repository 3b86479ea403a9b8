"""bench.py's command line on the host: more than one GPU is refused before
any device work, and the traffic figure is reported only for the kernel
sources it was measured on (CPU)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    import bench

    src = tmp_path / "step.hpp"
    src.write_text(open(bench.KERNEL_SOURCES[0]).read() + "\n// edited\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)] + bench.KERNEL_SOURCES[1:])
    assert bench.measured_traffic() is None

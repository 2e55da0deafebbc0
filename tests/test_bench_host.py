"""Host-side logic of bench.py (no GPU): the single-GPU guard, the
algorithmic bytes behind roofline.achieved, and the energy-stability
helper of the energy leg."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_pass_bytes_follow_the_traffic_model():
    # low-rank passes 1..30 at 74 bands: pass 1 reads the spectrum (296 B) and
    # writes alpha and r (16 B); passes 2..30 also read alpha^{j-2} and r
    assert bench.pass_bytes_per_px("lowrank", 30) == pytest.approx((312 + 29 * 320) / 30)
    assert bench.pass_bytes_per_px("lowrank", 1) == 312
    for form in ("fp64", "fp32", "bf16"):
        assert bench.pass_bytes_per_px(form, 30) == 296 + 16
    # algorithmic bytes of one streaming launch on the 598 x 8000 flightline
    assert round(598 * 8000 * bench.pass_bytes_per_px("lowrank", 30)) == 1529604267


def test_energy_stability_index():
    E = np.array([10.0, 5.0, 4.9999, 4.99989, 4.99989])
    assert bench._stable_from(E, 1e-4) == 1       # steps after E^1 are all within 1e-4
    assert bench._stable_from(E, 1e-12) == 3      # only the last step is exact
    assert bench._stable_from(np.array([1.0, 2.0, 3.0]), 1e-3) is None

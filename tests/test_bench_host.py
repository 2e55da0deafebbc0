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
    # scored passes 1..30 at 74 bands: pass 1 reads the spectrum (296 B) and
    # writes alpha^0 (FP32, 4 B); passes 2..30 also read alpha^{j-2}
    assert bench.pass_bytes_per_px(30) == pytest.approx((300 + 29 * 304) / 30)
    assert bench.pass_bytes_per_px(1) == 300
    # algorithmic bytes of one scored pass on the 598 x 8000 flightline
    assert round(598 * 8000 * bench.pass_bytes_per_px(30)) == 1453698133
    # the whole job: 32 passes over the spectrum plus the alpha traffic
    assert bench.job_bytes_per_px(30) == 9716


def test_gram_flops():
    assert bench.gram_flops_per_px(74) == 74 * 75
    assert bench.gram_tile_flops_per_px(74) == 15 * 512       # 5 blocks of 16: 15 tiles
    assert bench.gram_tile_flops_per_px(14) == 512            # B + 2 = 16: one tile


def test_compare_counts_flips_against_nonzero_pixels():
    ref = np.array([0.0, 0.0, 10.0, 20.0, 0.0])
    gpu = np.array([0.0, 1.0, 10.0, 0.0, 0.0])
    rep = bench.compare(gpu, ref)
    assert rep["pattern_flips"] == 2 and rep["nonzero_ref"] == 2
    assert rep["flips_over_nonzero"] == 1.0
    assert rep["pattern_agreement"] == pytest.approx(0.6)
    assert rep["tol_violations"] == 0          # flipped pixels are counted as flips


def test_energy_stability_index():
    E = np.array([10.0, 5.0, 4.9999, 4.99989, 4.99989])
    assert bench._stable_from(E, 1e-4) == 1       # steps after E^1 are all within 1e-4
    assert bench._stable_from(E, 1e-12) == 3      # only the last step is exact
    assert bench._stable_from(np.array([1.0, 2.0, 3.0]), 1e-3) is None

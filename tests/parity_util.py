"""Shared helpers of the GPU parity tests (no GPU code here)."""
import json
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# FP32 tolerance: |d alpha| <= 1e-4 |alpha| + 0.1 ppm*m on pixels whose
# zero/nonzero pattern agrees with the FP64 oracle, and pattern agreement on
# at least 99.9 % of the pixels.
REL_TOL = 1e-4
ABS_TOL = 0.1
PATTERN_MIN = 0.999


def config_lambda(name: str) -> float:
    with open(os.path.join(ROOT, "configs", f"{name}.json")) as f:
        return float(json.load(f)["lambda"])


def compare(gpu, ref, iterative=True):
    """Error report of a GPU result against the FP64 oracle."""
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if iterative:
        agree = (gpu > 0) == (ref > 0)
    else:
        agree = np.ones(gpu.shape, dtype=bool)
    both = agree & ((ref != 0) | (gpu != 0))
    err = np.abs(gpu - ref)
    tol = REL_TOL * np.abs(ref) + ABS_TOL
    ratio = np.where(both, err / tol, 0.0)
    nz = int((ref > 0).sum())
    flips = int((~agree).sum())
    return {
        "pixels": int(gpu.size),
        "pattern_agreement": float(agree.mean()),
        "pattern_flips": flips,
        "flips_over_nonzero": float(flips / nz) if nz else 0.0,
        "max_abs_err": float(err.max()) if err.size else 0.0,
        "rmse": float(np.sqrt((err ** 2).mean())) if err.size else 0.0,
        "max_err_over_tol": float(ratio.max()) if ratio.size else 0.0,
        "tol_violations": int((ratio > 1.0).sum()),
        "nonzero_ref": int((ref > 0).sum()),
    }


def assert_fp32_parity(gpu, ref, iterative=True, label=""):
    rep = compare(gpu, ref, iterative)
    print(label, rep, flush=True)
    assert rep["pattern_agreement"] >= PATTERN_MIN, rep
    assert rep["tol_violations"] == 0, rep
    return rep

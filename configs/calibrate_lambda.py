"""Pick the weight scale lambda for a synthetic workload with the FP64 oracle.

The paper's weights are w = 1/(alpha + eps) (Eq. 5), i.e. lambda = 1, and it
states no other hyper-parameter.  The synthetic scenes here have their own
noise level, so lambda is fixed per workload by this rule: the smallest value
on the grid 2^(j/4), j = -8..40, for which every pixel whose true enhancement
is exactly zero is retrieved as exactly zero by the FP64 oracle (30
iterations, eps = 1e-9).  The predicate is searched by bisection on j.

Run:  python configs/calibrate_lambda.py tiny|flightline|diff [--workers W]
Writes configs/<name>.json.  Calls only the oracle and the scene generator.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle.mf64 import host_cores, retrieve  # noqa: E402
from synth.scenes import diff_spec, flightline_spec, make_scene, tiny_spec  # noqa: E402

SPECS = {"tiny": tiny_spec, "flightline": flightline_spec, "diff": diff_spec}
N_ITER = 30
EPS = 1e-9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name", choices=sorted(SPECS))
    ap.add_argument("--workers", type=int, default=host_cores())
    args = ap.parse_args()
    spec = SPECS[args.name]()
    t0 = time.time()
    sc = make_scene(spec)
    zero = sc.alpha_true == 0
    print(f"scene {spec} generated in {time.time() - t0:.1f}s; "
          f"truth-zero pixels {zero.sum()}", flush=True)

    cache = {}

    def false_positives(j):
        if j not in cache:
            t1 = time.time()
            a, st = retrieve(sc.radiance, sc.s, N_ITER, 2.0 ** (j / 4), EPS,
                             workers=args.workers)
            cache[j] = (int((a[zero] != 0).sum()), int((a != 0).sum()), int(st.max()))
            print(f"  j={j:3d} lambda={2 ** (j / 4):.6g}: false positives {cache[j][0]}, "
                  f"nonzero {cache[j][1]}, max status {cache[j][2]} ({time.time() - t1:.1f}s)",
                  flush=True)
        return cache[j][0]

    lo, hi = -8, 40
    if false_positives(lo) == 0:
        hi = lo
    else:
        assert false_positives(hi) == 0, "no lambda on the grid zeroes every background pixel"
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if false_positives(mid) == 0:
                hi = mid
            else:
                lo = mid
    lam = 2.0 ** (hi / 4)
    out = {
        "workload": args.name,
        "spec": {k: (list(v) if isinstance(v, tuple) else v)
                 for k, v in spec.__dict__.items()},
        "n_iter": N_ITER, "epsilon": EPS, "lambda": lam, "lambda_grid_j": hi,
        "rule": "smallest 2^(j/4), j in [-8,40], with every truth-zero pixel exactly 0 "
                "in the FP64 oracle",
        "nonzero_pixels_at_lambda": cache[hi][1],
        "search": {str(j): v for j, v in sorted(cache.items())},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{args.name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"lambda = {lam} (j = {hi}) -> {path}")


if __name__ == "__main__":
    main()

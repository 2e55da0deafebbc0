"""Throughput benchmark of the MI355X retrieval on one full flightline.

Workload: 598 columns x 8000 lines x 74 bands (FP32 radiance, synthetic, seeded),
30 reweighting iterations, lambda from configs/flightline.json.  One "step" is
one whole retrieval (every pass of the hot path) of the flightline, with the
radiance already resident in HBM.

Prints ONE JSON line (rank 0).  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms lowrank,fp64,fp32,bf16,bf16x3]
                    [--no-cpu-baseline]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "retrieved pixels/s (74 bands, 30 iters): BF16-MFMA vs FP32 plain; fwd+bwd px/s"
HBM_PEAK_GBS = 8000.0
# arithmetic of each covariance form: per-pixel scores, moments and solves
# are FP64 in every form; the Gram forms accumulate their covariance on
# FP64, FP32 or BF16 MFMA (the radiance input is FP32 throughout)
FORM_DTYPE = {"lowrank": "f64", "fp64": "f64", "fp32": "f32 Gram, f64 scores and solves",
              "bf16": "bf16 Gram (f32 accumulate), f64 scores and solves",
              "bf16x3": "split bf16 Gram (hi hi' + hi lo' + lo hi', f32 accumulate), f64 scores and solves"}
FORM_LABEL = {"lowrank": "exact rank-3 covariance update (C^0 from one FP64 Gram; the low-rank variant)",
              "fp64": "per-iteration Gram on FP64 MFMA",
              "fp32": "plain FP32 form: per-iteration Gram on FP32 MFMA, FP64 Cholesky, refinement "
                      "against the exact C^k",
              "bf16": "precision form: per-iteration Gram on BF16 MFMA (FP32 accumulate), FP64 "
                      "Cholesky, refinement against the exact C^k",
              "bf16x3": "precision form, split BF16: per-iteration Gram on BF16 MFMA of hi + lo operands "
                        "(three products, FP32 accumulate), FP64 Cholesky, refinement against the exact C^k"}
# Algorithmic bytes per pixel of the method: every pass reads the B-band FP32
# spectrum once; alpha moves as FP32, written by pass 1 (alpha^0) and read and
# written by every later scored pass (alpha^{j-2} in, alpha^{j-1} out).  The
# dominant kernel of each form is its scored pass 1..K: 300 B/px for pass 1,
# 304 B/px for passes 2..K at 74 bands.  The whole job is K + 2 passes over
# the spectrum plus the alpha traffic: (K + 2) B 4 + 4 + 8 K = 9716 B/px.
def pass_bytes_per_px(K, B=74):
    return (B * 4 + 4 + (K - 1) * (B * 4 + 8)) / K


def job_bytes_per_px(K, B=74):
    return (K + 2) * B * 4 + 4 + 8 * K


# Algorithmic flops per pixel of one Gram pass: the B(B+1)/2 distinct products
# of the symmetric B x B Gram, two flops each; the MFMA tiles execute
# 16 x 16 x 2 flops per tile for the lower triangle of ceil((B + 2) / 16)
# blocks (15 tiles, 7680 flops at 74 bands).
def gram_flops_per_px(B=74):
    return B * (B + 1)


def gram_tile_flops_per_px(B=74):
    nb = (B + 2 + 15) // 16
    return nb * (nb + 1) // 2 * 16 * 16 * 2


# MI355X peaks: HBM 8 TB/s; dense MFMA FP32 157.3 TFLOP/s, BF16 2.5 PFLOP/s,
# FP64 78.6 TFLOP/s
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}
# MFMA products per tile and step (the split BF16 form adds two cross terms)
TILE_PRODUCTS = {"bf16x3": 3}


def compare(gpu, ref, iterative=True):
    """Error report of a result against the FP64 oracle: FP32 tolerance
    |d alpha| <= 1e-4 |alpha| + 0.1 ppm*m on pixels whose zero/nonzero pattern
    agrees, the agreement over all pixels, and the flipped pixels counted
    against the oracle's nonzero pixels."""
    import numpy as np
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    agree = (gpu > 0) == (ref > 0) if iterative else np.ones(gpu.shape, dtype=bool)
    both = agree & ((ref != 0) | (gpu != 0))
    err = np.abs(gpu - ref)
    tol = 1e-4 * np.abs(ref) + 0.1
    ratio = np.where(both, err / tol, 0.0)
    nz = int((ref > 0).sum())
    flips = int((~agree).sum())
    return {"pixels": int(gpu.size), "pattern_agreement": float(agree.mean()),
            "pattern_flips": flips, "nonzero_ref": nz,
            "flips_over_nonzero": float(flips / nz) if nz else 0.0,
            "max_abs_err": float(err.max()) if err.size else 0.0,
            "rmse": float(np.sqrt((err ** 2).mean())) if err.size else 0.0,
            "max_err_over_tol": float(ratio.max()) if ratio.size else 0.0,
            "tol_violations": int((ratio > 1.0).sum())}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


SOURCE = os.path.join(ROOT, "paper_2003_02978_amd", "csrc", "mf.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_digest():
    """sha256 prefix of the library's sources (mf.hip and its included parts)."""
    d = os.path.dirname(SOURCE)
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".inc")):
            h.update(name.encode())
            h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--forms", default="lowrank,fp64,fp32,bf16,bf16x3,bf16@1",
                    help="covariance forms; form@n runs it with n refinement steps")
    ap.add_argument("--streams", default="1,2,3,4",
                    help="concurrent partition groups per retrieval: one count, or candidates "
                         "of which each form takes the fastest (mf_plan_set_streams)")
    ap.add_argument("--chunks", default="",
                    help="work-item lengths (lines) each flightline form tunes with the stream count; "
                         "default 1024,2048,4096 for the low-rank form, 2048,4096,8192 for the Gram forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n-lines", type=int, default=8000)
    ap.add_argument("--save-alpha", default="", help="save each form's alpha as <path>_<form>.npy")
    ap.add_argument("--no-fwd-bwd", action="store_true",
                    help="skip the forward+backward leg on the 598x4000 differentiation scene")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched leg (32 ragged masked flightlines, ~37 GB)")
    ap.add_argument("--no-ingest", action="store_true",
                    help="skip the ingest leg (BIL repack; host-to-device campaign pipeline)")
    ap.add_argument("--no-energy", action="store_true",
                    help="skip the energy-monitor leg (tracking overhead and the long grouped run)")
    ap.add_argument("--energy-iters", type=int, default=200,
                    help="iterations of the energy monitor's convergence run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain 1 GiB device copies (known bytes) for HBM counter scaling")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: every column is an independent problem, "
              "so N GPUs would each run their own share; run it with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2003_02978_amd as mf
    from synth.scenes import flightline_spec, make_scene

    if args.copy_calibration:
        n = 1 << 28                                  # 2^28 floats = 1 GiB
        x = torch.ones(n, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {4 * n} bytes (read {4 * n}, write {4 * n} each)")
        return

    cfg = json.load(open(os.path.join(ROOT, "configs", "flightline.json")))
    lam, K, eps = cfg["lambda"], cfg["n_iter"], cfg["epsilon"]
    spec = flightline_spec(n_lines=args.n_lines)
    t0 = time.time()
    sc = make_scene(spec)
    S, N, B = sc.radiance.shape
    n_px = S * N
    log(f"scene {S}x{N}x{B} generated in {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    L = torch.from_numpy(sc.radiance).to(dev)
    s = torch.from_numpy(sc.s).to(dev)
    alpha = torch.empty((S, N), dtype=torch.float32, device=dev)
    status = torch.empty((S,), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    # measured read ceiling on the same buffer
    ceil = []
    for nb in (1024, 4096, 16384):
        for _ in range(3):
            ms = mf.stream_read_ms(L.view(-1), nb)
        ceil.append((L.numel() * 4 / (ms * 1e-3) / 1e9, nb))
    ceiling_GBps, ceiling_blocks = max(ceil)
    log(f"stream read ceiling: {ceiling_GBps:.0f} GB/s ({ceiling_blocks} blocks); all {ceil}")

    forms = [f for f in args.forms.split(",") if f]
    stream_candidates = [min(int(x), S) for x in args.streams.split(",") if x]
    head = forms[0]
    results = {}
    outputs = {}
    for label in forms:
        form, _, rs = label.partition("@")
        refine = int(rs) if rs else -1
        # launch choice: work-item length and concurrent partition groups,
        # timed together (every group count gives the same alpha bit for bit;
        # the length changes the order of the partial sums)
        chunk_cands = ([int(x) for x in args.chunks.split(",") if x] if args.chunks else
                       ([1024, 2048, 4096] if form == "lowrank" else [2048, 4096, 8192]))
        tune_ms = {}
        for ch in chunk_cands:
            plan = mf.Plan([(0, S, N)], B, K, lam, eps, True, form, refine_steps=refine, chunk_lines=ch)
            ws = plan.alloc_workspace(dev)
            plan.retrieve(L, s, alpha, None, status, ws)
            for ns in stream_candidates:
                plan.set_streams(ns)
                plan.retrieve(L, s, alpha, None, status, ws)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(3):
                    plan.retrieve(L, s, alpha, None, status, ws)
                torch.cuda.synchronize()
                tune_ms[(ch, ns)] = 1e3 * (time.perf_counter() - t0) / 3
            plan.close()
            del ws
        chunk, n_streams = min(tune_ms, key=tune_ms.get)
        stream_ms = {ns: v for (ch, ns), v in tune_ms.items() if ch == chunk}
        plan = mf.Plan([(0, S, N)], B, K, lam, eps, True, form, refine_steps=refine, chunk_lines=chunk)
        ws = plan.alloc_workspace(dev)
        plan.set_streams(n_streams)
        for _ in range(args.warmup):
            plan.retrieve(L, s, alpha, None, status, ws)
        torch.cuda.synchronize()
        steps = args.steps if form == head else max(3, args.steps // 4)
        # timed region (no instrumentation)
        t1 = time.perf_counter()
        for _ in range(steps):
            plan.retrieve(L, s, alpha, None, status, ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        outputs[label] = alpha.cpu().numpy().copy()      # the timed launch setting's result
        if args.save_alpha:
            np.save(f"{args.save_alpha}_{label}.npy", outputs[label])
        st = status.cpu().numpy()
        # instrumented region: per-kernel durations from HIP events recorded on
        # the stream the kernels run on, with one partition group, so that each
        # launch has the GPU to itself (its duration is the kernel's own), at the
        # work-item length that is fastest with one group
        one = {ch: v for (ch, ns), v in tune_ms.items() if ns == 1}
        chunk1 = min(one, key=one.get) if one else chunk
        if chunk1 != chunk:
            plan.close()
            del ws
            plan = mf.Plan([(0, S, N)], B, K, lam, eps, True, form, refine_steps=refine, chunk_lines=chunk1)
            ws = plan.alloc_workspace(dev)
            plan.retrieve(L, s, alpha, None, status, ws)
        plan.set_streams(1)
        plan.set_timing(True)
        plan.kernel_times()
        t2 = time.perf_counter()
        for _ in range(steps):
            plan.retrieve(L, s, alpha, None, status, ws)
        torch.cuda.synchronize()
        dt_ins = time.perf_counter() - t2
        kt = plan.kernel_times()
        plan.set_timing(False)
        res = {
            "px_per_s": n_px * steps / dt,
            "ms_per_step": 1e3 * dt / steps,
            "streams": n_streams,
            "chunk_lines": chunk,
            "kernel_timing_launch": {"streams": 1, "chunk_lines": chunk1},
            "ms_per_step_by_streams": {str(k): round(v, 3) for k, v in stream_ms.items()},
            "tune_ms": {f"chunk={c},streams={n}": round(v, 3) for (c, n), v in tune_ms.items()},
            "ms_per_step_instrumented": 1e3 * dt_ins / steps,
            "steps": steps,
            "columns_failed": int((st != 0).sum()),
            "kernels_ms_per_step": {k: round(v[0] / steps, 4) for k, v in kt.items()},
            "launches_per_step": {k: v[1] // steps for k, v in kt.items()},
        }
        # the dominant kernel of this form: its scored passes 1..K
        dom = "pass_vec" if form == "lowrank" else "pass_gram"
        avg_ms = kt[dom][0] / max(1, kt[dom][1])
        res["form"] = form
        res["refine_steps"] = plan.refine_steps
        res["dominant_kernel"] = dom
        res["dominant_avg_ms"] = avg_ms
        res["dominant_bytes_per_px"] = pass_bytes_per_px(K, B)
        res["dominant_GBps"] = res["dominant_bytes_per_px"] * n_px / (avg_ms * 1e-3) / 1e9
        if form != "lowrank":
            res["gram_TFLOPs_algorithmic"] = gram_flops_per_px(B) * n_px / (avg_ms * 1e-3) / 1e12
            res["gram_TFLOPs_tiles"] = (TILE_PRODUCTS.get(form, 1) * gram_tile_flops_per_px(B) * n_px /
                                        (avg_ms * 1e-3) / 1e12)
            res["gram_frac_of_mfma_peak_tiles"] = res["gram_TFLOPs_tiles"] / PEAK_TFLOPS[form]
        results[label] = res
        log(f"{label}: {res['px_per_s'] / 1e6:.1f} Mpx/s, {res['ms_per_step']:.3f} ms/step with {n_streams} "
            f"stream(s), {chunk}-line items {res['tune_ms']}, {dom} {avg_ms * 1e3:.1f} us = "
            f"{res['dominant_GBps']:.0f} GB/s, kernels {res['kernels_ms_per_step']}")
        plan.close()
        del ws

    # detector grouping (Sec. II-E): partitions of 5 adjacent columns, the
    # paper's setting for its real flightlines, low-rank form
    grouped = None
    if "lowrank" in forms:
        plan = mf.Plan([(0, S, N)], B, K, lam, eps, True, "lowrank", group=5)
        ws = plan.alloc_workspace(dev)
        gst = torch.empty((plan.n_columns,), dtype=torch.int32, device=dev)
        for _ in range(max(1, args.warmup)):
            plan.retrieve(L, s, alpha, None, gst, ws)
        torch.cuda.synchronize()
        g_ms = {}
        for ns in stream_candidates:
            plan.set_streams(min(ns, plan.n_columns))
            plan.retrieve(L, s, alpha, None, gst, ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                plan.retrieve(L, s, alpha, None, gst, ws)
            torch.cuda.synchronize()
            g_ms[ns] = 1e3 * (time.perf_counter() - t0) / 3
        g_streams = min(g_ms, key=g_ms.get)
        plan.set_streams(min(g_streams, plan.n_columns))
        gsteps = max(3, args.steps // 4)
        t6 = time.perf_counter()
        for _ in range(gsteps):
            plan.retrieve(L, s, alpha, None, gst, ws)
        torch.cuda.synchronize()
        dtg = (time.perf_counter() - t6) / gsteps
        grouped = {"workload": f"flightline {S}x{N}x{B}, partitions of 5 columns "
                               f"({plan.n_columns} partitions), {K} iterations, low-rank form",
                   "px_per_s": round(n_px / dtg, 1), "ms_per_step": round(1e3 * dtg, 3),
                   "streams": g_streams, "ms_per_step_by_streams": {str(k): round(v, 3) for k, v in g_ms.items()},
                   "partitions_failed": int((gst.cpu().numpy() != 0).sum())}
        log(f"grouped (5 columns): {grouped['px_per_s'] / 1e6:.1f} Mpx/s, {grouped['ms_per_step']:.2f} ms "
            f"with {g_streams} stream(s) {grouped['ms_per_step_by_streams']}")
        plan.close()
        del ws

    energy = None
    if "lowrank" in forms and not args.no_energy:
        energy = run_energy(mf, torch, np, dev, L, s, S, N, B, K, lam, eps, results["lowrank"]["ms_per_step"],
                            args.energy_iters, results["lowrank"]["chunk_lines"], results["lowrank"]["streams"])

    # forward + backward (hand-written adjoint) on the differentiation scene:
    # 598 x 4000 x 74, 30 iterations, J = sum (alpha - alpha_true)^2
    fwdbwd = None
    if not args.no_fwd_bwd:
        from synth.scenes import diff_spec
        dcfg = json.load(open(os.path.join(ROOT, "configs", "diff.json")))
        dsc = make_scene(diff_spec())
        dS, dN, _ = dsc.radiance.shape
        dL = torch.from_numpy(dsc.radiance).to(dev)
        ds_ = torch.from_numpy(dsc.s).to(dev)
        dtrue = torch.from_numpy(dsc.alpha_true.astype(np.float32)).to(dev)
        plan = mf.Plan([(0, dS, dN)], B, K, dcfg["lambda"], eps, True, "lowrank", save_for_backward=True)
        ws = plan.alloc_workspace(dev)
        da = torch.empty((dS, dN), dtype=torch.float32, device=dev)
        steps = max(3, args.steps // 4)

        def fb():
            plan.retrieve(dL, ds_, da, None, None, ws)
            g = 2.0 * (da - dtrue)
            return plan.backward(dL, ds_, g, None, ws)

        for _ in range(max(1, args.warmup)):
            fb()
        torch.cuda.synchronize()
        fb_ms = {}
        for ns in stream_candidates:                 # concurrent partition groups (both sweeps)
            plan.set_streams(ns)
            fb()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(2):
                fb()
            torch.cuda.synchronize()
            fb_ms[ns] = 1e3 * (time.perf_counter() - t0) / 2
        fb_streams = min(fb_ms, key=fb_ms.get)
        plan.set_streams(fb_streams)
        t4 = time.perf_counter()
        for _ in range(steps):
            fb()
        torch.cuda.synchronize()
        dtfb = (time.perf_counter() - t4) / steps
        t5 = time.perf_counter()
        for _ in range(steps):
            plan.retrieve(dL, ds_, da, None, None, ws)
        torch.cuda.synchronize()
        dtf = (time.perf_counter() - t5) / steps
        plan.set_streams(1)                           # kernel timing: each launch alone
        plan.set_timing(True)
        plan.kernel_times()
        fb()
        kt = plan.kernel_times()
        plan.set_timing(False)
        fwdbwd = {"workload": f"differentiation scene {dS}x{dN}x{B}, {K} iterations, lambda "
                              f"{dcfg['lambda']:.4g}, loss sum (alpha - alpha_true)^2",
                  "px_per_s": round(dS * dN / dtfb, 1), "ms_per_step": round(1e3 * dtfb, 3),
                  "streams": fb_streams, "ms_per_step_by_streams": {str(k): round(v, 3) for k, v in fb_ms.items()},
                  "forward_ms": round(1e3 * dtf, 3), "backward_ms": round(1e3 * (dtfb - dtf), 3),
                  "kernels_ms_fwd_plus_bwd": {k: round(v[0], 4) for k, v in kt.items()}}
        log(f"fwd+bwd: {fwdbwd['px_per_s'] / 1e6:.1f} Mpx/s, {fwdbwd['ms_per_step']:.2f} ms "
            f"(forward {fwdbwd['forward_ms']:.2f} ms) with {fb_streams} stream(s) {fwdbwd['ms_per_step_by_streams']}")
        plan.close()
        del ws, dL

    ingest = None
    if not args.no_ingest:
        ingest = run_ingest(mf, torch, np, dev, sc, K, lam, eps)
    del L, alpha, status
    torch.cuda.empty_cache()
    batch = None
    if not args.no_batch:
        batch = run_batch(mf, torch, np, dev, K, lam, eps, max(3, args.steps // 4), args.warmup)

    # CPU baseline: the FP64 oracle on the host cores; its output is also the
    # reference for every form's error report.
    cpu = None
    errors = {}
    if not args.no_cpu_baseline:
        from oracle.mf64 import host_cores, retrieve as oracle_retrieve
        from synth.scenes import tiny_spec
        # every core of the process's affinity set, at most the 16 CPUs a GPU
        # box allots to one GPU
        affinity = host_cores()
        cores = min(16, affinity)
        n_cols = S if cores >= 8 else min(S, 16 * cores)
        cols = list(range(n_cols))
        t3 = time.perf_counter()
        ref, rst = oracle_retrieve(sc.radiance, sc.s, K, lam, eps, columns=cols, workers=cores)
        dtc = time.perf_counter() - t3
        # single core on the tiny scene (64 x 512 x 74, its own lambda)
        tcfg = json.load(open(os.path.join(ROOT, "configs", "tiny.json")))
        tsc = make_scene(tiny_spec())
        t7 = time.perf_counter()
        oracle_retrieve(tsc.radiance, tsc.s, K, tcfg["lambda"], eps, workers=1)
        dt1 = time.perf_counter() - t7
        cpu = {"value": n_cols * N / dtc, "unit": "px/s", "cores": cores, "kind": "oracle",
               "sample": f"{n_cols} of {S} columns x {N} lines x {B} bands, 30 iterations, "
                         f"FP64 numpy/LAPACK, one process per core",
               "seconds": round(dtc, 2), "cores_in_affinity": affinity, "cpu_model": cpu_model(),
               "single_core_tiny": {"workload": "tiny scene 64x512x74, 30 iterations",
                                    "seconds": round(dt1, 3),
                                    "px_per_s": round(tsc.radiance.shape[0] * tsc.radiance.shape[1] / dt1, 1)}}
        log(f"oracle: {cpu['value']:.0f} px/s on {cores} cores ({dtc:.1f}s), {cpu['cpu_model']}; "
            f"tiny scene on one core {dt1:.2f}s")
        for form, a in outputs.items():
            rep = compare(a[:n_cols], ref)
            errors[form] = {k: (round(v, 6) if isinstance(v, float) else v) for k, v in rep.items()}
            log(f"{form} vs FP64: {errors[form]}")

    hr = results[head]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        tf = json.load(open(TRAFFIC_FILE))
        if tf.get("source_sha256_16") == source_digest() and tf.get("kernel") == hr["dominant_kernel"]:
            traffic = tf.get("bytes_per_launch")
    roof = {
        "bound": "hbm",
        "kernel": hr["dominant_kernel"],
        "achieved": round(hr["dominant_GBps"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(hr["dominant_GBps"] / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "algorithmic_bytes_per_launch": round(hr["dominant_bytes_per_px"] * n_px),
        "avg_launch_ms": round(hr["dominant_avg_ms"], 5),
        "measured_read_ceiling_GBps": round(ceiling_GBps, 1),
        "frac_of_measured_ceiling": round(hr["dominant_GBps"] / ceiling_GBps, 4),
        # each launch timed alone on the GPU (one partition group); the
        # timed throughput runs the groups of `config` concurrently
        "launch": hr["kernel_timing_launch"],
    }
    whole_job_GBps = job_bytes_per_px(K, B) * n_px / (hr["ms_per_step"] * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(hr["px_per_s"], 1),
        "unit": "px/s",
        "n_gpus": 1,
        "steps": hr["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(hr["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": FORM_DTYPE[head],
        "data": "synthetic",
        "config": {"workload": f"flightline {S}x{N}x{B}, {K} iterations, lambda {lam:.4g}, "
                               f"covariance form '{head}'",
                   "columns": S, "lines": N, "bands": B, "iterations": K,
                   "covariance": head, "radiance": "f32", "parallelism": "single GPU",
                   "streams": results[head]["streams"], "chunk_lines": results[head]["chunk_lines"]},
        "headline_form": FORM_LABEL.get(results[head]["form"], head),
        "roofline": roof,
        "cpu_baseline": cpu,
        "hbm_fraction_whole_job": round(whole_job_GBps / HBM_PEAK_GBS, 4),
        "forms": {f: {"dtype": FORM_DTYPE[r["form"]], "label": FORM_LABEL[r["form"]],
                      "refine_steps": r["refine_steps"],
                      "px_per_s": round(r["px_per_s"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                      "streams": r["streams"], "chunk_lines": r["chunk_lines"],
                      "ms_per_step_by_streams": r["ms_per_step_by_streams"],
                      "hbm_fraction_whole_job": round(job_bytes_per_px(K, B) * n_px /
                                                      (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "kernels_ms_per_step": r["kernels_ms_per_step"],
                      "dominant_kernel": r["dominant_kernel"],
                      "dominant_avg_us": round(1e3 * r["dominant_avg_ms"], 2),
                      "dominant_GBps": round(r["dominant_GBps"], 1),
                      **({"gram_TFLOPs_algorithmic": round(r["gram_TFLOPs_algorithmic"], 2),
                          "gram_TFLOPs_tiles": round(r["gram_TFLOPs_tiles"], 2),
                          "gram_frac_of_mfma_peak_tiles": round(r["gram_frac_of_mfma_peak_tiles"], 4)}
                         if "gram_TFLOPs_tiles" in r else {}),
                      "error_vs_fp64": errors.get(f)} for f, r in results.items()},
    }
    for f in ("fp32", "bf16", "bf16x3"):
        if f in results:
            out[f"{f}_px_per_s"] = round(results[f]["px_per_s"], 1)
    out["grouped"] = grouped
    out["energy"] = energy
    out["ingest"] = ingest
    out["fwd_bwd"] = fwdbwd
    out["batch"] = batch
    if "bf16" in results and "fp32" in results:
        out["bf16_vs_fp32_gram_speedup"] = round(results["bf16"]["px_per_s"] / results["fp32"]["px_per_s"], 3)
    if "bf16x3" in results and "fp32" in results:
        out["bf16x3_vs_fp32_gram_speedup"] = round(results["bf16x3"]["px_per_s"] / results["fp32"]["px_per_s"], 3)
    print(json.dumps(out), flush=True)


def _stable_from(E, rtol):
    """First k such that |E^j - E^{j-1}| <= rtol |E^j| for every j > k: the
    energy changes by at most rtol per step from E^k on (None if the last
    step still exceeds it)."""
    import numpy as np
    d = np.abs(np.diff(E)) <= rtol * np.abs(E[1:])
    if not d[-1]:
        return None
    k = len(E) - 1
    while k >= 1 and d[k - 1]:
        k -= 1
    return k


def run_energy(mf, torch, np, dev, L, s, S, N, B, K, lam, eps, plain_ms, n_long, chunk=0, streams=1):
    """The energy monitor (Eq. 8 per iteration, low-rank form): its cost at the
    flightline workload (K iterations, one partition per column), and a long
    run of n_long iterations with every detector of the flightline in one
    partition, reporting E^k and the iteration from which it stays within a
    relative 1e-6 (and 1e-4) of the previous one; also the per-column run at
    n_long iterations (fraction of columns stable by iteration 20)."""
    res = {}
    alpha = torch.empty((S, N), dtype=torch.float32, device=dev)
    plan = mf.Plan([(0, S, N)], B, K, lam, eps, True, "lowrank", track_energy=True, chunk_lines=chunk)
    plan.set_streams(streams)                  # the untracked run's launch setting
    ws = plan.alloc_workspace(dev)
    st = torch.empty((plan.n_columns,), dtype=torch.int32, device=dev)
    plan.retrieve(L, s, alpha, None, st, ws)
    torch.cuda.synchronize()
    steps = 5
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.retrieve(L, s, alpha, None, st, ws)
        E = plan.energy(ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    res["tracked_ms_per_step"] = round(1e3 * dt, 3)
    res["untracked_ms_per_step"] = round(plain_ms, 3)
    res["overhead_frac"] = round(1e3 * dt / plain_ms - 1.0, 4)
    plan.close()
    del ws
    log(f"energy tracking at K={K}: {1e3 * dt:.2f} ms vs {plain_ms:.2f} ms untracked")

    for label, group in (("all_detectors_one_partition", S), ("per_column", 1)):
        plan = mf.Plan([(0, S, N)], B, n_long, lam, eps, True, "lowrank", track_energy=True, group=group,
                       chunk_lines=8192 if group > 1 else 0)
        ws = plan.alloc_workspace(dev)
        st = torch.empty((plan.n_columns,), dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plan.retrieve(L, s, alpha, None, st, ws)
        E = plan.energy(ws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        E = E.cpu().numpy()
        ok = st.cpu().numpy() == 0
        r = {"partitions": plan.n_columns, "partitions_failed": int((~ok).sum()), "iterations": n_long,
             "ms": round(1e3 * dt, 2)}
        if group > 1:
            e = E[:, 0]
            marks = [k for k in (0, 1, 2, 3, 5, 10, 20, 30, 50, 100, 150, 200, n_long) if k <= n_long]
            r["E"] = {str(k): float(e[k]) for k in sorted(set(marks))}
            r["stable_from_rtol_1e-6"] = _stable_from(e, 1e-6)
            r["stable_from_rtol_1e-4"] = _stable_from(e, 1e-4)
            log(f"energy, {S} detectors in one partition, {n_long} iterations ({1e3 * dt:.0f} ms): "
                f"stable within 1e-6 from k={r['stable_from_rtol_1e-6']}, within 1e-4 from "
                f"k={r['stable_from_rtol_1e-4']}")
        else:
            ks = [_stable_from(E[:, c], 1e-6) for c in np.flatnonzero(ok)]
            k4 = [_stable_from(E[:, c], 1e-4) for c in np.flatnonzero(ok)]
            r["frac_stable_1e-6_by_20"] = round(float(np.mean([k is not None and k <= 20 for k in ks])), 4)
            r["frac_stable_1e-4_by_20"] = round(float(np.mean([k is not None and k <= 20 for k in k4])), 4)
            r["median_stable_from_1e-6"] = float(np.median([k if k is not None else n_long + 1 for k in ks]))
            log(f"energy, per column, {n_long} iterations ({1e3 * dt:.0f} ms): "
                f"{100 * r['frac_stable_1e-6_by_20']:.1f}% of columns stable within 1e-6 by k=20")
        res[label] = r
        plan.close()
        del ws
    return res


def run_ingest(mf, torch, np, dev, sc, K, lam, eps, n_fl=3):
    """Ingest of band-interleaved-by-line flightlines: the repack kernel's
    bandwidth, and a campaign pipeline (host-to-device copy of flightline f+1
    on a copy stream while flightline f is repacked and retrieved on a
    compute stream; double-buffered device BIL, events between the streams).
    The host cube is pinned memory; the end-to-end rate includes the copy."""
    S, N, B = sc.radiance.shape
    n_px = S * N
    bil_host = torch.from_numpy(np.ascontiguousarray(np.transpose(sc.radiance, (1, 2, 0)))).pin_memory()
    bil = [torch.empty((N, B, S), dtype=torch.float32, device=dev) for _ in range(2)]
    rad = torch.empty((S, N, B), dtype=torch.float32, device=dev)
    val = torch.empty((S, N), dtype=torch.uint8, device=dev)
    s = torch.from_numpy(sc.s).to(dev)
    alpha = torch.empty((S, N), dtype=torch.float32, device=dev)
    bil[0].copy_(bil_host)
    torch.cuda.synchronize()
    # repack bandwidth (events on the stream the kernel runs on)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    mf.repack_bil(bil[0], rad, val)
    e0.record()
    for _ in range(5):
        mf.repack_bil(bil[0], rad, val)
    e1.record()
    torch.cuda.synchronize()
    rp_ms = e0.elapsed_time(e1) / 5
    rp_bytes = 2 * n_px * B * 4 + n_px
    # host-to-device copy alone
    e0.record()
    bil[1].copy_(bil_host, non_blocking=True)
    e1.record()
    torch.cuda.synchronize()
    h2d_ms = e0.elapsed_time(e1)
    plan = mf.Plan([(0, S, N)], B, K, lam, eps, True, "lowrank")
    ws = plan.alloc_workspace(dev)
    plan.retrieve(rad, s, alpha, val, None, ws)
    torch.cuda.synchronize()
    cp, cs = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
    copied = [torch.cuda.Event() for _ in range(2)]
    freed = [torch.cuda.Event() for _ in range(2)]
    t0 = time.perf_counter()
    for f in range(n_fl):
        k = f % 2
        with torch.cuda.stream(cp):
            if f >= 2:
                cp.wait_event(freed[k])             # the compute stream is done with it
            bil[k].copy_(bil_host, non_blocking=True)
            copied[k].record(cp)
        with torch.cuda.stream(cs):
            cs.wait_event(copied[k])
            mf.repack_bil(bil[k], rad, val, stream=cs)
            freed[k].record(cs)
            plan.retrieve(rad, s, alpha, val, None, ws, stream=cs)
    torch.cuda.synchronize()
    pipe_s = time.perf_counter() - t0
    plan.close()
    del ws, bil, rad, val
    torch.cuda.empty_cache()
    res = {"workload": f"{n_fl} flightlines {S}x{N}x{B} from pinned host memory, BIL layout",
           "repack_ms": round(rp_ms, 4), "repack_GBps": round(rp_bytes / (rp_ms * 1e-3) / 1e9, 1),
           "h2d_ms_per_flightline": round(h2d_ms, 3),
           "h2d_GBps": round(n_px * B * 4 / (h2d_ms * 1e-3) / 1e9, 1),
           "pipeline_ms_per_flightline": round(1e3 * pipe_s / n_fl, 3),
           "end_to_end_px_per_s": round(n_fl * n_px / pipe_s, 1)}
    log(f"ingest: repack {res['repack_ms']:.3f} ms = {res['repack_GBps']:.0f} GB/s, "
        f"H2D {res['h2d_ms_per_flightline']:.1f} ms/flightline ({res['h2d_GBps']:.1f} GB/s), "
        f"pipeline {res['pipeline_ms_per_flightline']:.1f} ms/flightline, "
        f"{res['end_to_end_px_per_s'] / 1e6:.1f} Mpx/s end to end")
    return res


def run_batch(mf, torch, np, dev, K, lam, eps, steps, warmup):
    """Batched form: 32 ragged flightlines (598 columns, U{1000..12000} lines,
    0-20 % of each column masked in runs), one plan, chunk length picked by
    the autotuner (with the streaming tile shape and the persistent grid),
    launch sequence replayed as a HIP graph on a side stream.
    Columns of three flightlines are regenerated on the host and checked
    against the oracle."""
    from synth.scenes import batch_specs, make_scene, make_globals, make_column
    from oracle.mf64 import retrieve as oracle_retrieve
    specs = batch_specs()
    B = specs[0].n_bands
    fls, first = [], 0
    for sp in specs:
        fls.append((first, sp.n_columns, sp.n_lines))
        first += sp.n_columns * sp.n_lines
    total = first
    t0 = time.time()
    dL = torch.empty((total, B), dtype=torch.float32, device=dev)
    dV = torch.empty((total,), dtype=torch.uint8, device=dev)
    s_host = None
    for sp, (f0, S_, N_) in zip(specs, fls):
        sc = make_scene(sp)
        dL[f0:f0 + S_ * N_].copy_(torch.from_numpy(sc.radiance.reshape(-1, B)))
        dV[f0:f0 + S_ * N_].copy_(torch.from_numpy(sc.valid.reshape(-1)))
        s_host = sc.s
        del sc
    ds = torch.from_numpy(s_host).to(dev)
    torch.cuda.synchronize()
    gen_s = time.time() - t0
    n_valid = int(dV.sum().item())
    log(f"batch: {len(specs)} flightlines, {total} px ({total * B * 4 / 1e9:.1f} GB), "
        f"{n_valid / total:.3f} valid, generated and uploaded in {gen_s:.1f}s")
    side = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(side):
        t_tune = time.perf_counter()
        best, tune = mf.autotune(fls, dL, ds, dV, chunks=(1024, 2048, 4096),
                                 tiles=("32x4", "32x2", "64x2"), wgs=(0, 2, 3, 4), streams=(1, 2, 3, 4),
                                 reps=2, n_bands=B, n_iter=K, lam=lam, eps=eps)
        tune_s = time.perf_counter() - t_tune
        plan = mf.Plan(fls, B, K, lam, eps, True, "lowrank", chunk_lines=best["chunk_lines"])
        plan.set_launch(best["stream_tile"], best["wgs_per_cu"])
        plan.set_streams(best["streams"])
        plan.set_graph(True)
        ws = plan.alloc_workspace(dev)
        alpha = torch.empty((total,), dtype=torch.float32, device=dev)
        status = torch.empty((plan.n_columns,), dtype=torch.int32, device=dev)
        for _ in range(max(1, warmup)):
            plan.retrieve(dL, ds, alpha, dV, status, ws)
        side.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            plan.retrieve(dL, ds, alpha, dV, status, ws)
        side.synchronize()
        dt = (time.perf_counter() - t1) / steps
    a_host = alpha.cpu().numpy()
    st_host = status.cpu().numpy()
    # parity on sampled columns (the shortest, the longest and a middle flightline)
    order = np.argsort([sp.n_lines for sp in specs])
    picks = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    rng = np.random.default_rng(7)
    errs, n_checked = [], 0
    for f in picks:
        sp = specs[f]
        g = make_globals(sp)
        cols = sorted(set([int(g.plumes[0, 0]) % sp.n_columns] +
                          [int(c) for c in rng.choice(sp.n_columns, 2, replace=False)]))
        Ls, Vs = [], []
        for c in cols:
            Lc, _, vc = make_column(sp, g, c)
            Ls.append(Lc)
            Vs.append(vc)
        ref, _ = oracle_retrieve(np.stack(Ls), g.s, K, lam, eps, valid=np.stack(Vs), workers=len(cols))
        f0, S_, N_ = fls[f]
        got = np.stack([a_host[f0 + c * N_: f0 + (c + 1) * N_] for c in cols])
        errs.append(compare(got, ref))
        n_checked += len(cols)
    worst = max(errs, key=lambda e: e["max_err_over_tol"])
    res = {"workload": f"{len(specs)} flightlines x {specs[0].n_columns} columns, lines U(1000, 12000), "
                       f"{B} bands, 0-20 % masked per column, {K} iterations, lambda {lam:.4g}",
           "pixels": total, "valid_fraction": round(n_valid / total, 4),
           "px_per_s": round(total / dt, 1), "ms_per_step": round(dt * 1e3, 3), "steps": steps,
           "launch": best, "autotune_s": round(tune_s, 1),
           "autotune_ms": {str(k): round(v, 3) for k, v in tune.items()},
           "graph_replay": True, "columns_failed": int((st_host != 0).sum()),
           "sampled_columns_vs_fp64": {"columns": n_checked,
                                       "pixels": sum(e["pixels"] for e in errs),
                                       "pattern_agreement_min": min(e["pattern_agreement"] for e in errs),
                                       "max_err_over_tol": round(worst["max_err_over_tol"], 6),
                                       "tol_violations": sum(e["tol_violations"] for e in errs)}}
    log(f"batch: {res['px_per_s'] / 1e6:.1f} Mpx/s, {res['ms_per_step']:.1f} ms/step, launch {best}, "
        f"tune {res['autotune_ms']}, sampled vs FP64 {res['sampled_columns_vs_fp64']}")
    plan.close()
    del ws, dL, dV, alpha
    torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()

"""Python binding of libmf.so, the MI355X retrieval library (see include/mf.h).

Argument marshalling only: every step of the retrieval runs in the library's
HIP kernels.  PyTorch supplies device memory and the stream.  If the library
is missing, importing the binding works but every call raises: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmf.so")

MF_OK, MF_E_ARG, MF_E_SHAPE, MF_E_UNSUPPORTED, MF_E_DEVICE, MF_E_STATE = range(6)
MF_COL_OK, MF_COL_FEW_PIXELS, MF_COL_NOT_SPD, MF_COL_NONFINITE = range(4)
COV = {"lowrank": 0, "fp64": 1, "fp32": 2, "bf16": 3, "bf16x3": 4}

# Every symbol declared in include/mf.h.
EXPORTS = ("mf_abi_version", "mf_options_default", "mf_status_str", "mf_last_error",
           "mf_plan_create", "mf_workspace_bytes", "mf_plan_columns", "mf_plan_pixels",
           "mf_retrieve", "mf_backward", "mf_plan_set_graph", "mf_plan_set_timing",
           "mf_plan_kernel_times", "mf_plan_energy", "mf_repack_bil", "mf_stream_read",
           "mf_retrieve_noalloc", "mf_plan_refine_steps", "mf_plan_set_launch", "mf_plan_set_streams",
           "mf_plan_streams", "mf_plan_destroy")
TILES = {"32x4": 0, "32x2": 1, "64x2": 2, "64x1": 3}   # MF_TILE_*: pixels per wave chunk x waves
NOALLOC_SCRATCH_BYTES = 64 << 20   # MF_NOALLOC_SCRATCH_BYTES
MAX_STREAMS = 8                    # MF_MAX_STREAMS
MAX_BACKWARD_ITER = 1000           # MF_MAX_BACKWARD_ITER
KERNEL_KINDS = ("pass_gram", "pass_vec", "pass_last", "solve", "other", "pass_init")
ABI_VERSION = 4          # MF_ABI_VERSION of include/mf.h (mf_options layout)


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n_bands", ctypes.c_int32),
                ("n_iter", ctypes.c_int32), ("albedo", ctypes.c_int32),
                ("lambda_", ctypes.c_double), ("epsilon", ctypes.c_double),
                ("cov", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("save_for_backward", ctypes.c_int32), ("chunk_lines", ctypes.c_int32),
                ("group", ctypes.c_int32), ("track_energy", ctypes.c_int32)]


class Flightline(ctypes.Structure):
    _fields_ = [("first_px", ctypes.c_int64), ("n_columns", ctypes.c_int32),
                ("n_lines", ctypes.c_int32)]


class MFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mf error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmf.so (built by paper_2003_02978_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2003_02978_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    lib.mf_abi_version.restype = ctypes.c_int
    lib.mf_options_default.argtypes = [ctypes.POINTER(Options)]
    lib.mf_status_str.restype = ctypes.c_char_p
    lib.mf_status_str.argtypes = [ctypes.c_int]
    lib.mf_last_error.restype = ctypes.c_char_p
    lib.mf_plan_create.restype = ctypes.c_int
    lib.mf_plan_create.argtypes = [ctypes.POINTER(Options), ctypes.POINTER(Flightline), i32,
                                   ctypes.POINTER(vp)]
    lib.mf_workspace_bytes.restype = sz
    lib.mf_workspace_bytes.argtypes = [vp]
    lib.mf_plan_columns.restype = i64
    lib.mf_plan_columns.argtypes = [vp]
    lib.mf_plan_pixels.restype = i64
    lib.mf_plan_pixels.argtypes = [vp]
    lib.mf_plan_refine_steps.restype = i32
    lib.mf_plan_refine_steps.argtypes = [vp]
    lib.mf_retrieve.restype = ctypes.c_int
    lib.mf_retrieve.argtypes = [vp] * 8
    lib.mf_retrieve_noalloc.restype = ctypes.c_int
    lib.mf_retrieve_noalloc.argtypes = [vp] * 7
    lib.mf_plan_destroy.argtypes = [vp]
    lib.mf_backward.restype = ctypes.c_int
    lib.mf_backward.argtypes = [vp] * 9
    lib.mf_plan_set_graph.restype = ctypes.c_int
    lib.mf_plan_set_graph.argtypes = [vp, ctypes.c_int]
    lib.mf_plan_set_launch.restype = ctypes.c_int
    lib.mf_plan_set_launch.argtypes = [vp, i32, i32]
    lib.mf_plan_set_streams.restype = ctypes.c_int
    lib.mf_plan_set_streams.argtypes = [vp, i32]
    lib.mf_plan_streams.restype = i32
    lib.mf_plan_streams.argtypes = [vp]
    lib.mf_plan_set_timing.restype = ctypes.c_int
    lib.mf_plan_set_timing.argtypes = [vp, ctypes.c_int]
    lib.mf_plan_kernel_times.restype = ctypes.c_int
    lib.mf_plan_kernel_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    lib.mf_stream_read.restype = ctypes.c_int
    lib.mf_stream_read.argtypes = [vp, i64, vp, i32, ctypes.POINTER(ctypes.c_float), vp]
    lib.mf_plan_energy.restype = ctypes.c_int
    lib.mf_plan_energy.argtypes = [vp, vp, vp, vp]
    lib.mf_repack_bil.restype = ctypes.c_int
    lib.mf_repack_bil.argtypes = [vp, i64, i32, i32, vp, vp, i64, i32, ctypes.c_float, vp]
    if lib.mf_abi_version() != ABI_VERSION:
        raise ImportError(f"libmf.so ABI version {lib.mf_abi_version()}, binding expects {ABI_VERSION}")
    _lib = lib
    return lib


def _check(code: int):
    if code != MF_OK:
        lib = load_library()
        raise MFError(code, lib.mf_last_error().decode() or lib.mf_status_str(code).decode())


def default_options() -> Options:
    o = Options()
    load_library().mf_options_default(ctypes.byref(o))
    return o


class Plan:
    """A retrieval plan for a batch of flightlines (see mf_plan_create).

    flightlines: iterable of (first_px, n_columns, n_lines).  Must be created
    with the target GPU current (torch.cuda.set_device).
    """

    def __init__(self, flightlines: Iterable[Tuple[int, int, int]], n_bands: int = 74,
                 n_iter: int = 30, lam: float = 1.0, eps: float = 1e-9, albedo: bool = True,
                 cov: str = "lowrank", refine_steps: int = -1, chunk_lines: int = 0,
                 save_for_backward: bool = False, group: int = 1, track_energy: bool = False):
        lib = load_library()
        o = default_options()
        o.n_bands, o.n_iter, o.albedo = n_bands, n_iter, int(bool(albedo))
        o.lambda_, o.epsilon, o.cov = float(lam), float(eps), COV[cov]
        o.refine_steps, o.chunk_lines = refine_steps, chunk_lines
        o.save_for_backward = int(bool(save_for_backward))
        o.group = int(group)
        o.track_energy = int(bool(track_energy))
        fls = list(flightlines)
        arr = (Flightline * max(1, len(fls)))(*[Flightline(int(a), int(b), int(c)) for a, b, c in fls])
        h = ctypes.c_void_p()
        _check(lib.mf_plan_create(ctypes.byref(o), arr, len(fls), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self.options = o
        self.flightlines = fls
        self.n_bands = n_bands
        self.workspace_bytes = int(lib.mf_workspace_bytes(h))
        self.n_columns = int(lib.mf_plan_columns(h))
        self.n_pixels = int(lib.mf_plan_pixels(h))
        self.refine_steps = int(lib.mf_plan_refine_steps(h))
        self.max_px = max(a + b * c for a, b, c in fls)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.mf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, enable: bool):
        """Replay the launch sequence as one HIP graph (see mf_plan_set_graph)."""
        _check(self._lib.mf_plan_set_graph(self._h, int(bool(enable))))

    def set_launch(self, stream_tile="32x4", wgs_per_cu: int = 0):
        """Launch shape of the streaming passes (see mf_plan_set_launch):
        tile "32x4" | "32x2" | "64x2" | "64x1" (pixels per wave chunk x waves
        per workgroup); wgs_per_cu 0 = one workgroup per work item, n = a
        persistent launch of n workgroups per compute unit with a work queue."""
        t = TILES[stream_tile] if isinstance(stream_tile, str) else int(stream_tile)
        _check(self._lib.mf_plan_set_launch(self._h, t, int(wgs_per_cu)))
        self.stream_tile, self.wgs_per_cu = t, int(wgs_per_cu)

    def set_streams(self, n: int = 1):
        """Run the partitions in n groups, each on its own stream (see
        mf_plan_set_streams); call with the plan's device current."""
        _check(self._lib.mf_plan_set_streams(self._h, int(n)))

    @property
    def streams(self) -> int:
        return int(self._lib.mf_plan_streams(self._h))

    def set_timing(self, enable: bool):
        _check(self._lib.mf_plan_set_timing(self._h, int(bool(enable))))

    def kernel_times(self):
        """{kind: (total_ms, launches)} since the last call (waits for the GPU)."""
        n = len(KERNEL_KINDS)
        t = (ctypes.c_double * n)()
        c = (ctypes.c_int64 * n)()
        _check(self._lib.mf_plan_kernel_times(self._h, t, c, n))
        return {k: (t[i], int(c[i])) for i, k in enumerate(KERNEL_KINDS)}

    def energy(self, workspace, stream=None):
        """E^0..E^K of every partition from the last retrieval on `workspace`
        (a plan made with track_energy=True): float64 [n_iter + 1, n_columns]
        on the workspace's device, NaN from the iteration a partition failed."""
        import torch
        out = torch.empty((self.options.n_iter + 1, self.n_columns), dtype=torch.float64,
                          device=workspace.device)
        if stream is None:
            stream = torch.cuda.current_stream(workspace.device)
        ws = workspace.data_ptr()
        _check(self._lib.mf_plan_energy(self._h, (ws + 255) & ~255, out.data_ptr(), stream.cuda_stream))
        return out

    def alloc_workspace(self, device=None):
        import torch
        return torch.empty(self.workspace_bytes + 256, dtype=torch.uint8,
                           device=device or torch.cuda.current_device())

    def retrieve(self, radiance, s, alpha, valid=None, column_status=None, workspace=None,
                 stream=None):
        """Enqueue one retrieval; tensors are CUDA tensors (contiguous)."""
        import torch
        self._check_io(radiance, s, alpha, valid, column_status)
        if workspace is None:
            workspace = self.alloc_workspace(radiance.device)
        ws = workspace.data_ptr()
        ws_al = (ws + 255) & ~255
        if ws_al + self.workspace_bytes > ws + workspace.numel() * workspace.element_size():
            raise ValueError("workspace too small (allocate workspace_bytes + 256)")
        if stream is None:
            stream = torch.cuda.current_stream(radiance.device)
        _check(self._lib.mf_retrieve(
            self._h, radiance.data_ptr(), None if valid is None else valid.data_ptr(),
            s.data_ptr(), alpha.data_ptr(),
            None if column_status is None else column_status.data_ptr(), ws_al,
            stream.cuda_stream))
        return alpha

    def _check_io(self, radiance, s, alpha, valid, column_status):
        import torch
        B = self.n_bands
        _need(radiance, torch.float32, "radiance")
        _need(s, torch.float32, "s")
        _need(alpha, torch.float32, "alpha")
        if radiance.numel() < self.max_px * B or alpha.numel() < self.max_px or s.numel() != B:
            raise ValueError("radiance/alpha/s are smaller than the plan's geometry")
        if valid is not None:
            _need(valid, torch.uint8, "valid")
            if valid.numel() < self.max_px:
                raise ValueError("valid is smaller than the plan's geometry")
        if column_status is not None:
            _need(column_status, torch.int32, "column_status")
            if column_status.numel() < self.n_columns:
                raise ValueError("column_status is smaller than the number of columns")

    def retrieve_noalloc(self, radiance, s, alpha, valid=None, column_status=None, stream=None):
        """mf_retrieve_noalloc: the same retrieval on the library's fixed device
        scratch (no workspace; plans up to NOALLOC_SCRATCH_BYTES of workspace)."""
        import torch
        self._check_io(radiance, s, alpha, valid, column_status)
        if stream is None:
            stream = torch.cuda.current_stream(radiance.device)
        _check(self._lib.mf_retrieve_noalloc(
            self._h, radiance.data_ptr(), None if valid is None else valid.data_ptr(),
            s.data_ptr(), alpha.data_ptr(),
            None if column_status is None else column_status.data_ptr(), stream.cuda_stream))
        return alpha


def autotune_chunk(flightlines, radiance, s, valid=None, candidates=(512, 1024, 2048, 4096),
                   reps: int = 3, cache_path: Optional[str] = None, **plan_kwargs):
    """Pick chunk_lines (pixels per work item) for a batch geometry by timing
    whole retrievals with each candidate; results are cached in a JSON file
    keyed by the geometry, options and device.  Returns (best, {chunk: ms})."""
    import hashlib
    import json
    import time
    import torch
    fls = [tuple(int(v) for v in f) for f in flightlines]
    key_src = json.dumps([fls, sorted(plan_kwargs.items()), list(candidates),
                          torch.cuda.get_device_name(radiance.device)], default=str)
    key = hashlib.sha256(key_src.encode()).hexdigest()[:20]
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return int(cache[key]["best"]), {int(k): v for k, v in cache[key]["ms"].items()}
    max_px = max(a + b * c for a, b, c in fls)
    alpha = torch.empty(max_px, dtype=torch.float32, device=radiance.device)
    times = {}
    for ch in candidates:
        plan = Plan(fls, chunk_lines=int(ch), **plan_kwargs)
        ws = plan.alloc_workspace(radiance.device)
        plan.retrieve(radiance, s, alpha, valid, None, ws)
        torch.cuda.synchronize(radiance.device)
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.retrieve(radiance, s, alpha, valid, None, ws)
        torch.cuda.synchronize(radiance.device)
        times[int(ch)] = 1e3 * (time.perf_counter() - t0) / reps
        plan.close()
        del ws
    best = min(times, key=times.get)
    if cache_path:
        cache[key] = {"best": best, "ms": times}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, times


def autotune(flightlines, radiance, s, valid=None, chunks=(512, 1024, 2048, 4096),
             tiles=("32x4", "32x2", "64x2", "64x1"), wgs=(0, 1, 2, 3, 4), streams=(1, 2, 3, 4),
             reps: int = 2, cache_path: Optional[str] = None, **plan_kwargs):
    """Pick the launch configuration of a batch geometry by timing whole
    retrievals: the work-item length (chunk_lines) and the number of
    concurrent partition groups (streams) together (the best length depends
    on the group count), then the streaming tile shape (pixels per wave chunk
    x waves per workgroup), then the persistent grid (workgroups per compute
    unit, 0 = one workgroup per work item), each step at the best of the
    previous ones.  Every configuration but the work-item length gives the
    same alpha bit for bit (the length changes the order of the partial
    sums).  Results are cached in a JSON file keyed by the geometry, options,
    candidates and device.  Returns (best, {config: ms}) with best =
    {"chunk_lines", "stream_tile", "wgs_per_cu", "streams"}."""
    import hashlib
    import json
    import time
    import torch
    fls = [tuple(int(v) for v in f) for f in flightlines]
    key_src = json.dumps([fls, sorted(plan_kwargs.items()), list(chunks), list(tiles), list(wgs),
                          list(streams), torch.cuda.get_device_name(radiance.device)], default=str)
    key = hashlib.sha256(key_src.encode()).hexdigest()[:20]
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]["best"], cache[key]["ms"]
    max_px = max(a + b * c for a, b, c in fls)
    alpha = torch.empty(max_px, dtype=torch.float32, device=radiance.device)
    times = {}

    def timed(chunk, tile, w, ns):
        name = f"chunk={chunk},tile={tile},wgs_per_cu={w},streams={ns}"
        if name in times:
            return times[name]
        plan = Plan(fls, chunk_lines=int(chunk), **plan_kwargs)
        plan.set_launch(tile, w)
        plan.set_streams(min(int(ns), plan.n_columns))
        ws = plan.alloc_workspace(radiance.device)
        plan.retrieve(radiance, s, alpha, valid, None, ws)
        torch.cuda.synchronize(radiance.device)
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.retrieve(radiance, s, alpha, valid, None, ws)
        torch.cuda.synchronize(radiance.device)
        times[name] = 1e3 * (time.perf_counter() - t0) / reps
        plan.close()
        del ws
        return times[name]

    best = {"chunk_lines": int(chunks[0]), "stream_tile": tiles[0], "wgs_per_cu": int(wgs[0]),
            "streams": int(streams[0])}
    joint = {(int(c), int(n)): timed(c, best["stream_tile"], best["wgs_per_cu"], n)
             for c in chunks for n in streams}
    best["chunk_lines"], best["streams"] = min(joint, key=joint.get)
    for field, cands in (("stream_tile", tiles), ("wgs_per_cu", wgs)):
        scores = {}
        for c in cands:
            cfg = dict(best, **{field: c})
            scores[c] = timed(cfg["chunk_lines"], cfg["stream_tile"], cfg["wgs_per_cu"], cfg["streams"])
        best[field] = min(scores, key=scores.get)
    if cache_path:
        cache[key] = {"best": best, "ms": times}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, times


def repack_bil(bil, radiance=None, valid=None, first_px: int = 0, nodata=None, stream=None):
    """Band-interleaved-by-line cube bil [n_lines, B, n_samples] (float32,
    GPU) to the retrieval layout: returns (radiance, valid) where radiance is
    [n_samples, n_lines, B] (or, if given, the caller's flat buffer written at
    pixel first_px) and valid the uint8 mask (0 where a band is non-finite or
    equals nodata), or None if valid is False."""
    import torch
    _need(bil, torch.float32, "bil")
    nl, B, ns = bil.shape
    if radiance is None:
        radiance = torch.empty((ns, nl, B), dtype=torch.float32, device=bil.device)
        first_px = 0
    else:
        _need(radiance, torch.float32, "radiance")
        if radiance.numel() < (first_px + ns * nl) * B:
            raise ValueError("radiance buffer is too small")
    if valid is None:
        valid = torch.empty((first_px + ns * nl,) if first_px else (ns, nl), dtype=torch.uint8,
                            device=bil.device)
    elif valid is False:
        valid = None
    if valid is not None:
        _need(valid, torch.uint8, "valid")
        if valid.numel() < first_px + ns * nl:
            raise ValueError("valid buffer is too small")
    if stream is None:
        stream = torch.cuda.current_stream(bil.device)
    _check(load_library().mf_repack_bil(bil.data_ptr(), nl, B, ns, radiance.data_ptr(),
                                        None if valid is None else valid.data_ptr(), first_px,
                                        0 if nodata is None else 1,
                                        0.0 if nodata is None else float(nodata),
                                        stream.cuda_stream))
    return radiance, valid


def stream_read_ms(x, n_blocks: int = 4096) -> float:
    """Time one plain read of the float32 tensor x (the HBM read ceiling)."""
    import torch
    _need(x, torch.float32, "x")
    sink = torch.empty(n_blocks, dtype=torch.float32, device=x.device)
    ms = ctypes.c_float()
    _check(load_library().mf_stream_read(x.data_ptr(), x.numel() - x.numel() % 4, sink.data_ptr(),
                                         n_blocks, ctypes.byref(ms),
                                         torch.cuda.current_stream(x.device).cuda_stream))
    return ms.value


def _plan_backward(plan, radiance, s, grad_alpha, valid=None, workspace=None, stream=None):
    """Enqueue mf_backward; returns (grad_radiance float32 like radiance, grad_s float64 [B])."""
    import torch
    _need(radiance, torch.float32, "radiance")
    _need(s, torch.float32, "s")
    _need(grad_alpha, torch.float32, "grad_alpha")
    if workspace is None:
        raise ValueError("backward needs the forward's workspace")
    if valid is not None:
        _need(valid, torch.uint8, "valid")
    # the library writes every plan pixel; rows outside the plan stay zero
    full = plan.n_pixels * plan.n_bands == radiance.numel()
    grad_L = torch.empty_like(radiance) if full else torch.zeros_like(radiance)
    grad_s = torch.empty(plan.n_bands, dtype=torch.float64, device=radiance.device)
    ws = workspace.data_ptr()
    ws_al = (ws + 255) & ~255
    if stream is None:
        stream = torch.cuda.current_stream(radiance.device)
    _check(plan._lib.mf_backward(plan._h, radiance.data_ptr(),
                                 None if valid is None else valid.data_ptr(), s.data_ptr(),
                                 grad_alpha.data_ptr(), grad_L.data_ptr(), grad_s.data_ptr(),
                                 ws_al, stream.cuda_stream))
    return grad_L, grad_s


Plan.backward = _plan_backward


def _make_autograd():
    import torch

    class RetrieveFunction(torch.autograd.Function):
        """alpha^K of a [S, N, B] radiance cube, differentiable in radiance and s
        through the library's hand-written adjoint (mf_backward)."""

        @staticmethod
        def forward(ctx, radiance, s, n_iter, lam, eps, albedo, valid, refine_steps, chunk_lines,
                    group, streams):
            S, N, B = radiance.shape
            plan = Plan([(0, S, N)], B, n_iter, lam, eps, albedo, "lowrank", refine_steps,
                        chunk_lines, save_for_backward=True, group=group)
            plan.set_streams(min(int(streams), plan.n_columns))
            ws = plan.alloc_workspace(radiance.device)
            L = radiance.detach().contiguous()
            sv = s.detach().contiguous()
            vv = None if valid is None else valid.contiguous()
            alpha = torch.empty((S, N), dtype=torch.float32, device=radiance.device)
            plan.retrieve(L, sv, alpha, vv, None, ws)
            ctx.state = (plan, ws, L, sv, vv)
            return alpha

        @staticmethod
        def backward(ctx, grad_alpha):
            plan, ws, L, sv, vv = ctx.state
            gL, gs = plan.backward(L, sv, grad_alpha.contiguous().float(), vv, ws)
            ctx.state = None
            return gL, gs.to(sv.dtype), None, None, None, None, None, None, None, None, None

    return RetrieveFunction


_RetrieveFunction = None


def retrieve_differentiable(radiance, s, n_iter: int = 30, lam: float = 1.0, eps: float = 1e-9,
                            albedo: bool = True, valid=None, refine_steps: int = -1,
                            chunk_lines: int = 0, group: int = 1, streams: int = 1):
    """alpha [S, N] with autograd support (radiance and s), low-rank form,
    n_iter up to MAX_BACKWARD_ITER; streams: concurrent partition groups of
    both sweeps (Plan.set_streams)."""
    global _RetrieveFunction
    if _RetrieveFunction is None:
        _RetrieveFunction = _make_autograd()
    return _RetrieveFunction.apply(radiance, s, n_iter, lam, eps, albedo, valid, refine_steps,
                                   chunk_lines, group, streams)


def _need(t, dtype, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def retrieve(radiance, s, n_iter: int = 30, lam: float = 1.0, eps: float = 1e-9,
             albedo: bool = True, cov: str = "lowrank", valid=None, refine_steps: int = -1,
             chunk_lines: int = 0, group: int = 1, stream_tile="32x4", wgs_per_cu: int = 0,
             streams: int = 1):
    """Retrieve alpha (ppm*m) for a [S, N, B] float32 radiance cube on the GPU.

    group > 1 pools `group` adjacent columns per partition (the last one takes
    the remainder); stream_tile and wgs_per_cu set the launch shape (see
    Plan.set_launch), streams the concurrent partition groups (see
    Plan.set_streams).  Returns (alpha [S, N] float32, status int32 per
    partition [ceil(S / group)]), both on the GPU.
    """
    import torch
    S, N, B = radiance.shape
    plan = Plan([(0, S, N)], B, n_iter, lam, eps, albedo, cov, refine_steps, chunk_lines,
                group=group)
    plan.set_launch(stream_tile, wgs_per_cu)
    plan.set_streams(min(int(streams), plan.n_columns))
    alpha = torch.empty((S, N), dtype=torch.float32, device=radiance.device)
    status = torch.empty((plan.n_columns,), dtype=torch.int32, device=radiance.device)
    plan.retrieve(radiance.contiguous(), s.contiguous(), alpha,
                  None if valid is None else valid.contiguous(), status)
    return alpha, status

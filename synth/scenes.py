"""Seeded synthetic imaging-spectrometer scenes.

This module only draws inputs: it holds none of the retrieval's arithmetic, and
both the FP64 oracle and the GPU path consume what it returns, bit for bit.

The scenes stand in for AVIRIS-NG flightlines, which are not available here.
Their shapes follow the paper's description of the data: about 600 cross-track
detectors and several thousand along-track lines (Sec. II-B), 5 nm bands
(Sec. II-F), enhancements of up to 10000 ppm*m (Sec. II-D) and a target given
as a unit absorption spectrum s (Sec. II-D, Eq. 9).

Physical model (Beer-Lambert, Sec. II-A):  L = L0 * exp(alpha * s) + n, with
s <= 0 the slope of ln L per ppm*m and alpha >= 0 the enhancement.

Recipe (all random numbers come from numpy PCG64):
  * wavelengths  lambda_b = 2122 + 5 b nm, b = 0..B-1
  * 8 endmembers g_m = sum_{j<4} h_j exp(-(lambda-c_j)^2 / 2 w_j^2),
    c_j ~ U(2000,2600), w_j ~ U(60,250), h_j ~ U(0.2,1);  e_m = 1 + 9 g_m / max g_m
  * s = -kappa sum_{j<20} h_j exp(-(lambda-c_j)^2 / 2 w_j^2), c_j ~ U(2200,2400),
    w_j ~ U(2,8), h_j ~ U(0.2,1); kappa fixed so exp(1000 min s) = 0.97
  * plumes: isotropic Gaussians in (column, line) pixel space, centres uniform,
    cut to exactly 0 beyond 3 sigma
  * per column: albedo a ~ U(0.3,1.5), abundances ~ Dirichlet(1_8),
    L0 = a * (abundances @ E), noise n_b ~ N(0, (0.01 m_b)^2) with m_b the
    expected background mean in band b (0.9 * mean_m e_m(b))
  * optional masks: per column a fraction f ~ U(0, mask_max) in runs of
    length U{1..64} at uniform starts until >= f N pixels are masked; masked
    radiance is NaN so that any leak of an invalid pixel poisons the result.

Every column draws from its own child stream SeedSequence(seed, spawn_key=
(flightline, column)), so any column can be regenerated alone and columns can
be generated in parallel; globals (endmembers, s, plumes) draw from
SeedSequence(seed, spawn_key=(flightline,)).
"""
from __future__ import annotations

import os
from dataclasses import dataclass, replace, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

N_ENDMEMBERS = 8
DIP_AT_1000 = 0.97  # transmittance at 1000 ppm*m at the deepest band


@dataclass(frozen=True)
class SceneSpec:
    n_columns: int
    n_lines: int
    n_bands: int = 74
    n_plumes: int = 3
    peak_range: Tuple[float, float] = (500.0, 5000.0)
    sigma_range: Tuple[float, float] = (3.0, 30.0)
    seed: int = 1000
    flightline: int = 0
    mask_max_frac: float = 0.0     # 0 => no mask
    noise_frac: float = 0.01
    s_flightline: int = -1         # >= 0: use that flightline's target spectrum


@dataclass
class SceneGlobals:
    wavelengths: np.ndarray     # [B] nm
    endmembers: np.ndarray      # [8, B]
    s: np.ndarray               # [B] float32, (ppm*m)^-1, <= 0
    plumes: np.ndarray          # [P, 4]: column, line, sigma, peak
    band_mean: np.ndarray       # [B] expected background mean m_b


@dataclass
class Scene:
    spec: SceneSpec
    radiance: np.ndarray        # [S, N, B] float32
    s: np.ndarray               # [B] float32
    alpha_true: np.ndarray      # [S, N] float64
    valid: Optional[np.ndarray] # [S, N] uint8 or None
    wavelengths: np.ndarray


def _gauss(x, c, w):
    return np.exp(-((x[None, :] - c[:, None]) ** 2) / (2.0 * w[:, None] ** 2))


def make_globals(spec: SceneSpec) -> SceneGlobals:
    rng = np.random.Generator(np.random.PCG64(
        np.random.SeedSequence(spec.seed, spawn_key=(spec.flightline,))))
    B = spec.n_bands
    wl = 2122.0 + 5.0 * np.arange(B, dtype=np.float64)
    # endmembers
    E = np.empty((N_ENDMEMBERS, B))
    for m in range(N_ENDMEMBERS):
        c = rng.uniform(2000.0, 2600.0, 4)
        w = rng.uniform(60.0, 250.0, 4)
        h = rng.uniform(0.2, 1.0, 4)
        g = (h[:, None] * _gauss(wl, c, w)).sum(0)
        E[m] = 1.0 + 9.0 * g / g.max()
    # unit absorption spectrum
    c = rng.uniform(2200.0, 2400.0, 20)
    w = rng.uniform(2.0, 8.0, 20)
    h = rng.uniform(0.2, 1.0, 20)
    shape = (h[:, None] * _gauss(wl, c, w)).sum(0)
    kappa = -np.log(DIP_AT_1000) / 1000.0 / shape.max()
    s = (-kappa * shape).astype(np.float32)
    if spec.s_flightline >= 0 and spec.s_flightline != spec.flightline:
        # one gas and one instrument for a whole batch: a shared spectrum
        # (drawn after this flightline's own, so its other draws are unchanged)
        s = make_globals(replace(spec, flightline=spec.s_flightline, s_flightline=-1)).s
    # plumes
    P = spec.n_plumes
    pc = rng.uniform(0.0, spec.n_columns, P)
    pl = rng.uniform(0.0, spec.n_lines, P)
    ps = rng.uniform(spec.sigma_range[0], spec.sigma_range[1], P)
    pk = rng.uniform(spec.peak_range[0], spec.peak_range[1], P)
    plumes = np.stack([pc, pl, ps, pk], axis=1) if P else np.zeros((0, 4))
    band_mean = 0.9 * E.mean(axis=0)   # E[a] * E[abundance] summed over endmembers
    return SceneGlobals(wl, E, s, plumes, band_mean)


def plume_column(spec: SceneSpec, g: SceneGlobals, col: int) -> np.ndarray:
    """True enhancement alpha (ppm*m) along one column, float64 [N]."""
    N = spec.n_lines
    lines = np.arange(N, dtype=np.float64) + 0.5
    x = col + 0.5
    alpha = np.zeros(N)
    for pc, pl, ps, pk in g.plumes:
        dx = x - pc
        if abs(dx) > 3.0 * ps:
            continue
        r2 = dx * dx + (lines - pl) ** 2
        inside = r2 <= (3.0 * ps) ** 2
        alpha += np.where(inside, pk * np.exp(-r2 / (2.0 * ps * ps)), 0.0)
    return alpha


def make_column(spec: SceneSpec, g: SceneGlobals, col: int):
    """(radiance float32 [N,B], alpha_true float64 [N], valid uint8 [N] or None)."""
    rng = np.random.Generator(np.random.PCG64(
        np.random.SeedSequence(spec.seed, spawn_key=(spec.flightline, col))))
    N, B = spec.n_lines, spec.n_bands
    alpha = plume_column(spec, g, col)
    a = rng.uniform(0.3, 1.5, N)
    ab = rng.dirichlet(np.ones(N_ENDMEMBERS), N)
    L0 = a[:, None] * (ab @ g.endmembers)
    noise = rng.standard_normal((N, B)) * (spec.noise_frac * g.band_mean)[None, :]
    L = L0 * np.exp(alpha[:, None] * g.s.astype(np.float64)[None, :]) + noise
    L = L.astype(np.float32)
    valid = None
    if spec.mask_max_frac > 0.0:
        f = rng.uniform(0.0, spec.mask_max_frac)
        m = np.zeros(N, dtype=bool)
        target = f * N
        while m.sum() < target:
            start = int(rng.integers(0, N))
            run = int(rng.integers(1, 65))
            m[start:start + run] = True
        valid = (~m).astype(np.uint8)
        L[m] = np.nan
    return L, alpha, valid


def make_scene(spec: SceneSpec, workers: int = 0) -> Scene:
    g = make_globals(spec)
    S, N, B = spec.n_columns, spec.n_lines, spec.n_bands
    L = np.empty((S, N, B), dtype=np.float32)
    A = np.empty((S, N), dtype=np.float64)
    V = np.empty((S, N), dtype=np.uint8) if spec.mask_max_frac > 0 else None
    if workers == 0:
        workers = 1 if S * N < 1 << 20 else min(16, len(os.sched_getaffinity(0)))

    def fill(c):
        Lc, ac, vc = make_column(spec, g, c)
        L[c] = Lc
        A[c] = ac
        if V is not None:
            V[c] = vc

    if workers <= 1:
        for c in range(S):
            fill(c)
    else:
        # numpy releases the GIL in its bulk kernels; one BLAS thread per worker
        from concurrent.futures import ThreadPoolExecutor
        try:
            from threadpoolctl import threadpool_limits
            ctx = threadpool_limits(1)
        except Exception:  # pragma: no cover
            ctx = None
        try:
            with ThreadPoolExecutor(workers) as ex:
                list(ex.map(fill, range(S)))
        finally:
            if ctx is not None:
                ctx.unregister() if hasattr(ctx, "unregister") else ctx.restore_original_limits()
    return Scene(spec, L, g.s.copy(), A, V, g.wavelengths)


# ---------------------------------------------------------------------------
# Named workloads

def tiny_spec(seed: int = 1000) -> SceneSpec:
    """64 columns x 512 lines x 74 bands, 3 plumes of 500-5000 ppm*m."""
    return SceneSpec(64, 512, 74, 3, (500.0, 5000.0), (3.0, 30.0), seed)


def flightline_spec(seed: int = 1001, n_lines: int = 8000) -> SceneSpec:
    """598 columns x 8000 lines x 74 bands, 40 plumes of 200-8000 ppm*m."""
    return SceneSpec(598, n_lines, 74, 40, (200.0, 8000.0), (3.0, 30.0), seed)


def diff_spec(seed: int = 1004) -> SceneSpec:
    """598 columns x 4000 lines x 74 bands (the differentiation workload)."""
    return SceneSpec(598, 4000, 74, 40, (200.0, 8000.0), (3.0, 30.0), seed)


def batch_specs(seed: int = 1003, n_flightlines: int = 32,
                n_columns: int = 598) -> List[SceneSpec]:
    """Ragged batch: lengths U{1000..12000}, 0-20 % masked per column, one
    target spectrum (flightline 0's) for the whole batch."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    lens = rng.integers(1000, 12001, n_flightlines)
    return [SceneSpec(n_columns, int(n), 74, 40, (200.0, 8000.0), (3.0, 30.0),
                      seed, f, 0.2, s_flightline=0) for f, n in enumerate(lens)]

/*
 * mf.h - C ABI of the MI355X (gfx950) sparse, albedo-corrected matched-filter
 * methane retrieval.
 *
 * The library computes, for every detector partition (one cross-track column
 * of a pushbroom flightline, Sec. II-E), the iteration of the algorithm figure
 * "AlbedoReWeightL1Filter" (Fig. 1) of Foote et al., "Fast and Accurate
 * Retrieval of Methane Concentration from Imaging Spectrometer Data Using
 * Sparsity Prior", IEEE TGRS 2020:
 *
 *   mu^0 = mean L_i,  C^0 = sample covariance,  r_i = L_i.mu^0 / mu^0.mu^0 (Eq. 7)
 *   alpha^0_i = (L_i - mu^0)^T C^0^-1 t^0 / (r_i t^0^T C^0^-1 t^0),  t = mu (.) s (Eq. 9)
 *   for k = 1..K:
 *     w_i   = lambda / (alpha_i^{k-1} + eps)                            (Eq. 5)
 *     mu^k  = mean (L_i - r_i alpha_i^{k-1} mu^{k-1} (.) s)              (Eq. 10)
 *     C^k   = mean d_i d_i^T, d_i = L_i - r_i alpha_i^{k-1} t^k - mu^k  (Eq. 11)
 *     alpha_i^k = max(((L_i - mu^k)^T C^k^-1 t^k - w_i) / (r_i t^k^T C^k^-1 t^k), 0)
 *                                                                     (Eqs. 6, 8)
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers on the plan's device, owned by the
 *    caller, unless stated otherwise.  The library does not keep them.
 *  - Work is enqueued on the caller's HIP stream (hipStream_t passed as void*;
 *    NULL = the default stream).  No entry point synchronises the stream.
 *  - Argument and shape errors are detected on the host before anything is
 *    enqueued and returned as an mf_status; nothing is launched then.
 *  - Numerical failures are per partition and asynchronous: they are written
 *    to column_status (see MF_COL_*) and the partition's alpha is set to 0.
 *    A partition is one detector column, or `group` adjacent columns
 *    (mf_options.group); "column" below means a partition.
 *  - No C++ exception crosses this boundary.
 *
 * Radiance layout: float32, band-contiguous pixels ("[px][B]").  Flightline f
 * has n_columns columns of n_lines pixels each; pixel (column c, line l) of
 * flightline f is the global pixel index first_px + c * n_lines + l, so each
 * column is a contiguous run of n_lines * B floats.  Flightlines may be
 * ragged and need not be adjacent, but their pixel ranges must not overlap.
 */
#ifndef MF_H
#define MF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__) || defined(__clang__)
#define MF_API __attribute__((visibility("default")))
#else
#define MF_API
#endif

#define MF_ABI_VERSION 4
#define MF_MAX_BANDS 78      /* B + 2 <= 80: five 16-band MFMA blocks */
#define MF_MAX_BACKWARD_ITER 1000  /* n_iter limit of a plan with save_for_backward */

typedef struct mf_plan_s* mf_plan;

typedef enum {
  MF_OK = 0,
  MF_E_ARG = 1,          /* NULL pointer, bad option value, bad struct_size */
  MF_E_SHAPE = 2,        /* inconsistent or overlapping flightline geometry */
  MF_E_UNSUPPORTED = 3,  /* e.g. n_bands outside [2, MF_MAX_BANDS] */
  MF_E_DEVICE = 4,       /* a HIP runtime call failed */
  MF_E_STATE = 5         /* mf_backward without a saved forward */
} mf_status;

/* Per-column status written by mf_retrieve (int32 per column). */
enum {
  MF_COL_OK = 0,
  MF_COL_FEW_PIXELS = 1, /* N_valid <= B: the sample covariance is singular */
  MF_COL_NOT_SPD = 2,    /* Cholesky pivot <= 0, or t^T C^-1 t <= 0 */
  MF_COL_NONFINITE = 3   /* a valid pixel holds NaN or Inf */
};

/* How C^k of Eq. 11 is formed.  Every form computes the same matrix in exact
   arithmetic; they differ in rounding and speed.  The per-pixel scores
   (Eqs. 6-7) and the factorisation are FP64 in every form. */
typedef enum {
  MF_COV_LOWRANK = 0,    /* default.  C^0 from one exact Gram (FP64 MFMA); C^k
                            from C^0 by an exact rank-3 update built from
                            sum c_i (L_i - mean L), sum c_i, sum c_i^2 */
  MF_COV_GRAM_FP64 = 1,  /* a Gram of the residuals every iteration (the
                            paper's canonical formulas, Sec. II-E), FP64 MFMA */
  MF_COV_GRAM_FP32 = 2,  /* ... on FP32 MFMA (FP32 accumulation per wave,
                            FP64 across waves and work items) */
  MF_COV_GRAM_BF16 = 3,  /* ... with BF16 operands on MFMA (FP32 accumulate) */
  MF_COV_GRAM_BF16X3 = 4 /* ... with split BF16 operands: each residual is
                            hi + lo (both BF16, lo the rounded remainder) and
                            the Gram adds hi hi' + hi lo' + lo hi' on the same
                            MFMA (FP32 accumulate).
                            In the three rounded forms the FP64 Cholesky factor
                            of the rounded C^k preconditions iterative
                            refinement whose residual t - C^k v takes C^k
                            exactly (C^0 from the FP64 Gram of the first pass
                            plus the rank-3 update from FP64 moments of the
                            same pass) */
} mf_cov;

typedef struct {
  uint32_t struct_size;   /* = sizeof(mf_options); guards ABI drift */
  int32_t  n_bands;       /* B, 2..MF_MAX_BANDS (74 for the 2122-2487 nm window) */
  int32_t  n_iter;        /* K >= 0 reweighting iterations (the paper uses 30).
                             K = 0 returns alpha^0 unclamped (the non-iterative
                             filter, which has negative values). */
  int32_t  albedo;        /* 1: r_i from Eq. 7; 0: r_i = 1 (Fig. 1 caption) */
  double   lambda;        /* >= 0, weight scale: w = lambda / (alpha + eps).
                             1 = the paper's Eq. 5; 0 = no sparsity prior. */
  double   epsilon;       /* > 0, ppm*m (Eq. 5) */
  int32_t  cov;           /* mf_cov */
  int32_t  refine_steps;  /* iterative-refinement steps of C^-1 t, 0..8, or -1
                             for the form's default: 1 for the exact forms, 3
                             for MF_COV_GRAM_FP32, 5 for MF_COV_GRAM_BF16, 4 for
                             MF_COV_GRAM_BF16X3 (the steps that take the
                             rounded forms to FP64 rounding) */
  int32_t  save_for_backward; /* 1: mf_retrieve keeps alpha^0..alpha^K and the
                             per-iteration column state for mf_backward (needs
                             MF_COV_LOWRANK and n_iter <= MF_MAX_BACKWARD_ITER;
                             a workspace about 32 (K + 1) bytes per pixel larger,
                             plus 8 B per pixel and band when K > 30) */
  int32_t  chunk_lines;   /* pixels per work item along a column (multiple of
                             128; 0 = library default: 1024 for the low-rank
                             form, 4096 for the Gram forms) */
  int32_t  group;         /* detectors per partition (Sec. II-E), >= 1: each run
                             of `group` adjacent columns of a flightline (the
                             last run takes the remainder) shares one mean and
                             covariance; 1 = one partition per column */
  int32_t  track_energy;  /* 1: mf_retrieve also records the objective E^k of
                             every iteration (Eq. 8 with the 1/2 of the alpha
                             update; see mf_plan_energy); needs MF_COV_LOWRANK */
} mf_options;

typedef struct {
  int64_t first_px;       /* global index of pixel (column 0, line 0) */
  int32_t n_columns;      /* detectors (cross-track), >= 1 */
  int32_t n_lines;        /* along-track lines, >= 1 */
} mf_flightline;

/* Library ABI version (MF_ABI_VERSION). */
MF_API int mf_abi_version(void);

/* Fills *opt with defaults: B = 74, K = 30, albedo on, lambda 1, eps 1e-9,
   low-rank covariance form, the form's refinement steps, automatic chunking. */
MF_API void mf_options_default(mf_options* opt);

/* Static text for a status code (never NULL). */
MF_API const char* mf_status_str(mf_status s);

/* Text of the last error raised on this thread by any mf_* call ("" if none). */
MF_API const char* mf_last_error(void);

/* Builds a plan for a batch of flightlines on the current HIP device.  The
   flightline array is host memory and is copied.  The plan owns small device
   tables (work items, column descriptors) allocated here; all per-call device
   memory comes from the caller's workspace.  *out is NULL on error. */
MF_API mf_status mf_plan_create(const mf_options* opt, const mf_flightline* flightlines,
                         int32_t n_flightlines, mf_plan* out);

/* Bytes of device workspace mf_retrieve needs (256-byte aligned start). */
MF_API size_t mf_workspace_bytes(mf_plan plan);

/* Number of partitions (columns when group = 1, else sum over flightlines of
   ceil(n_columns / group)) and of pixels (sum of n_columns * n_lines). */
MF_API int64_t mf_plan_columns(mf_plan plan);
MF_API int64_t mf_plan_pixels(mf_plan plan);

/* Refinement steps the plan's solves take (refine_steps, or the form's
   default when it was -1); -1 for a NULL plan. */
MF_API int32_t mf_plan_refine_steps(mf_plan plan);

/* Runs Fig. 1 on every column of the plan.
     radiance       [max_px][B] float32, uW cm^-2 sr^-1 nm^-1 (read only); any
                    float-aligned pointer (16-byte alignment is not required)
     valid          [max_px] uint8, nonzero = valid pixel, or NULL (all valid).
                    Invalid pixels are excluded from every mean and covariance
                    (censored data is skipped, Sec. III-A) and get alpha = 0;
                    their radiance values are ignored (the memory must exist).
     s              [B] float32 unit absorption spectrum, (ppm*m)^-1 (Sec. II-D)
     alpha          [max_px] float32 output, ppm*m; only the plan's pixels are written
     column_status  [mf_plan_columns] int32 output (MF_COL_*), or NULL
     workspace      device memory of mf_workspace_bytes(plan), 256-byte aligned;
                    contents need not be initialised and are clobbered
     stream         hipStream_t or NULL
   max_px is the largest first_px + n_columns * n_lines over the flightlines.
   Calls that share a workspace must be ordered on one stream. */
MF_API mf_status mf_retrieve(mf_plan plan, const float* radiance, const uint8_t* valid,
                      const float* s, float* alpha, int32_t* column_status,
                      void* workspace, void* stream);

/* mf_retrieve without a workspace argument, for callers that cannot
   allocate device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc): the workspace is a fixed device array of
   MF_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
   until the process ends, so this call allocates nothing.  Arguments,
   outputs and errors as mf_retrieve, plus:
     MF_E_UNSUPPORTED  mf_workspace_bytes(plan) > MF_NOALLOC_SCRATCH_BYTES
                       (e.g. up to about 1.2 M pixels of 74 bands at K = 30 in
                       the low-rank form), or a plan with save_for_backward
                       or track_energy (their state would live in the scratch)
     MF_E_STATE        kernel timing is on for the plan
   Every call on one GPU shares that GPU's scratch and leaves its contents
   there: calls that may overlap on one GPU (different streams, or threads)
   race and must be ordered by the caller.  Plain launches (no graph replay).
   The plan itself is created beforehand (mf_plan_create allocates its tables). */
#define MF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
MF_API mf_status mf_retrieve_noalloc(mf_plan plan, const float* radiance, const uint8_t* valid,
                                     const float* s, float* alpha, int32_t* column_status,
                                     void* stream);

/* Adjoint of mf_retrieve (reverse mode through the K unrolled iterations of
   Fig. 1): given grad_alpha = dJ/dalpha^K for a scalar loss J (e.g.
   J = sum (alpha^K - alpha_true)^2 gives 2 (alpha^K - alpha_true)), writes
     grad_radiance [max_px][B] float32 = dJ/dL  (0 on invalid pixels and on
                   columns whose status is not MF_COL_OK; only plan pixels written)
     grad_s        [B] float64 = dJ/ds summed over every column
   The plan needs save_for_backward = 1, and the preceding mf_retrieve on the
   same workspace (and the same radiance, valid and s) must be ordered before
   it on the stream.  The derivative of max(z, 0) is 1 for z > 0, else 0.
   Device pointers; enqueued on the stream. */
MF_API mf_status mf_backward(mf_plan plan, const float* radiance, const uint8_t* valid,
                             const float* s, const float* grad_alpha, float* grad_radiance,
                             double* grad_s, void* workspace, void* stream);

/* Per-iteration energy (Sec. III-B, Eq. 8): after an mf_retrieve of a plan
   created with track_energy = 1, copies E^0..E^K of every partition into
   energy_out [K + 1][mf_plan_columns] float64 (device memory), where
     E^k = sum_i 1/2 (L_i - r_i alpha^k_i t^k - mu^k)^T C^k^-1 (.)
           + r_i w^k_i alpha^k_i,   w^0 = 0, w^k = lambda / (alpha^{k-1} + eps),
   the sum over the partition's valid pixels, alpha^0 clamped at 0 when K >= 1
   (the objective each alpha update minimises with mu^k and C^k held fixed).
   Entries of a partition whose status is not MF_COL_OK are NaN from the
   iteration where it failed on.  The retrieval on the same workspace must be
   ordered before this call on the stream; enqueued on the stream. */
MF_API mf_status mf_plan_energy(mf_plan plan, const void* workspace, double* energy_out,
                                void* stream);

/* Graph replay.  While enabled, mf_retrieve captures its launch sequence on
   the caller's stream into a HIP graph the first time it sees a set of
   pointers and stream, and replays it (one graph launch) on later calls with
   the same set; a different set is captured anew.  Not used on the NULL
   stream or while kernel timing is on (plain launches then). */
MF_API mf_status mf_plan_set_graph(mf_plan plan, int enable);

/* Launch shape of the streaming passes (a tuning choice: every shape gives
   the same result, bit for bit).
     stream_tile  MF_TILE_*: pixels per wave chunk x waves per workgroup of the
                  low-rank form's streaming passes
     wgs_per_cu   0: one workgroup per work item (the default); n in [1, 16]:
                  one persistent launch per pass with n workgroups per compute
                  unit, which take the work items (longest first) from a
                  per-pass queue counter in the workspace (cleared by the
                  retrieval itself, no memset); no workgroup waits for another
   A graph captured with the previous shape is dropped. */
enum {
  MF_TILE_32x4 = 0,  /* 32-pixel chunks (two lanes per pixel), 4 waves (default) */
  MF_TILE_32x2 = 1,
  MF_TILE_64x2 = 2,  /* 64-pixel chunks (one lane per pixel) */
  MF_TILE_64x1 = 3
};
MF_API mf_status mf_plan_set_launch(mf_plan plan, int32_t stream_tile, int32_t wgs_per_cu);

/* Concurrent partition groups (a tuning choice: every setting gives the same
   result, bit for bit).  The partitions are independent problems (Sec. II-E),
   so mf_retrieve splits the plan's partitions into n_streams contiguous
   groups of about equal pixel counts and runs each group's launch sequence
   on its own stream: group 0 on the caller's stream, the others on streams
   the plan owns (default priority), forked from the caller's stream by an
   event at the start and joined back into it before the call's last launch.
   The call therefore still orders like one launch sequence on the caller's
   stream.  While one group's streaming pass drains or its latency-bound
   solves run, another group's pass keeps the GPU busy.
     n_streams   1 (the default) .. MF_MAX_STREAMS, at most the plan's
                 partitions
   Call it with the plan's device current: it creates the streams and events
   on first use (mf_retrieve and mf_retrieve_noalloc only record and wait on
   them).  Graph capture follows the fork and join; a graph captured with the
   previous setting is dropped.  With persistent launches (wgs_per_cu > 0)
   each group takes its work items in plan order from its own counters.
   mf_backward runs its reverse sweep the same way, one group per stream.
   Two calls on one plan that overlap in time race on these streams, as they
   would on the workspace. */
#define MF_MAX_STREAMS 8
MF_API mf_status mf_plan_set_streams(mf_plan plan, int32_t n_streams);

/* The plan's current n_streams. */
MF_API int32_t mf_plan_streams(mf_plan plan);

/* Kernel timing for benchmarks.  While enabled, mf_retrieve brackets each of
   its kernel launches with HIP events on the caller's stream (a few
   microseconds of extra stream work per launch). */
enum {
  MF_KERNEL_PASS_GRAM = 0,  /* scored pass (1..K) that also accumulates a Gram */
  MF_KERNEL_PASS_VEC = 1,   /* streaming pass of the low-rank form (vector moments) */
  MF_KERNEL_PASS_LAST = 2,  /* final streaming pass (alpha^K only) */
  MF_KERNEL_SOLVE = 3,      /* per-column FP64 combine, Cholesky and solve */
  MF_KERNEL_OTHER = 4,      /* setup and status copy */
  MF_KERNEL_PASS_INIT = 5,  /* pass 0: the FP64 Gram of C^0 (every form) */
  MF_KERNEL_KINDS = 6
};
MF_API mf_status mf_plan_set_timing(mf_plan plan, int enable);

/* Waits for every event recorded since the last call, then writes the summed
   kernel time in milliseconds (times_ms[kind]) and the number of launches
   (counts[kind]) for kind < n (n <= MF_KERNEL_KINDS), and clears the record.
   Either output pointer may be NULL.  Host pointers. */
MF_API mf_status mf_plan_kernel_times(mf_plan plan, double* times_ms, int64_t* counts, int n);

/* Ingest: repacks a band-interleaved-by-line cube bil [n_lines][n_bands]
   [n_samples] (the ENVI "BIL" layout of imaging-spectrometer radiance files,
   one detector per sample) into the column-contiguous layout mf_retrieve
   reads: pixel (sample c, line l) goes to radiance[first_px + c * n_lines + l]
   (n_bands floats), i.e. one flightline of n_samples columns and n_lines lines
   starting at first_px.  If valid is non-NULL, valid[that pixel] = 0 when any
   band is NaN or +-Inf, or (use_nodata = 1) equals nodata exactly, else 1
   (censored samples are excluded from the statistics, Sec. III-A).  Device
   pointers; bil and radiance must not overlap; enqueued on the stream. */
MF_API mf_status mf_repack_bil(const float* bil, int64_t n_lines, int32_t n_bands,
                               int32_t n_samples, float* radiance, uint8_t* valid,
                               int64_t first_px, int32_t use_nodata, float nodata,
                               void* stream);

/* Diagnostic: reads n floats of src (device, 16-byte aligned, n a multiple of
   4) once with n_blocks workgroups, each reading a contiguous span of about
   n / n_blocks floats (at most 2^29) with the streaming passes' non-temporal
   loads, and discards them: the achievable HBM read bandwidth used as the
   measured ceiling of the streaming passes.  sink (device, n_blocks floats) is
   never written in practice.  If ms_out (host) is non-NULL the call waits and
   stores the kernel time measured with HIP events.  MF_E_ARG for a span over
   2^29 floats. */
MF_API mf_status mf_stream_read(const float* src, int64_t n, float* sink, int32_t n_blocks,
                                float* ms_out, void* stream);

/* Releases the plan and its device tables (synchronises the device first). */
MF_API void mf_plan_destroy(mf_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* MF_H */

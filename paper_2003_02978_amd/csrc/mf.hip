// MI355X (gfx950) kernels and C ABI of the albedo-corrected reweighted-l1
// matched filter (Foote et al., IEEE TGRS 2020, Fig. 1; Eqs. 5-11).
//
// Data flow of one retrieval (one stream, no host synchronisation):
//   setup      one wave per column: shift point z = first valid pixel
//   pass j=0   per pixel y = L - z; Gram of [y, 1] on MFMA      -> partials
//   solve j=0  FP64: mu^0, C^0, Cholesky, v^0 = C^0^-1 t^0, q^0  -> column state
//   pass j     (1 <= j <= K+1) per pixel p = (L - mu^{j-1}).v^{j-1},
//              r = L.mu^0/|mu^0|^2, alpha^{j-1} (soft threshold, Eq. 6/8),
//              c = r alpha^{j-1}, and the moments the covariance needs (j <= K)
//   solve j    FP64: mu^j = mean(L) - mean(c) t^{j-1} (Eq. 10), C^j (Eq. 11),
//              Cholesky, v^j, q^j
// The last pass writes alpha^K to the caller's buffer and computes no moments.
//
// Covariance forms (mf_cov), all exact algebra for C^j of Eq. 11:
//  * per-iteration Gram (GRAM_FP64 / GRAM_FP32 / GRAM_BF16 / GRAM_BF16X3).  With d_i the
//    residual of Eq. 11 and y_i = L_i - mu_used - c_i t_used as the pass
//    computed it (mu_used, t_used = the FP32 values it subtracted),
//      d_i = y_i + D + c_i e,   D = mu_used - mu^j,   e = t_used - t^j,
//      N C^j = G + g1 D^T + D g1^T + g2 e^T + e g2^T + N D D^T
//              + S1 (D e^T + e D^T) + S2 e e^T,
//    G = sum y y^T, g1 = sum y, g2 = sum c y, S1 = sum c, S2 = sum c^2,
//    N = sum 1.  The pass gets g1, g2, N, S1, S2 for free by appending the
//    constants 1 and c to each pixel's vector as two extra "bands" of the Gram.
//  * LOWRANK (default): the Gram is formed once, exactly (FP64 MFMA), for C^0.
//    With Lt_i = L_i - mean(L), a = S1/N and m = sum c_i Lt_i,
//      N C^j = N C^0 + N a^2 (t^{j-1} - t^j)(t^{j-1} - t^j)^T
//              + (S2 - N a^2) t^j t^j^T - (m t^j^T + t^j m^T),
//    so each later pass only accumulates the vector m and S1, S2.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mf.h"

namespace {

#include "layout.inc"
#include "setup.inc"
#include "gram_pass.inc"
#include "stream_pass.inc"
#include "solve.inc"
#include "adjoint.inc"
#include "misc.inc"

// ---------------------------------------------------------------------------
// Device scratch of mf_retrieve_noalloc: the workspace of plans small enough
// to need no caller memory.  Every GPU the library runs on holds its own copy
// for the life of the process; in host code `scratch` is only a symbol
// handle, so kernels receive the per-device address from hipGetSymbolAddress.
constexpr size_t kScratchBytes = MF_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// ---------------------------------------------------------------------------
// Host side

thread_local std::string g_last_error;

constexpr int kMaxDevices = 64;
constexpr int kMaxBackwardIter = MF_MAX_BACKWARD_ITER;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once per
// device, at plan creation); null and a message if the lookup fails.
void* scratch_address(int device, std::string& err) {
  if (device < 0 || device >= kMaxDevices) {
    err = "device index beyond the scratch table";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

mf_status fail_with(mf_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct GraphKey {
  const void *L, *valid, *s, *alpha, *status, *ws, *stream;
  bool operator==(const GraphKey& o) const {
    return L == o.L && valid == o.valid && s == o.s && alpha == o.alpha && status == o.status &&
           ws == o.ws && stream == o.stream;
  }
};

struct TimedLaunch {
  int kind;
  hipEvent_t start, stop;
};

struct mf_plan_s {
  mf_options opt;
  bool wide = false;         // band layout of the passes (B >= 64)
  bool timing = false;
  bool use_graph = false;
  GraphKey graph_key{};
  hipGraphExec_t graph_exec = nullptr;
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> event_pool;
  int nb = 0;
  int device = 0;
  int64_t n_cols = 0, n_items = 0, n_px = 0, max_px = 0;
  int64_t n_words = 0;       // sparse alpha: mask words (32-pixel pieces of every work item)
  ColInfo* cols_d = nullptr;
  WorkItem* items_d = nullptr;
  size_t off_state = 0, off_partials = 0, off_c0 = 0, off_pinv = 0, off_alpha0 = 0, off_alpha1 = 0;
  size_t off_mask0 = 0, off_mask1 = 0;   // sparse alpha: one word per 32-pixel piece
  size_t off_ck_mask = 0;                // save_for_backward: the masks of alpha^0..alpha^K
  // save_for_backward: checkpoints and adjoint buffers
  size_t off_r = 0, off_ck_alpha = 0, off_ck_col = 0, off_ck_p = 0, off_bw_px = 0, off_bw_coef = 0, off_bw_u = 0,
         off_bw_col = 0, off_bw_acc = 0;
  size_t off_energy = 0;     // track_energy: E^k per partition [K+1][n_cols]
  size_t ws_bytes = 0;
  void* scratch_d = nullptr; // this device's `scratch` (mf_retrieve_noalloc)
  // launch shape of the passes (mf_plan_set_launch)
  int stream_tile = 0;       // MF_TILE_*
  int wgs_per_cu = 0;        // 0: one workgroup per work item; n: persistent grid
  int n_cu = 0;
  int32_t* order_d = nullptr; // work items, longest first (persistent launches)
  size_t off_queue = 0;      // K + 2 queue counters per column group
  // column groups (mf_plan_set_streams): group g holds columns
  // [grp_col[g], grp_col[g + 1]) and their work items [grp_item[g],
  // grp_item[g + 1]); group 0 runs on the caller's stream, group g >= 1 on
  // aux[g - 1], forked from and joined to the caller's stream by events
  int n_groups = 1;
  std::vector<int64_t> grp_col, grp_item;
  std::vector<ColInfo> cols_h;          // host copy of the column table
  hipStream_t aux[MF_MAX_STREAMS - 1] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[MF_MAX_STREAMS - 1] = {};
};

namespace {

hipEvent_t take_event(mf_plan_s* p) {
  hipEvent_t e = nullptr;
  if (!p->event_pool.empty()) {
    e = p->event_pool.back();
    p->event_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

// Records events around one launch when timing is on.
struct LaunchTimer {
  mf_plan_s* p;
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  LaunchTimer(mf_plan_s* p_, int kind_, hipStream_t s_) : p(p_), kind(kind_), s(s_) {
    if (p->timing) {
      a = take_event(p);
      b = take_event(p);
      if (a && b) (void)hipEventRecord(a, s);
    }
  }
  ~LaunchTimer() {
    if (a && b) {
      (void)hipEventRecord(b, s);
      p->pending.push_back({kind, a, b});
    } else {
      if (a) p->event_pool.push_back(a);
      if (b) p->event_pool.push_back(b);
    }
  }
};

// Grid of a pass: one workgroup per work item, or the persistent grid of
// wgs_per_cu workgroups per compute unit (at most one per work item).
unsigned pass_grid(const mf_plan_s* p, const PassArgs& a) {
  if (!a.queue) return (unsigned)a.n_items;
  return (unsigned)std::min<int64_t>(a.n_items, (int64_t)p->wgs_per_cu * p->n_cu);
}

template <int CHUNK, int SW>
void launch_stream(const mf_plan_s* p, const PassArgs& a, int mode, hipStream_t s) {
  using T = StreamTile<CHUNK, SW>;
  const dim3 g(pass_grid(p, a)), b(T::kThreads);
  if (a.queue) {                           // + the ticket slot
    if (mode == PM_NONE) hipLaunchKernelGGL((stream_kernel<PM_NONE, CHUNK, SW, true>), g, b, T::kLds + 16, s, a);
    else hipLaunchKernelGGL((stream_kernel<PM_VEC, CHUNK, SW, true>), g, b, T::kLds + 16, s, a);
  } else {
    if (mode == PM_NONE) hipLaunchKernelGGL((stream_kernel<PM_NONE, CHUNK, SW, false>), g, b, T::kLds, s, a);
    else hipLaunchKernelGGL((stream_kernel<PM_VEC, CHUNK, SW, false>), g, b, T::kLds, s, a);
  }
}

template <int NB, bool WIDE>
void launch_pass_nb(const mf_plan_s* p, const PassArgs& a, int mode, hipStream_t s) {
  const dim3 g((unsigned)a.n_items), b(kBlock);
  const bool sc = a.j >= 1;
  const bool rin = a.r_in != nullptr;
  switch (mode) {
    case PM_F64:
      if (!sc) hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_F64, false, false>), g, b, 0, s, a);
      else if (rin) hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_F64, true, true>), g, b, 0, s, a);
      else hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_F64, true, false>), g, b, 0, s, a);
      break;
    case PM_F32:      // scored passes only (pass 0 is FP64 in every form)
      if (rin) hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_F32, true, true>), g, b, 0, s, a);
      else hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_F32, true, false>), g, b, 0, s, a);
      break;
    case PM_BF16:
      if (rin) hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_BF16, true, true>), g, b, 0, s, a);
      else hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_BF16, true, false>), g, b, 0, s, a);
      break;
    default:
      if (rin) hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_BF16X3, true, true>), g, b, 0, s, a);
      else hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_BF16X3, true, false>), g, b, 0, s, a);
      break;
  }
}

void dispatch_pass(const mf_plan_s* p, const PassArgs& a, int mode, hipStream_t s) {
  if (mode == PM_NONE || mode == PM_VEC) {
    switch (p->stream_tile) {
      case MF_TILE_32x2: launch_stream<32, 2>(p, a, mode, s); break;
      case MF_TILE_64x2: launch_stream<64, 2>(p, a, mode, s); break;
      case MF_TILE_64x1: launch_stream<64, 1>(p, a, mode, s); break;
      default: launch_stream<32, 4>(p, a, mode, s); break;
    }
    return;
  }
  switch (p->nb) {
    case 1: launch_pass_nb<1, false>(p, a, mode, s); break;
    case 2: launch_pass_nb<2, false>(p, a, mode, s); break;
    case 3: launch_pass_nb<3, false>(p, a, mode, s); break;
    case 4: launch_pass_nb<4, false>(p, a, mode, s); break;
    default:
      if (p->wide) launch_pass_nb<5, true>(p, a, mode, s);
      else launch_pass_nb<5, false>(p, a, mode, s);
      break;
  }
}

void dispatch_solve(const mf_plan_s* p, const SolveArgs& a, int64_t n_cols, hipStream_t s) {
  const dim3 g((unsigned)n_cols), b(kBlock);
  switch (p->nb) {
    case 1: hipLaunchKernelGGL((solve_kernel<1, false>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((solve_kernel<2, false>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((solve_kernel<3, false>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((solve_kernel<4, false>), g, b, 0, s, a); break;
    default:
      if (p->wide) hipLaunchKernelGGL((solve_kernel<5, true>), g, b, 0, s, a);
      else hipLaunchKernelGGL((solve_kernel<5, false>), g, b, 0, s, a);
      break;
  }
}

// The Gram forms with rounded operands (FP32, BF16, split BF16): their solve
// refines against the exact C^j from FP64 moments kept beside the Gram.
bool rounded_form(int cov) {
  return cov == MF_COV_GRAM_FP32 || cov == MF_COV_GRAM_BF16 || cov == MF_COV_GRAM_BF16X3;
}

// Doubles per work item in the partial buffer: the item's partial Gram (T
// tiles of 16 x 16; the low-rank form's vector moments fit in it), plus the
// exact moments of the rounded Gram forms.
int64_t partial_stride(const mf_plan_s* p) {
  const bool rounded = rounded_form(p->opt.cov);
  return (int64_t)n_tiles(p->nb) * 256 + (rounded ? kXMomSlots : 0);
}

// Refinement steps of a form when the options ask for the default (-1): the
// exact forms refine once; the rounded Gram forms converge to FP64 rounding
// in 3 (FP32 Gram) and 5 (BF16 Gram) steps against the exact C^j.
int refine_steps_of(const mf_options& o) {
  if (o.refine_steps >= 0) return o.refine_steps;
  switch (o.cov) {
    case MF_COV_GRAM_FP32: return 3;
    case MF_COV_GRAM_BF16: return 5;
    case MF_COV_GRAM_BF16X3: return 4;
    default: return 1;
  }
}

// Pass mode of pass j for a covariance form.
int pass_mode(int cov, int j, int K) {
  if (j == K + 1) return PM_NONE;
  // pass 0 is the exact FP64 Gram in every form: C^0 anchors the rounded
  // forms' refinement (and gives the exact alpha^0)
  switch (cov) {
    case MF_COV_GRAM_FP32: return j == 0 ? PM_F64 : PM_F32;
    case MF_COV_GRAM_BF16: return j == 0 ? PM_F64 : PM_BF16;
    case MF_COV_GRAM_BF16X3: return j == 0 ? PM_F64 : PM_BF16X3;
    case MF_COV_GRAM_FP64: return PM_F64;
    default: return j == 0 ? PM_F64 : PM_VEC;   // MF_COV_LOWRANK
  }
}


}  // namespace

namespace {
// The launch sequence of one retrieval (also what a graph captures).  Each
// column group runs its own sequence on its own stream; the groups share
// nothing but the read-only inputs, so their launches interleave freely on
// the GPU (one group's streaming pass fills the machine while another drains
// or solves).
void enqueue_retrieve(mf_plan_s* p, const float* radiance, const uint8_t* valid, const float* s,
                      float* alpha, int32_t* column_status, void* workspace, hipStream_t st) {
  char* ws = (char*)workspace;
  ColState* state = (ColState*)(ws + p->off_state);
  double* partials = (double*)(ws + p->off_partials);
  double* abuf[2] = {(double*)(ws + p->off_alpha0), (double*)(ws + p->off_alpha1)};
  uint32_t* mbuf[2] = {(uint32_t*)(ws + p->off_mask0), (uint32_t*)(ws + p->off_mask1)};
  const int64_t mask_words = p->n_words + 2;
  uint32_t* ck_mask = p->opt.save_for_backward ? (uint32_t*)(ws + p->off_ck_mask) : nullptr;
  double* ck_alpha = p->opt.save_for_backward ? (double*)(ws + p->off_ck_alpha) : nullptr;
  double* ck_p = p->opt.save_for_backward ? (double*)(ws + p->off_ck_p) : nullptr;
  const int B = p->opt.n_bands;
  const int K = p->opt.n_iter;
  const int G = p->n_groups;
  double* energy = p->opt.track_energy ? (double*)(ws + p->off_energy) : nullptr;
  int* queue = p->wgs_per_cu > 0 ? (int*)(ws + p->off_queue) : nullptr;
  hipStream_t gs[MF_MAX_STREAMS];
  gs[0] = st;
  if (G > 1) {
    (void)hipEventRecord(p->fork_ev, st);
    for (int g = 1; g < G; ++g) {
      gs[g] = p->aux[g - 1];
      (void)hipStreamWaitEvent(gs[g], p->fork_ev, 0);
    }
  }

  PassArgs pa{};
  pa.L = radiance;
  pa.valid = valid;
  pa.items = p->items_d;
  pa.state = state;
  pa.partials = partials;
  pa.B = B;
  pa.albedo = p->opt.albedo;
  pa.lam = p->opt.lambda;
  pa.eps = p->opt.epsilon;
  pa.n_floats = p->max_px * B;
  pa.partial_stride = (int)partial_stride(p);
  pa.order = G == 1 ? p->order_d : nullptr;   // longest-first order over the whole plan
  SolveArgs sa{};
  sa.cols = p->cols_d;
  sa.state = state;
  sa.partials = partials;
  sa.c0 = (double*)(ws + p->off_c0);
  sa.pinv = (double*)(ws + p->off_pinv);
  sa.partial_stride = (int)partial_stride(p);
  sa.s = s;
  sa.B = B;
  sa.refine = refine_steps_of(p->opt);
  sa.lowrank = p->opt.cov == MF_COV_LOWRANK;
  sa.exact_ref = rounded_form(p->opt.cov);
  sa.ck = p->opt.save_for_backward ? (double*)(ws + p->off_ck_col) : nullptr;
  sa.n_cols = (int)p->n_cols;
  sa.energy = energy;
  // a group's queue counters: K + 2 per group
  auto group_queue = [&](int g) { return queue ? queue + (int64_t)g * (K + 2) : nullptr; };
  for (int g = 0; g < G; ++g) {
    const int64_t c0 = p->grp_col[g], nc = p->grp_col[g + 1] - c0;
    LaunchTimer tm(p, MF_KERNEL_OTHER, gs[g]);
    hipLaunchKernelGGL(setup_kernel, dim3((unsigned)nc), dim3(64), 0, gs[g], radiance, valid, p->cols_d,
                       state, B, energy, K + 1, p->n_cols, group_queue(g), K + 2, (int)c0);
  }
  // pass j and solve j of every group before pass j + 1 of any, so that the
  // groups start together
  for (int j = 0; j <= K + 1; ++j) {
    pa.j = j;
    pa.track_energy = (energy && j >= 1) ? 1 : 0;
    pa.unclamped = (j == 1 && K == 0) ? 1 : 0;
    if (ck_alpha) {          // save_for_backward: keep alpha^0..alpha^K
      pa.alpha_prev = j >= 2 ? ck_alpha + (int64_t)(j - 2) * p->max_px : nullptr;
      pa.alpha_out = j >= 1 ? ck_alpha + (int64_t)(j - 1) * p->max_px : nullptr;
    } else {
      pa.alpha_prev = j >= 2 ? abuf[(j - 2) & 1] : nullptr;
      pa.alpha_out = (j >= 1 && j <= K) ? abuf[(j - 1) & 1] : nullptr;
    }
    // sparse alpha between the passes, the checkpoints included (each
    // checkpoint with its own mask array)
    if (ck_alpha) {
      pa.mask_prev = j >= 2 ? ck_mask + (int64_t)(j - 2) * mask_words : nullptr;
      pa.mask_out = j >= 1 ? ck_mask + (int64_t)(j - 1) * mask_words : nullptr;
    } else {
      pa.mask_prev = pa.alpha_prev ? mbuf[(j - 2) & 1] : nullptr;
      pa.mask_out = pa.alpha_out ? mbuf[(j - 1) & 1] : nullptr;
    }
    pa.alpha_final = j == K + 1 ? alpha : nullptr;
    pa.p_save = (ck_p && j >= 1) ? ck_p + (int64_t)(j - 1) * p->max_px : nullptr;
    // r per pixel: written by pass 1 (the adjoint reads it too), read by the
    // later Gram passes; the streaming passes form it again from the
    // radiance tile they hold (same arithmetic as pass 1), which costs FP64
    // FMAs they have room for and saves 8 bytes per pixel of traffic
    const bool mom = j <= K;
    const int mode = pass_mode(p->opt.cov, j, K);
    double* rbuf = (double*)(ws + p->off_r);
    // (read by the Gram passes and the adjoint; the low-rank form's
    // streaming passes without checkpoints have no reader, so skip the write)
    pa.r_out = (j == 1 && (p->opt.cov != MF_COV_LOWRANK || ck_alpha)) ? rbuf : nullptr;
    pa.r_in = (j >= 2 && mode != PM_VEC && mode != PM_NONE) ? rbuf : nullptr;
    sa.j = j;
    for (int g = 0; g < G; ++g) {
      pa.queue = queue ? group_queue(g) + j : nullptr;
      pa.item_base = (int)p->grp_item[g];
      pa.n_items = (int)(p->grp_item[g + 1] - p->grp_item[g]);
      {
        LaunchTimer tm(p, j == 0 ? MF_KERNEL_PASS_INIT
                          : mode == PM_NONE ? MF_KERNEL_PASS_LAST
                          : mode == PM_VEC ? MF_KERNEL_PASS_VEC : MF_KERNEL_PASS_GRAM, gs[g]);
        dispatch_pass(p, pa, mode, gs[g]);
      }
      if (mom) {
        sa.col_base = (int)p->grp_col[g];
        const int64_t nc = p->grp_col[g + 1] - p->grp_col[g];
        LaunchTimer tm(p, MF_KERNEL_SOLVE, gs[g]);
        if (sa.lowrank && j >= 1)
          hipLaunchKernelGGL(lowrank_kernel, dim3((unsigned)nc), dim3(kBlock), 0, gs[g], sa);
        else
          dispatch_solve(p, sa, nc, gs[g]);
      }
    }
  }
  if (G > 1)
    for (int g = 1; g < G; ++g) {
      (void)hipEventRecord(p->join_ev[g - 1], gs[g]);
      (void)hipStreamWaitEvent(st, p->join_ev[g - 1], 0);
    }
  if (energy) {
    LaunchTimer tm(p, MF_KERNEL_OTHER, st);
    hipLaunchKernelGGL(energy_last_kernel, dim3((unsigned)((p->n_cols + 255) / 256)), dim3(256), 0, st,
                       (const ColInfo*)p->cols_d, (const ColState*)state, (const double*)partials,
                       partial_stride(p), energy + (int64_t)K * p->n_cols, p->n_cols);
  }
  if (column_status) {
    const unsigned nb = (unsigned)((p->n_cols + 255) / 256);
    LaunchTimer tm(p, MF_KERNEL_OTHER, st);
    hipLaunchKernelGGL(status_kernel, dim3(nb), dim3(256), 0, st, state, column_status, p->n_cols);
  }
}

}  // namespace

extern "C" {

int mf_abi_version(void) { return MF_ABI_VERSION; }

void mf_options_default(mf_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(mf_options);
  o->n_bands = 74;
  o->n_iter = 30;
  o->albedo = 1;
  o->lambda = 1.0;
  o->epsilon = 1e-9;
  o->cov = MF_COV_LOWRANK;
  o->refine_steps = -1;
  o->save_for_backward = 0;
  o->chunk_lines = 0;
  o->group = 1;
  o->track_energy = 0;
}

const char* mf_status_str(mf_status s) {
  switch (s) {
    case MF_OK: return "ok";
    case MF_E_ARG: return "invalid argument";
    case MF_E_SHAPE: return "invalid shape";
    case MF_E_UNSUPPORTED: return "unsupported configuration";
    case MF_E_DEVICE: return "HIP runtime error";
    case MF_E_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* mf_last_error(void) { return g_last_error.c_str(); }

mf_status mf_plan_create(const mf_options* opt, const mf_flightline* fl, int32_t n_fl,
                         mf_plan* out) {
  if (!out) return fail_with(MF_E_ARG, "out is NULL");
  *out = nullptr;
  if (!opt || !fl) return fail_with(MF_E_ARG, "options or flightlines is NULL");
  if (opt->struct_size != sizeof(mf_options))
    return fail_with(MF_E_ARG, "mf_options.struct_size mismatch");
  if (opt->n_bands < 2 || opt->n_bands > MF_MAX_BANDS)
    return fail_with(MF_E_UNSUPPORTED, "n_bands must be in [2, 78]");
  if (opt->n_iter < 0) return fail_with(MF_E_ARG, "n_iter must be >= 0");
  if (!(opt->lambda >= 0.0) || !std::isfinite(opt->lambda))
    return fail_with(MF_E_ARG, "lambda must be finite and >= 0");
  if (!(opt->epsilon > 0.0) || !std::isfinite(opt->epsilon))
    return fail_with(MF_E_ARG, "epsilon must be finite and > 0");
  if (opt->albedo != 0 && opt->albedo != 1) return fail_with(MF_E_ARG, "albedo must be 0 or 1");
  if (opt->cov < MF_COV_LOWRANK || opt->cov > MF_COV_GRAM_BF16X3)
    return fail_with(MF_E_ARG, "cov must be one of MF_COV_*");
  if (opt->refine_steps < -1 || opt->refine_steps > 8)
    return fail_with(MF_E_ARG, "refine_steps must be -1 (the form's default) or in [0, 8]");
  if (opt->save_for_backward != 0 && opt->save_for_backward != 1)
    return fail_with(MF_E_ARG, "save_for_backward must be 0 or 1");
  if (opt->save_for_backward && opt->cov != MF_COV_LOWRANK)
    return fail_with(MF_E_UNSUPPORTED, "save_for_backward needs the low-rank covariance form");
  if (opt->save_for_backward && opt->n_iter > kMaxBackwardIter)
    return fail_with(MF_E_UNSUPPORTED,
                     "save_for_backward supports n_iter <= " + std::to_string(kMaxBackwardIter));
  if (opt->chunk_lines < 0 || opt->chunk_lines % 128 != 0)
    return fail_with(MF_E_ARG, "chunk_lines must be a non-negative multiple of 128");
  if (opt->group < 1) return fail_with(MF_E_ARG, "group must be >= 1");
  if (opt->track_energy != 0 && opt->track_energy != 1)
    return fail_with(MF_E_ARG, "track_energy must be 0 or 1");
  if (opt->track_energy && opt->cov != MF_COV_LOWRANK)
    return fail_with(MF_E_UNSUPPORTED, "track_energy needs the low-rank covariance form");
  if (n_fl < 1) return fail_with(MF_E_SHAPE, "need at least one flightline");

  const int chunk = opt->chunk_lines ? opt->chunk_lines
                                     : (opt->cov == MF_COV_LOWRANK ? kDefaultChunkLowrank : kDefaultChunkGram);
  std::vector<ColInfo> cols;
  std::vector<WorkItem> items;
  std::vector<std::pair<int64_t, int64_t>> ranges;
  int64_t n_px = 0, max_px = 0, n_words = 0;
  for (int f = 0; f < n_fl; ++f) {
    const mf_flightline& F = fl[f];
    if (F.n_columns < 1 || F.n_lines < 1 || F.first_px < 0)
      return fail_with(MF_E_SHAPE, "flightline " + std::to_string(f) + " has an empty or negative shape");
    const int64_t np = (int64_t)F.n_columns * F.n_lines;
    ranges.push_back({F.first_px, F.first_px + np});
    n_px += np;
    max_px = std::max(max_px, F.first_px + np);
    // partitions of `group` adjacent columns (the last one takes the remainder)
    const int g = opt->group;
    if ((int64_t)std::min(g, F.n_columns) * F.n_lines > (int64_t)INT32_MAX)
      return fail_with(MF_E_SHAPE, "flightline " + std::to_string(f) + ": a partition exceeds 2^31 pixels");
    for (int c = 0; c < F.n_columns; c += g) {
      const int ncol = std::min(g, F.n_columns - c);
      const int npart = ncol * F.n_lines;
      ColInfo ci{};
      ci.first_px = F.first_px + (int64_t)c * F.n_lines;
      ci.n_px = npart;
      ci.first_item = (int32_t)items.size();
      const int nit = (int)(((int64_t)npart + chunk - 1) / chunk);
      // split evenly, in multiples of 128 pixels
      int per = (int)(((int64_t)npart + nit - 1) / nit);
      per = (per + 127) / 128 * 128;
      int done = 0;
      for (int k = 0; k < nit && done < npart; ++k) {
        WorkItem w{};
        w.px_begin = ci.first_px + done;
        w.word0 = n_words;
        w.col = (int32_t)cols.size();
        w.n_px = std::min(per, npart - done);
        done += w.n_px;
        n_words += (w.n_px + 31) / 32;
        items.push_back(w);
      }
      ci.n_items = (int32_t)items.size() - ci.first_item;
      cols.push_back(ci);
      if (items.size() > (size_t)INT32_MAX) return fail_with(MF_E_SHAPE, "too many work items");
    }
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t i = 1; i < ranges.size(); ++i)
    if (ranges[i].first < ranges[i - 1].second)
      return fail_with(MF_E_SHAPE, "flightline pixel ranges overlap");

  mf_plan_s* p = new (std::nothrow) mf_plan_s();
  if (!p) return fail_with(MF_E_ARG, "out of host memory");
  p->opt = *opt;
  p->nb = (opt->n_bands + 2 + 15) / 16;
  p->wide = opt->n_bands >= 64;
  p->n_cols = (int64_t)cols.size();
  p->n_items = (int64_t)items.size();
  p->n_px = n_px;
  p->max_px = max_px;
  p->n_words = n_words;
  p->cols_h = cols;
  p->grp_col = {0, p->n_cols};
  p->grp_item = {0, p->n_items};
  if (hipGetDevice(&p->device) != hipSuccess ||
      hipMalloc(&p->cols_d, cols.size() * sizeof(ColInfo)) != hipSuccess ||
      hipMalloc(&p->items_d, items.size() * sizeof(WorkItem)) != hipSuccess ||
      hipMemcpy(p->cols_d, cols.data(), cols.size() * sizeof(ColInfo), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->items_d, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice) != hipSuccess) {
    const std::string e = hipGetErrorString(hipGetLastError());
    if (p->cols_d) (void)hipFree(p->cols_d);
    if (p->items_d) (void)hipFree(p->items_d);
    delete p;
    return fail_with(MF_E_DEVICE, "plan tables: " + e);
  }
  {
    // work items longest first, for the persistent launches' queue (ragged
    // batches: the short items fill the tail); ties keep the plan's order
    std::vector<int32_t> order(items.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return items[x].n_px > items[y].n_px; });
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, p->device) != hipSuccess ||
        hipMalloc(&p->order_d, order.size() * sizeof(int32_t)) != hipSuccess ||
        hipMemcpy(p->order_d, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
      const std::string e = hipGetErrorString(hipGetLastError());
      if (p->order_d) (void)hipFree(p->order_d);
      (void)hipFree(p->cols_d);
      (void)hipFree(p->items_d);
      delete p;
      return fail_with(MF_E_DEVICE, "plan tables: " + e);
    }
    p->n_cu = prop.multiProcessorCount;
  }
  {
    std::string err;
    p->scratch_d = scratch_address(p->device, err);
    if (!p->scratch_d) {
      (void)hipFree(p->cols_d);
      (void)hipFree(p->items_d);
      (void)hipFree(p->order_d);
      delete p;
      return fail_with(MF_E_DEVICE, err);
    }
  }
  size_t off = 0;
  p->off_state = off;
  off = align256(off + (size_t)p->n_cols * sizeof(ColState));
  p->off_partials = off;
  off = align256(off + (size_t)p->n_items * (size_t)partial_stride(p) * sizeof(double));
  p->off_c0 = off;
  if (opt->cov != MF_COV_GRAM_FP64) off = align256(off + (size_t)p->n_cols * kNBlk * 16 * sizeof(double));
  p->off_pinv = off;
  if (opt->cov == MF_COV_LOWRANK) off = align256(off + (size_t)p->n_cols * kNBlk * 16 * sizeof(double));
  p->off_alpha0 = off;
  off = align256(off + (size_t)max_px * sizeof(double));
  p->off_alpha1 = off;
  off = align256(off + (size_t)max_px * sizeof(double));
  const size_t mask_words = (size_t)p->n_words + 2;
  p->off_mask0 = off;
  off = align256(off + mask_words * sizeof(uint32_t));
  p->off_mask1 = off;
  off = align256(off + mask_words * sizeof(uint32_t));
  p->off_r = off;                              // r per pixel (written by pass 1)
  off = align256(off + (size_t)max_px * sizeof(double));
  if (opt->save_for_backward) {
    const size_t K1 = (size_t)opt->n_iter + 1;
    p->off_ck_alpha = off;
    off = align256(off + K1 * (size_t)max_px * sizeof(double));
    p->off_ck_mask = off;                    // K + 1 mask arrays of mask_words words
    off = align256(off + K1 * mask_words * sizeof(uint32_t));
    p->off_ck_col = off;
    off = align256(off + K1 * (size_t)p->n_cols * kCk * sizeof(double));
    p->off_ck_p = off;                       // p^0..p^K
    off = align256(off + K1 * (size_t)max_px * sizeof(double));
    p->off_bw_px = off;
    off = align256(off + 3 * (size_t)max_px * sizeof(double));
    p->off_bw_coef = off;
    off = align256(off + 2 * K1 * (size_t)max_px * sizeof(double));
    p->off_bw_u = off;
    off = align256(off + K1 * (size_t)p->n_cols * kPad * sizeof(double));
    p->off_bw_col = off;
    off = align256(off + (size_t)p->n_cols * kBw * sizeof(double));
    if (asm_blocks(opt->n_iter) > 1) {       // FP64 running sum of the gradient assembly
      p->off_bw_acc = off;
      off = align256(off + (size_t)max_px * opt->n_bands * sizeof(double));
    }
  }
  if (opt->track_energy) {
    p->off_energy = off;
    off = align256(off + ((size_t)opt->n_iter + 1) * (size_t)p->n_cols * sizeof(double));
  }
  p->off_queue = off;                          // persistent launches' queue counters
  off = align256(off + (size_t)MF_MAX_STREAMS * ((size_t)opt->n_iter + 2) * sizeof(int));
  p->ws_bytes = off;
  *out = p;
  g_last_error.clear();
  return MF_OK;
}

size_t mf_workspace_bytes(mf_plan p) { return p ? p->ws_bytes : 0; }
int64_t mf_plan_columns(mf_plan p) { return p ? p->n_cols : 0; }
int64_t mf_plan_pixels(mf_plan p) { return p ? p->n_px : 0; }
int32_t mf_plan_refine_steps(mf_plan p) { return p ? refine_steps_of(p->opt) : -1; }

mf_status mf_retrieve(mf_plan p, const float* radiance, const uint8_t* valid, const float* s,
                      float* alpha, int32_t* column_status, void* workspace, void* stream) {
  if (!p) return fail_with(MF_E_ARG, "plan is NULL");
  if (!radiance || !s || !alpha || !workspace)
    return fail_with(MF_E_ARG, "radiance, s, alpha and workspace must be non-NULL");
  if (((uintptr_t)workspace & 255) != 0) return fail_with(MF_E_ARG, "workspace must be 256-byte aligned");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail_with(MF_E_DEVICE, "current device differs from the plan's device");
  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  // Graph replay: the whole launch sequence captured once per set of
  // pointers and stream (not on the legacy default stream, not while timing).
  if (p->use_graph && st != nullptr && !p->timing) {
    const GraphKey key{radiance, valid, s, alpha, column_status, workspace, stream};
    if (!(p->graph_exec && p->graph_key == key)) {
      if (p->graph_exec) {
        (void)hipGraphExecDestroy(p->graph_exec);
        p->graph_exec = nullptr;
      }
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail_with(MF_E_DEVICE, "hipStreamBeginCapture failed");
      enqueue_retrieve(p, radiance, valid, s, alpha, column_status, workspace, st);
      const hipError_t ec = hipStreamEndCapture(st, &g);
      if (ec != hipSuccess || !g) return fail_with(MF_E_DEVICE, std::string("capture: ") + hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        p->graph_exec = nullptr;
        return fail_with(MF_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
      }
      p->graph_key = key;
    }
    const hipError_t e = hipGraphLaunch(p->graph_exec, st);
    if (e != hipSuccess) return fail_with(MF_E_DEVICE, std::string("graph launch: ") + hipGetErrorString(e));
    return MF_OK;
  }
  enqueue_retrieve(p, radiance, valid, s, alpha, column_status, workspace, st);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_with(MF_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
  return MF_OK;
}

mf_status mf_retrieve_noalloc(mf_plan p, const float* radiance, const uint8_t* valid, const float* s,
                              float* alpha, int32_t* column_status, void* stream) {
  if (!p) return fail_with(MF_E_ARG, "plan is NULL");
  if (!radiance || !s || !alpha) return fail_with(MF_E_ARG, "radiance, s and alpha must be non-NULL");
  if (p->ws_bytes > kScratchBytes)
    return fail_with(MF_E_UNSUPPORTED, "the plan needs " + std::to_string(p->ws_bytes) +
                                           " bytes of workspace; mf_retrieve_noalloc has " +
                                           std::to_string(kScratchBytes));
  if (p->opt.save_for_backward || p->opt.track_energy)
    return fail_with(MF_E_UNSUPPORTED,
                     "mf_retrieve_noalloc keeps no state for mf_backward or mf_plan_energy");
  if (p->timing) return fail_with(MF_E_STATE, "kernel timing is on (it records events)");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail_with(MF_E_DEVICE, "current device differs from the plan's device");
  if (!p->scratch_d) return fail_with(MF_E_STATE, "no scratch address for the plan's device");
  (void)hipGetLastError();
  // plain launches (no graph: instantiating one allocates), on the scratch
  enqueue_retrieve(p, radiance, valid, s, alpha, column_status, p->scratch_d, (hipStream_t)stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_with(MF_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
  return MF_OK;
}

mf_status mf_backward(mf_plan p, const float* radiance, const uint8_t* valid, const float* s,
                      const float* grad_alpha, float* grad_radiance, double* grad_s,
                      void* workspace, void* stream) {
  if (!p) return fail_with(MF_E_ARG, "plan is NULL");
  if (!p->opt.save_for_backward)
    return fail_with(MF_E_STATE, "the plan was created without save_for_backward");
  if (!radiance || !s || !grad_alpha || !grad_radiance || !grad_s || !workspace)
    return fail_with(MF_E_ARG, "radiance, s, grad_alpha, grad_radiance, grad_s and workspace must be non-NULL");
  if (((uintptr_t)workspace & 255) != 0) return fail_with(MF_E_ARG, "workspace must be 256-byte aligned");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail_with(MF_E_DEVICE, "current device differs from the plan's device");
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  const int B = p->opt.n_bands, K = p->opt.n_iter;
  const int64_t mp = p->max_px;
  ColState* state = (ColState*)(ws + p->off_state);
  double* partials = (double*)(ws + p->off_partials);
  double* ck_alpha = (double*)(ws + p->off_ck_alpha);
  const uint32_t* ck_mask = (const uint32_t*)(ws + p->off_ck_mask);
  const int64_t mask_words = p->n_words + 2;
  double* ck_col = (double*)(ws + p->off_ck_col);
  double* ck_p = (double*)(ws + p->off_ck_p);
  double* bwpx = (double*)(ws + p->off_bw_px);
  double* coef = (double*)(ws + p->off_bw_coef);
  double* u_hist = (double*)(ws + p->off_bw_u);
  double* bwcol = (double*)(ws + p->off_bw_col);
  const int pstride = (int)partial_stride(p);
  (void)hipGetLastError();
  {
    const int64_t n = p->n_cols * kBw;
    LaunchTimer tm(p, MF_KERNEL_OTHER, st);
    hipLaunchKernelGGL(bwd_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, bwcol, n);
  }
  BwArgs ba{};
  ba.L = radiance;
  ba.n_floats = mp * B;
  ba.valid = valid;
  ba.items = p->items_d;
  ba.state = state;
  ba.grad_alpha = grad_alpha;
  ba.r_px = (double*)(ws + p->off_r);
  ba.abar = bwpx;
  ba.rbar = bwpx + mp;
  ba.pbar = bwpx + 2 * mp;
  ba.bwcol = bwcol;
  ba.partials = partials;
  ba.partial_stride = pstride;
  ba.B = B;
  ba.K = K;
  ba.lam = p->opt.lambda;
  ba.eps = p->opt.epsilon;
  ba.albedo = p->opt.albedo;
  BwColArgs ca{};
  ca.cols = p->cols_d;
  ca.state = state;
  ca.c0 = (double*)(ws + p->off_c0);
  ca.pinv = (double*)(ws + p->off_pinv);
  ca.partials = partials;
  ca.bwcol = bwcol;
  ca.s = s;
  ca.partial_stride = pstride;
  ca.B = B;
  ca.refine = refine_steps_of(p->opt);
  ca.albedo = p->opt.albedo;
  const size_t lds = bwd_lds_bytes<false>(B), ldsF = bwd_lds_bytes<true>(B), ldsA = bwdA_lds_bytes(B);
  // per-iteration pointers of the pass arguments (k = iteration of pass B)
  auto set_iter = [&](int k) {
    ba.k = k;
    ba.ck_k = ck_col + (int64_t)k * p->n_cols * kCk;
    ba.ck_km1 = k >= 1 ? ck_col + (int64_t)(k - 1) * p->n_cols * kCk : nullptr;
    ba.a_k = ck_alpha + (int64_t)k * mp;
    ba.a_km1 = k >= 1 ? ck_alpha + (int64_t)(k - 1) * mp : nullptr;
    ba.a_km2 = k >= 2 ? ck_alpha + (int64_t)(k - 2) * mp : nullptr;
    ba.m_km1 = k >= 1 ? ck_mask + (int64_t)(k - 1) * mask_words : nullptr;
    ba.m_km2 = k >= 2 ? ck_mask + (int64_t)(k - 2) * mask_words : nullptr;
    ba.p_k = ck_p + (int64_t)k * mp;
    ba.p_km1 = k >= 1 ? ck_p + (int64_t)(k - 1) * mp : nullptr;
    ba.coef_v = coef + (int64_t)(2 * k) * mp;
    ba.coef_u = coef + (int64_t)(2 * k + 1) * mp;
    ba.u_k = u_hist + (int64_t)k * p->n_cols * kPad;
  };
  auto set_col = [&](int k, int fused) {
    ca.k = k;
    ca.fused = fused;
    ca.ck_k = ck_col + (int64_t)k * p->n_cols * kCk;
    ca.ck_km1 = k >= 1 ? ck_col + (int64_t)(k - 1) * p->n_cols * kCk : nullptr;
    ca.u_k = u_hist + (int64_t)k * p->n_cols * kPad;
    ca.ck_b = fused ? ck_col + (int64_t)(k + 1) * p->n_cols * kCk : nullptr;
    ca.u_b = fused ? u_hist + (int64_t)(k + 1) * p->n_cols * kPad : nullptr;
  };
  // pass A(K) and its column step, then per iteration k = K..1 one fused pass
  // B(k) + A(k-1) followed by one column kernel (col B(k), then col A(k-1)),
  // then pass B(0) and col B(0); every step for each partition group on its
  // own stream (mf_plan_set_streams), forked after the init kernel
  const int G = p->n_groups;
  hipStream_t gs[MF_MAX_STREAMS];
  gs[0] = st;
  if (G > 1) {
    (void)hipEventRecord(p->fork_ev, st);
    for (int g = 1; g < G; ++g) {
      gs[g] = p->aux[g - 1];
      (void)hipStreamWaitEvent(gs[g], p->fork_ev, 0);
    }
  }
  auto pass = [&](int g, auto kernel, int kind, size_t lds_bytes, int block) {
    ba.item_base = (int)p->grp_item[g];
    const unsigned n = (unsigned)(p->grp_item[g + 1] - p->grp_item[g]);
    LaunchTimer tm(p, kind, gs[g]);
    hipLaunchKernelGGL(kernel, dim3(n), dim3(block), lds_bytes, gs[g], ba);
  };
  auto column = [&](int g, auto kernel, int block) {
    ca.col_base = (int)p->grp_col[g];
    const unsigned n = (unsigned)(p->grp_col[g + 1] - p->grp_col[g]);
    LaunchTimer tm(p, MF_KERNEL_SOLVE, gs[g]);
    hipLaunchKernelGGL(kernel, dim3(n), dim3(block), 0, gs[g], ca);
  };
  set_iter(K);
  set_col(K, 0);
  for (int g = 0; g < G; ++g) {
    pass(g, bwd_passA_kernel, MF_KERNEL_PASS_VEC, ldsA, kABlock);
    column(g, bwd_colA_kernel, kBlock);
  }
  for (int k = K; k >= 1; --k) {
    set_iter(k);
    set_col(k - 1, 1);
    for (int g = 0; g < G; ++g) {
      pass(g, bwd_passB_kernel<true>, MF_KERNEL_PASS_VEC, ldsF, kSBlock);
      column(g, bwd_colA_kernel, kBlock);
    }
  }
  set_iter(0);
  set_col(0, 0);
  for (int g = 0; g < G; ++g) {
    pass(g, bwd_passB_kernel<false>, MF_KERNEL_PASS_VEC, lds, kSBlock);
    column(g, bwd_colB_kernel, 128);
  }
  BwAsmArgs aa{};
  aa.items = p->items_d;
  aa.state = state;
  aa.valid = valid;
  aa.ck = ck_col;
  aa.u_hist = u_hist;
  aa.coef = coef;
  aa.rbar = bwpx + mp;
  aa.bwcol = bwcol;
  aa.grad_L = grad_radiance;
  aa.max_px = mp;
  aa.n_cols = (int)p->n_cols;
  aa.B = B;
  aa.K = K;
  aa.albedo = p->opt.albedo;
  aa.n_blocks = asm_blocks(K);
  aa.acc = aa.n_blocks > 1 ? (double*)(ws + p->off_bw_acc) : nullptr;
  for (int g = 0; g < G; ++g) {
    aa.item_base = (int)p->grp_item[g];
    const unsigned n = (unsigned)(p->grp_item[g + 1] - p->grp_item[g]);
    for (int q = 0; q < aa.n_blocks; ++q) {      // in order on the group's stream
      aa.block = q;
      LaunchTimer tm(p, MF_KERNEL_PASS_LAST, gs[g]);
      const size_t lds = asm_lds_bytes(B, K);
      if (aa.n_blocks == 1)
        hipLaunchKernelGGL(bwd_assemble_kernel<kAsmOnly>, dim3(n), dim3(256), lds, gs[g], aa);
      else if (q == 0)
        hipLaunchKernelGGL(bwd_assemble_kernel<kAsmFirst>, dim3(n), dim3(256), lds, gs[g], aa);
      else if (q + 1 < aa.n_blocks)
        hipLaunchKernelGGL(bwd_assemble_kernel<kAsmMid>, dim3(n), dim3(256), lds, gs[g], aa);
      else
        hipLaunchKernelGGL(bwd_assemble_kernel<kAsmLast>, dim3(n), dim3(256), lds, gs[g], aa);
    }
  }
  if (G > 1)
    for (int g = 1; g < G; ++g) {
      (void)hipEventRecord(p->join_ev[g - 1], gs[g]);
      (void)hipStreamWaitEvent(st, p->join_ev[g - 1], 0);
    }
  {
    LaunchTimer tm(p, MF_KERNEL_OTHER, st);
    hipLaunchKernelGGL(bwd_sbar_kernel, dim3((unsigned)B), dim3(256), 0, st, state, bwcol,
                       (int)p->n_cols, grad_s);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_with(MF_E_DEVICE, std::string("backward launch: ") + hipGetErrorString(e));
  return MF_OK;
}

mf_status mf_plan_set_graph(mf_plan p, int enable) {
  if (!p) return fail_with(MF_E_ARG, "plan is NULL");
  p->use_graph = enable != 0;
  return MF_OK;
}

mf_status mf_repack_bil(const float* bil, int64_t n_lines, int32_t n_bands, int32_t n_samples,
                        float* radiance, uint8_t* valid, int64_t first_px, int32_t use_nodata,
                        float nodata, void* stream) {
  if (!bil || !radiance) return fail_with(MF_E_ARG, "bil or radiance is NULL");
  if (n_lines < 1 || n_samples < 1 || first_px < 0)
    return fail_with(MF_E_SHAPE, "n_lines and n_samples must be >= 1, first_px >= 0");
  if (n_bands < 1 || n_bands > MF_MAX_BANDS)
    return fail_with(MF_E_UNSUPPORTED, "n_bands must be in [1, 78]");
  if (use_nodata != 0 && use_nodata != 1) return fail_with(MF_E_ARG, "use_nodata must be 0 or 1");
  const int64_t ly = (n_lines + kRpL - 1) / kRpL;
  const int64_t sy = (n_samples + kRpS - 1) / kRpS;
  if (ly > INT32_MAX || sy > 65535) return fail_with(MF_E_SHAPE, "cube too large for one call");
  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  const size_t lds = (size_t)kRpL * n_bands * kRpRow * sizeof(float);
  const dim3 grid((unsigned)ly, (unsigned)sy);
  hipLaunchKernelGGL(repack_bil_kernel, grid, dim3(256), lds, st, bil, n_lines, (int)n_bands,
                     (int)n_samples, radiance, valid, first_px, (int)use_nodata, nodata);
  if (hipGetLastError() != hipSuccess) return fail_with(MF_E_DEVICE, "repack launch failed");
  return MF_OK;
}

mf_status mf_stream_read(const float* src, int64_t n, float* sink, int32_t n_blocks,
                         float* ms_out, void* stream) {
  if (!src || !sink || n < 4 || n % 4 != 0 || ((uintptr_t)src & 15) != 0 || n_blocks < 1)
    return fail_with(MF_E_ARG, "src/sink NULL, n not a positive multiple of 4, or src not 16-byte aligned");
  // a contiguous span per workgroup; its byte offsets (plus the unrolled
  // loads' stride) stay below 2^31
  int64_t per = (n + n_blocks - 1) / n_blocks;
  per = (per + 3) / 4 * 4;
  if (per * 4 > (int64_t)INT32_MAX - 65536)
    return fail_with(MF_E_ARG, "n / n_blocks exceeds 2^29 floats per workgroup");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms_out && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    return fail_with(MF_E_DEVICE, "event creation failed");
  if (ms_out) (void)hipEventRecord(e0, st);
  hipLaunchKernelGGL(stream_read_kernel, dim3((unsigned)n_blocks), dim3(kBlock), 0, st, src, n, per, sink);
  mf_status rc = MF_OK;
  if (hipGetLastError() != hipSuccess) rc = fail_with(MF_E_DEVICE, "stream_read launch failed");
  if (ms_out) {
    float ms = 0.f;
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      rc = fail_with(MF_E_DEVICE, "event timing failed");
    *ms_out = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return rc;
}

mf_status mf_plan_set_launch(mf_plan p, int32_t stream_tile, int32_t wgs_per_cu) {
  if (!p) return fail_with(MF_E_ARG, "plan is NULL");
  if (stream_tile < MF_TILE_32x4 || stream_tile > MF_TILE_64x1)
    return fail_with(MF_E_ARG, "stream_tile must be one of MF_TILE_*");
  if (wgs_per_cu < 0 || wgs_per_cu > 16) return fail_with(MF_E_ARG, "wgs_per_cu must be in [0, 16]");
  if (p->stream_tile != stream_tile || p->wgs_per_cu != wgs_per_cu) {
    p->stream_tile = stream_tile;
    p->wgs_per_cu = wgs_per_cu;
    if (p->graph_exec) {                       // the captured launches no longer apply
      (void)hipGraphExecDestroy(p->graph_exec);
      p->graph_exec = nullptr;
    }
  }
  return MF_OK;
}

mf_status mf_plan_set_streams(mf_plan p, int32_t n_streams) {
  if (!p) return fail_with(MF_E_ARG, "plan is NULL");
  if (n_streams < 1 || n_streams > MF_MAX_STREAMS)
    return fail_with(MF_E_ARG, "n_streams must be in [1, " + std::to_string(MF_MAX_STREAMS) + "]");
  if (n_streams > p->n_cols) return fail_with(MF_E_ARG, "n_streams exceeds the plan's partitions");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
    return fail_with(MF_E_DEVICE, "current device differs from the plan's device");
  if (n_streams > 1 && !p->fork_ev &&
      hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming) != hipSuccess)
    return fail_with(MF_E_DEVICE, "event creation failed");
  for (int g = 1; g < n_streams; ++g) {
    // default priority (streams of other priorities are not used here)
    if (!p->aux[g - 1] && hipStreamCreateWithFlags(&p->aux[g - 1], hipStreamNonBlocking) != hipSuccess)
      return fail_with(MF_E_DEVICE, "stream creation failed");
    if (!p->join_ev[g - 1] && hipEventCreateWithFlags(&p->join_ev[g - 1], hipEventDisableTiming) != hipSuccess)
      return fail_with(MF_E_DEVICE, "event creation failed");
  }
  // contiguous partition ranges of about equal pixel counts, each non-empty
  std::vector<int64_t> gc(n_streams + 1, 0), gi(n_streams + 1, 0);
  int64_t total = 0;
  for (const ColInfo& c : p->cols_h) total += c.n_px;
  int64_t acc = 0, c = 0;
  for (int g = 1; g < n_streams; ++g) {
    const int64_t target = total * g / n_streams;
    while (c < p->n_cols - (n_streams - g) && (c < gc[g - 1] + 1 || acc + p->cols_h[c].n_px <= target))
      acc += p->cols_h[c++].n_px;
    gc[g] = c;
  }
  gc[n_streams] = p->n_cols;
  for (int g = 0; g < n_streams; ++g) gi[g] = p->cols_h[gc[g]].first_item;
  gi[n_streams] = p->n_items;
  if (n_streams != p->n_groups || gc != p->grp_col) {
    p->n_groups = n_streams;
    p->grp_col = gc;
    p->grp_item = gi;
    if (p->graph_exec) {                       // the captured launches no longer apply
      (void)hipGraphExecDestroy(p->graph_exec);
      p->graph_exec = nullptr;
    }
  }
  return MF_OK;
}

int32_t mf_plan_streams(mf_plan p) { return p ? p->n_groups : 0; }

mf_status mf_plan_set_timing(mf_plan p, int enable) {
  if (!p) return fail_with(MF_E_ARG, "plan is NULL");
  p->timing = enable != 0;
  return MF_OK;
}

mf_status mf_plan_energy(mf_plan p, const void* workspace, double* energy_out, void* stream) {
  if (!p || !workspace || !energy_out) return fail_with(MF_E_ARG, "plan, workspace or energy_out is NULL");
  if (!p->opt.track_energy) return fail_with(MF_E_STATE, "the plan was created without track_energy");
  const size_t bytes = ((size_t)p->opt.n_iter + 1) * (size_t)p->n_cols * sizeof(double);
  if (hipMemcpyAsync(energy_out, (const char*)workspace + p->off_energy, bytes, hipMemcpyDeviceToDevice,
                     (hipStream_t)stream) != hipSuccess)
    return fail_with(MF_E_DEVICE, std::string("energy copy: ") + hipGetErrorString(hipGetLastError()));
  return MF_OK;
}

mf_status mf_plan_kernel_times(mf_plan p, double* times_ms, int64_t* counts, int n) {
  if (!p) return fail_with(MF_E_ARG, "plan is NULL");
  if (n < 0 || n > MF_KERNEL_KINDS) return fail_with(MF_E_ARG, "n out of range");
  double t[MF_KERNEL_KINDS] = {};
  int64_t c[MF_KERNEL_KINDS] = {};
  mf_status rc = MF_OK;
  for (const TimedLaunch& l : p->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(l.stop) != hipSuccess ||
        hipEventElapsedTime(&ms, l.start, l.stop) != hipSuccess)
      rc = fail_with(MF_E_DEVICE, "event timing failed");
    t[l.kind] += ms;
    c[l.kind] += 1;
    p->event_pool.push_back(l.start);
    p->event_pool.push_back(l.stop);
  }
  p->pending.clear();
  for (int k = 0; k < n; ++k) {
    if (times_ms) times_ms[k] = t[k];
    if (counts) counts[k] = c[k];
  }
  return rc;
}

void mf_plan_destroy(mf_plan p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  for (const TimedLaunch& l : p->pending) {
    (void)hipEventDestroy(l.start);
    (void)hipEventDestroy(l.stop);
  }
  for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  for (int g = 0; g < MF_MAX_STREAMS - 1; ++g) {
    if (p->aux[g]) (void)hipStreamDestroy(p->aux[g]);
    if (p->join_ev[g]) (void)hipEventDestroy(p->join_ev[g]);
  }
  if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
  if (p->cols_d) (void)hipFree(p->cols_d);
  if (p->items_d) (void)hipFree(p->items_d);
  if (p->order_d) (void)hipFree(p->order_d);
  delete p;
}

}  // extern "C"

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
//  * per-iteration Gram (GRAM_FP64 / GRAM_FP32 / GRAM_BF16).  With d_i the
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

constexpr int kBlock = 256;      // 4 waves of 64
constexpr int kPad = 80;         // bands of the per-column state (5 x 16)
constexpr int kMaxTri = 80 * 81 / 2;
// Default work-item lengths (lines): the low-rank form's partials are 82
// doubles per item, so short items balance the streaming passes best; the
// Gram forms combine a 30 KB partial Gram per item in every solve, so they
// prefer long items.
constexpr int kDefaultChunkLowrank = 1024;
constexpr int kDefaultChunkGram = 4096;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// What a pass accumulates besides alpha.
enum PassMode {
  PM_NONE = 0,   // last pass: alpha only
  PM_VEC = 1,    // m = sum c (L - mean L), S1, S2 in FP64 (low-rank form)
  PM_F64 = 2,    // Gram of [y, 1, c] on v_mfma_f64_16x16x4_f64 (exact)
  PM_F32 = 3,    // Gram on v_mfma_f32_16x16x4_f32, FP32 accumulation per wave
  PM_BF16 = 4    // Gram on v_mfma_f32_16x16x32_bf16, FP32 accumulation per wave
};
constexpr int kVecS1 = 80, kVecS2 = 81;   // PM_VEC partial layout: m in [0, B)
// FP32 / BF16 Gram passes: after the T tiles of the item's partial Gram, the
// exact FP64 moments sum c L (bands [0, 80)), sum c, sum c^2.
constexpr int kXS1 = 80, kXS2 = 81, kXMom = 82;
constexpr int kXMomSlots = 128;            // doubles reserved per item for them
constexpr int kVecE = 82;      // energy: pixel part of E^{j-1} (both streaming modes)

// One partition (Sec. II-E): `group` adjacent detector columns of a
// flightline, contiguous in memory, solved as one problem.
struct ColInfo {
  int64_t first_px;
  int32_t n_px;              // pixels of the partition
  int32_t first_item;
  int32_t n_items;
  int32_t pad;
};

struct WorkItem {
  int64_t px_begin;
  int32_t col;
  int32_t n_px;
};

// Per-column state, written by the solve kernel and read by the next pass.
struct alignas(16) ColState {
  double mu[kPad];     // mu^j, subtracted by the next pass (shift z before pass 0)
  double t[kPad];      // t^j = mu^j (.) s
  double v[kPad];      // v^j = C^j^-1 t^j
  double m0[kPad];     // mu^0 / |mu^0|^2, the albedo projection of Eq. 7
  double lbar[kPad];   // plain mean mu^0
  double q;            // t^T C^-1 t
  double n_valid;      // N, from pass 0
  int32_t status;
  int32_t pad[3];
};

struct PassArgs {
  const float* L;
  const uint8_t* valid;
  const WorkItem* items;
  const ColState* state;
  const double* alpha_prev;  // alpha^{j-2} (j >= 2), FP64 workspace copy
  double* alpha_out;         // alpha^{j-1} (1 <= j <= K), FP64 workspace copy
  float* alpha_final;        // alpha^K (j = K + 1), the caller's FP32 output
  double* partials;          // [item][T][16][16] FP64
  double* p_save;            // save_for_backward: p^{j-1} = (L - mu) . v per pixel (j >= 1)
  int64_t n_floats;          // floats of the radiance array (max_px * B)
  int track_energy;          // accumulate the pixel part of E^{j-1} (partial slot kVecE)
  double* r_out;             // r per pixel written by this pass (j = 1)
  const double* r_in;        // r per pixel from pass 1, or null: computed here
  int B;
  int j;
  int albedo;
  int unclamped;             // K == 0: return alpha^0 without the clamp
  double lam;
  double eps;
  int partial_stride;        // doubles per work item in the partial buffer
  // persistent launch: the workgroups take work items from this pass's
  // counter (zeroed by setup_kernel) in the order of `order`; null: one
  // workgroup per work item (blockIdx.x)
  int* queue;
  const int32_t* order;
  int n_items;
};

struct SolveArgs {
  const ColInfo* cols;
  ColState* state;
  const double* partials;
  double* c0;                // LOWRANK: C^0 per column, register-block layout
  double* pinv;              // LOWRANK: (C^0)^-1 per column, same layout
  const float* s;
  int B;
  int j;
  int refine;
  int lowrank;
  int exact_ref;             // FP32 / BF16 Gram forms: refine against the exact C^j
                             // (C^0 + rank-3 update) and keep C^0 from pass 0
  int partial_stride;        // doubles per work item in the partial buffer
  double* ck;                // save_for_backward: column checkpoints [K+1][n_cols][kCk]
  double* energy;            // track_energy: E^k per partition [K+1][n_cols], or null
  int n_cols;
};

__host__ __device__ constexpr int n_tiles(int nb) { return nb * (nb + 1) / 2; }
// Block row I of lower-triangle tile u = n_tiles(I) + J, J <= I.
__host__ __device__ constexpr int tile_row(int u) {
  int I = 0;
  while (n_tiles(I + 1) <= u) ++I;
  return I;
}
__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }  // j <= i

// ---------------------------------------------------------------------------
// setup: per column, the shift point z (first valid pixel) and a clean state.

__global__ void __launch_bounds__(64) setup_kernel(const float* __restrict__ L,
                                                   const uint8_t* __restrict__ valid,
                                                   const ColInfo* __restrict__ cols,
                                                   ColState* __restrict__ state, int B,
                                                   double* __restrict__ energy, int K1,
                                                   int64_t n_cols, int* __restrict__ queue,
                                                   int n_queue) {
  const int col = blockIdx.x;
  const int lane = threadIdx.x;
  if (queue && col == 0)   // the passes' work-queue counters (persistent launches)
    for (int k = lane; k < n_queue; k += 64) queue[k] = 0;
  const ColInfo ci = cols[col];
  int64_t z = -1;
  if (valid == nullptr) {
    z = ci.n_px > 0 ? ci.first_px : -1;
  } else {
    for (int64_t l0 = 0; l0 < ci.n_px; l0 += 64) {
      const bool v = (l0 + lane < ci.n_px) && valid[ci.first_px + l0 + lane] != 0;
      const unsigned long long m = __ballot(v);
      if (m) {
        z = ci.first_px + l0 + (__ffsll(m) - 1);
        break;
      }
    }
  }
  ColState& st = state[col];
  for (int b = lane; b < kPad; b += 64) {
    st.mu[b] = (z >= 0 && b < B) ? (double)L[z * B + b] : 0.0;
    st.t[b] = 0.0;
    st.v[b] = 0.0;
    st.m0[b] = 0.0;
    st.lbar[b] = 0.0;
  }
  if (lane == 0) {
    st.q = 1.0;
    st.n_valid = 0.0;
    st.status = z >= 0 ? MF_COL_OK : MF_COL_FEW_PIXELS;
  }
  if (energy)              // E^k stays NaN for a partition that fails before iteration k
    for (int k = lane; k < K1; k += 64) energy[(int64_t)k * n_cols + col] = __builtin_nan("");
}

// ---------------------------------------------------------------------------
// pass: one streaming pass over a work item (a run of pixels of one column).
//
// Wave layout: a wave handles 4 pixels per sub-step, one per 16-lane row.
// The lane in column c of the row holds NB "register blocks" of that pixel;
// block k, lane c holds band band_of<NB, WIDE>(k, c).  Narrow layout: band
// c + 16k.  Wide layout (B >= 64): bands 4c..4c+3 in blocks 0..3 (one 16-byte
// load) and band 64 + c in block 4 (one 4-byte load).  Either way the
// registers of block I are, per 4 pixels, the A operand (A[m][k] from lane
// m + 16k) and the B operand of a 16x16x4 MFMA, so the Gram of block I
// against block J is one MFMA per 4 pixels; the solve undoes the band
// permutation.  Eight sub-steps make a 32-pixel super-step; packed to BF16
// the same registers are the operands of the 16x16x32 BF16 MFMA with pixel
// 4s+g of the super-step in k = 8g+s.
//
// Per-pixel arithmetic (scores, albedo factor, alpha, moments) is FP64: near
// the sparsity threshold the reweighting map alpha <- z - w has a derivative
// far above 1 and amplifies any rounding, and FP64 costs the same VALU rate
// as unpacked FP32 on CDNA.  The Gram inputs y of the FP32 and BF16 forms are
// formed in FP32, the precision they are rounded to.

// Loads through a buffer resource that covers [p, p + bytes): offsets at or
// past the end read zeros (raw buffer range check), so a partial last group
// or a null pointer (bytes = 0) needs neither a branch nor a select.
constexpr int kBufWord3 = 0x00020000;
constexpr int kOffNone = 0x7ffffff0;       // an offset past every resource
// Cache policy of the streaming loads: non-temporal.  Every pass reads the
// radiance (and the per-pixel vectors) exactly once, and the hint lets the
// loads stream past the caches: a plain contiguous read of a flightline runs
// at about 6.1 TB/s with it off and 7.0 TB/s with it on.
constexpr int kLoadNT = 2;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t chunk_rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, kBufWord3);
}
__device__ __forceinline__ float4 load16(__amdgpu_buffer_rsrc_t rs, int off) {
  typedef int intx4 __attribute__((ext_vector_type(4)));
  const intx4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, kLoadNT);
  return float4{__int_as_float(v.x), __int_as_float(v.y), __int_as_float(v.z), __int_as_float(v.w)};
}
__device__ __forceinline__ float load4(__amdgpu_buffer_rsrc_t rs, int off) {
  return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, kLoadNT));
}
__device__ __forceinline__ double load8(__amdgpu_buffer_rsrc_t rs, int off) {
  typedef int intx2 __attribute__((ext_vector_type(2)));
  const intx2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, kLoadNT);
  return __hiloint2double(v.y, v.x);
}
template <typename T>
__device__ __forceinline__ T ntl(const T* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ uint32_t load1(__amdgpu_buffer_rsrc_t rs, int off) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, off, 0, kLoadNT);
}

template <int NB, bool WIDE>
__host__ __device__ constexpr int band_of(int k, int c) {
  return WIDE ? (k < 4 ? 4 * c + k : 64 + c) : c + 16 * k;
}

// Blocks that can hold band B or B + 1, the 1 and c columns of the Gram
// (NB is the smallest block count with B + 2 <= 16 NB): the last two blocks
// of the narrow layout, block 4 of the wide one.
template <int NB, bool WIDE>
__host__ __device__ constexpr bool holds_tail(int k) {
  return WIDE ? k == 4 : k >= NB - 2;
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double row_sum16_f64(double x) {
  x += dpp_f64<0xB1>(x);
  x += dpp_f64<0x4E>(x);
  x += dpp_f64<0x124>(x);
  x += dpp_f64<0x128>(x);
  return x;
}

// Issues the loads of one super-step (the 32 pixels from base, pixel 4s + row
// in sub-step s) through buffer resources sized to the pixels that exist:
// rows past the work item's end, and alpha / valid when their pointer is
// null, read zeros.  No load is conditional, so the next super-step's loads
// stay in flight while the current one is computed.  Lane l (mod 32) holds
// alpha^{j-2} and the valid flag of pixel base + l.
template <int NB, bool WIDE>
__device__ __forceinline__ void load_super(const PassArgs& a, int64_t base, int64_t end, int lane,
                                           int row, int c16, float (&Lv)[8][NB], double& ap,
                                           uint32_t& vb, double& rp) {
  const int B = a.B;
  const int n = (int)max<int64_t>(0, min<int64_t>(32, end - base));
  const __amdgpu_buffer_rsrc_t ra = chunk_rsrc(a.alpha_prev ? a.alpha_prev + base : nullptr,
                                               a.alpha_prev ? n * 8 : 0);
  const __amdgpu_buffer_rsrc_t rr = chunk_rsrc(a.r_in ? a.r_in + base : nullptr, a.r_in ? n * 8 : 0);
  const __amdgpu_buffer_rsrc_t rv = chunk_rsrc(a.valid ? a.valid + base : nullptr, a.valid ? n : 0);
  // one resource per sub-step (its 4 rows, or fewer at the item's end), so
  // the lane offsets are the same in every sub-step and every range check is
  // on the offset itself
  const int o4 = (row * B + 4 * c16) * 4;
  const int o1 = 64 + c16 < B ? (row * B + 64 + c16) * 4 : kOffNone;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int rows = __builtin_amdgcn_readfirstlane(max(0, min(4, n - 4 * s)));   // wave-uniform
    const __amdgpu_buffer_rsrc_t rl = chunk_rsrc(a.L + (base + 4 * s) * B, rows * B * 4);
    if constexpr (WIDE) {        // bands 4c..4c+3 < 64 <= B never straddle a row
      const float4 v4 = load16(rl, o4);
      Lv[s][0] = v4.x;
      Lv[s][1] = v4.y;
      Lv[s][2] = v4.z;
      Lv[s][3] = v4.w;
      Lv[s][4] = load4(rl, o1);
    } else {
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const int b = band_of<NB, WIDE>(k, c16);
        Lv[s][k] = load4(rl, b < B ? (row * B + b) * 4 : kOffNone);
      }
    }
  }
  ap = load8(ra, (lane & 31) * 8);
  vb = load1(rv, lane & 31);
  rp = load8(rr, (lane & 31) * 8);
}

// SCORE: passes j >= 1 (alpha^{j-1} and c = r alpha enter the Gram); pass 0
// (SCORE = false) is the Gram of the shifted radiance alone.
// RIN: the albedo factor r of each pixel comes from the buffer pass 1 wrote
// (a.r_in), so the score needs only L . v; otherwise r = L . m0 is formed
// here (pass 1 also writes it when a.r_out is set).
template <int NB, bool WIDE, int MODE, bool SCORE, bool RIN>
__device__ __forceinline__ void pass_item(const PassArgs& a, int item) {
  constexpr int T = n_tiles(NB);
  static_assert(MODE >= PM_F64, "the Gram pass; the streaming passes are stream_kernel");
  constexpr bool F32ACC = MODE == PM_F32 || MODE == PM_BF16;
  // FP32 and BF16 Gram: FP32 accumulation over the wave's share of the item,
  // FP64 only across waves and items.  The rounded Gram only preconditions
  // the solve, which refines against the exact C^j (see solve_kernel), so
  // its accumulation error sets the refinement's rate, not the result.
  // The rounded forms also accumulate, exactly in FP64, the moments of the
  // rank-3 identity for C^j: sum c L (per band), sum c and sum c^2.
  constexpr bool XMOM = SCORE && F32ACC;
  const WorkItem it = a.items[item];
  const ColState& st = a.state[it.col];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  const int row = lane >> 4, c16 = lane & 15;
  const int B = a.B;
  const int64_t begin = it.px_begin, end = begin + it.n_px;

  if (st.status != MF_COL_OK) {          // failed column: alpha = 0, no moments
    for (int64_t px = begin + tid; px < end; px += kBlock) {
      if (a.alpha_out) a.alpha_out[px] = 0.0;
      if (a.alpha_final) a.alpha_final[px] = 0.f;
    }
    return;
  }

  [[maybe_unused]] double mu[NB], vv[NB], tt[NB], m0[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int b = band_of<NB, WIDE>(k, c16);
    const bool in = b < B;
    mu[k] = in ? st.mu[b] : 0.0;
    if constexpr (SCORE) {
      vv[k] = in ? st.v[b] : 0.0;
      tt[k] = in ? st.t[b] : 0.0;
      m0[k] = in ? st.m0[b] : 0.0;
    }
  }
  [[maybe_unused]] double muv = 0.0;            // mu . v, the same in every row
  if constexpr (SCORE) {
    double d = 0.0;
#pragma unroll
    for (int k = 0; k < NB; ++k) d = fma(mu[k], vv[k], d);
    muv = row_sum16_f64(d);
  }
  [[maybe_unused]] float muf[NB], ttf[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    muf[k] = (float)mu[k];
    if constexpr (SCORE) ttf[k] = (float)tt[k];
  }
  const double q = st.q;
  const double lam = a.lam, eps = a.eps;
  const int j = a.j;

  [[maybe_unused]] floatx4 acc[F32ACC ? T : 1];
  // XMOM: the wave's sums of c L per band, sum c and sum c^2, in LDS (only
  // super-steps with a nonzero c add to them, so no register holds them)
  __shared__ double xred[XMOM ? 4 : 1][kXMom];
  if constexpr (XMOM) {
    for (int e = lane; e < kXMom; e += 64) xred[wid][e] = 0.0;
  }
  doublex4 dacc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) dacc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
  if constexpr (F32ACC) {
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  }

  // The Gram passes run one or two waves per SIMD: the next super-step's
  // loads are in flight while the current one is computed, and are waited
  // for only when they are moved into place after it.
  auto compute = [&](const float (&Lc)[8][NB], double apl, uint32_t vbl, double rpl, int64_t bx) {
    [[maybe_unused]] bf16x8 ybf[NB];
    // SCORE: c = r alpha^{j-1} of pixel 4s + row of the super-step, or -1
    // for a pixel that stays out of the Gram (invalid, or past the item)
    [[maybe_unused]] double cs[8];
    if constexpr (SCORE) {
      // The lane's partial dot products for its row's 8 pixels:
      // L . v in v16[s] (p = L . v - mu . v), r = m0 . L in v16[8 + s]
      // (bands past B hold zeros in L, v and m0).
      // Transpose reduction over the 16 lanes of each row: at each step a
      // lane keeps half of its values, sends the other half to its partner
      // (partners differ in one bit of the lane's column) and adds what it
      // receives.  With 16 values (L . v and L . m0 of the row's 8 pixels)
      // lane c of the row ends with the row total of value c; with the 8 of
      // L . v alone, lanes 2s and 2s + 1 end with that of value s.
      double v8[8], v4[4], v2[2];
      if constexpr (!RIN) {
        double v16[16];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          double pe = 0.0, re = 0.0;
#pragma unroll
          for (int k = 0; k < NB; ++k) {
            const double l = (double)Lc[s][k];
            pe = fma(l, vv[k], pe);
            re = fma(l, m0[k], re);
          }
          v16[s] = pe;
          v16[8 + s] = re;
        }
        const bool hi = (c16 & 8) != 0;        // row_mirror: c <-> 15 - c
#pragma unroll
        for (int i = 0; i < 8; ++i)
          v8[i] = (hi ? v16[i + 8] : v16[i]) + dpp_f64<0x140>(hi ? v16[i] : v16[i + 8]);
      } else {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          double pe = 0.0;
#pragma unroll
          for (int k = 0; k < NB; ++k) pe = fma((double)Lc[s][k], vv[k], pe);
          v8[s] = pe;
        }
      }
      constexpr int kMirror = RIN ? 0x140 : 0x141;   // first 8-value step: row_mirror
      {
        const bool hi = (c16 & (RIN ? 8 : 4)) != 0;  // then row_half_mirror
#pragma unroll
        for (int i = 0; i < 4; ++i)
          v4[i] = (hi ? v8[i + 4] : v8[i]) + dpp_f64<kMirror>(hi ? v8[i] : v8[i + 4]);
      }
      {
        constexpr int kStep = RIN ? 0x141 : 0x4E;   // row_half_mirror, or c <-> c ^ 2
        const bool hi = (c16 & (RIN ? 4 : 2)) != 0;
#pragma unroll
        for (int i = 0; i < 2; ++i)
          v2[i] = (hi ? v4[i + 2] : v4[i]) + dpp_f64<kStep>(hi ? v4[i] : v4[i + 2]);
      }
      double v1;
      {
        constexpr int kStep = RIN ? 0x4E : 0xB1;    // c <-> c ^ 2, or c <-> c ^ 1
        const bool hi1 = (c16 & (RIN ? 2 : 1)) != 0;
        v1 = (hi1 ? v2[1] : v2[0]) + dpp_f64<kStep>(hi1 ? v2[0] : v2[1]);
        if constexpr (RIN) v1 += dpp_f64<0xB1>(v1);   // c <-> c ^ 1: the full row total
      }
      // One pixel per lane from here: lane l (and l + 32) holds pixel
      // qx = l mod 32 of the super-step, sub-step qx / 4, row qx mod 4.
      const int qx = lane & 31;
      const double pp = __shfl(v1, 16 * (qx & 3) + (RIN ? 2 : 1) * (qx >> 2), 64) - muv;
      const double rr = RIN ? rpl : __shfl(v1, 16 * (qx & 3) + 8 + (qx >> 2), 64);
      const int64_t px = bx + qx;
      const bool ok = px < end && (a.valid == nullptr || vbl != 0u);
      const double r = a.albedo ? rr : 1.0;
      const double num = (j == 1) ? pp : pp - lam / (apl + eps);
      double al = num / (r * q);
      const bool dark = !(r > 0.0);
      if (!a.unclamped) al = al > 0.0 ? al : 0.0;
      if (!ok || dark) al = 0.0;
      if (lane < 32 && px < end) {
        if (a.alpha_out) a.alpha_out[px] = al;
        if (a.alpha_final) a.alpha_final[px] = (float)al;
        if constexpr (!RIN) {
          if (a.r_out) a.r_out[px] = ok ? r : 0.0;
        }
      }
      const double cenc = ok ? ((!dark && al > 0.0) ? r * al : 0.0) : -1.0;
#pragma unroll
      for (int s = 0; s < 8; ++s) cs[s] = __shfl(cenc, 4 * s + row, 64);
      if constexpr (XMOM) {
        // only where some pixel of the super-step has c > 0 (the enhancement
        // is sparse); the test is wave-uniform
        if (__ballot(cenc > 0.0) != 0ull) {
          double c1 = (lane < 32 && cenc > 0.0) ? cenc : 0.0;
          double c2 = c1 * c1;
          for (int off = 32; off >= 1; off >>= 1) {
            c1 += __shfl_xor(c1, off, 64);
            c2 += __shfl_xor(c2, off, 64);
          }
          // one band block at a time into LDS, so that no register holds a
          // running sum across the pass (the rows hold the same bands of
          // different pixels)
#pragma unroll
          for (int k = 0; k < NB; ++k) {
            double x = 0.0;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
              // a fresh value: the FP64 conversions of the scores above are
              // not kept alive for this rarely taken branch
              float l = Lc[s][k];
              asm volatile("" : "+v"(l));
              x = cs[s] > 0.0 ? fma(cs[s], (double)l, x) : x;   // invalid rows may hold NaN
            }
            x += __shfl_xor(x, 16, 64);
            x += __shfl_xor(x, 32, 64);
            if (lane < 16) xred[wid][band_of<NB, WIDE>(k, c16)] += x;
          }
          if (lane == 0) {
            xred[wid][kXS1] += c1;
            xred[wid][kXS2] += c2;
          }
        }
      }
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      bool ok;
      double c = 0.0;
      if constexpr (SCORE) {
        ok = cs[s] >= 0.0;
        c = ok ? cs[s] : 0.0;
      } else {
        const int64_t px = bx + 4 * s + row;
        const uint32_t vb = (uint32_t)__shfl((int)vbl, 4 * s + row, 64);
        ok = px < end && (a.valid == nullptr || vb != 0u);
      }
      // y = L - mu - c t (Eq. 11), then the 1 and c columns past band B;
      // bands past B + 1 hold zeros in L, mu and t
      if constexpr (MODE == PM_F64) {
        double y[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const int b = band_of<NB, WIDE>(k, c16);
          const double x = (double)Lc[s][k] - mu[k];
          y[k] = ok ? (SCORE ? fma(-c, tt[k], x) : x) : 0.0;
          if (holds_tail<NB, WIDE>(k) && b == B) y[k] = ok ? 1.0 : 0.0;
          if (holds_tail<NB, WIDE>(k) && b == B + 1) y[k] = c;
        }
#pragma unroll
        for (int I = 0; I < NB; ++I)
#pragma unroll
          for (int J = 0; J <= I; ++J)
            dacc[n_tiles(I) + J] =
                __builtin_amdgcn_mfma_f64_16x16x4f64(y[I], y[J], dacc[n_tiles(I) + J], 0, 0, 0);
      } else {
        // FP32 and BF16 Gram: y is formed in FP32 (it is rounded to the
        // Gram's input precision anyway; mu and t enter rounded to FP32)
        const float cf = (float)c;
        float yf[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const int b = band_of<NB, WIDE>(k, c16);
          const float x = Lc[s][k] - muf[k];
          yf[k] = ok ? (SCORE ? fmaf(-cf, ttf[k], x) : x) : 0.f;
          if (holds_tail<NB, WIDE>(k) && b == B) yf[k] = ok ? 1.f : 0.f;
          if (holds_tail<NB, WIDE>(k) && b == B + 1) yf[k] = cf;
        }
        if constexpr (MODE == PM_F32) {
#pragma unroll
          for (int I = 0; I < NB; ++I)
#pragma unroll
            for (int J = 0; J <= I; ++J)
              acc[n_tiles(I) + J] =
                  __builtin_amdgcn_mfma_f32_16x16x4f32(yf[I], yf[J], acc[n_tiles(I) + J], 0, 0, 0);
        } else {
#pragma unroll
          for (int k = 0; k < NB; ++k) ybf[k][s] = (__bf16)yf[k];
        }
      }
    }
    if constexpr (MODE == PM_BF16) {
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J)
          acc[n_tiles(I) + J] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(ybf[I], ybf[J], acc[n_tiles(I) + J], 0, 0, 0);
    }
  };

  int64_t base = begin + 32 * wid;
  if (base < end) {
    float LA[8][NB], LB[8][NB];
    double apA, apB, rA, rB;
    uint32_t vA, vB;
    load_super<NB, WIDE>(a, base, end, lane, row, c16, LA, apA, vA, rA);
    auto super_step = [&](int64_t bx) {
      load_super<NB, WIDE>(a, bx + 128, end, lane, row, c16, LB, apB, vB, rB);
      compute(LA, apA, vA, rA, bx);
      __builtin_amdgcn_sched_barrier(0);   // the copy below waits for the loads
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int k = 0; k < NB; ++k) LA[s][k] = LB[s][k];
      apA = apB;
      vA = vB;
      rA = rB;
    };
    for (; base < end; base += 128) super_step(base);
  }

  double* out = a.partials + (int64_t)item * a.partial_stride;
  if constexpr (XMOM) {
    // the exact moments: the waves' sums in order
    __syncthreads();
    if (tid < kXMom) out[T * 256 + tid] = ((xred[0][tid] + xred[1][tid]) + xred[2][tid]) + xred[3][tid];
  }
  if constexpr (F32ACC) {
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) dacc[t][i] += (double)acc[t][i];
  }
  // Deterministic cross-wave reduction in LDS, wave 0 first.
  __shared__ double red[T * 256];
  for (int w = 0; w < 4; ++w) {
    if (wid == w) {
#pragma unroll
      for (int t = 0; t < T; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          // Where D[m][n] of a tile lives: f32 MFMA lane n + 16 (m / 4),
          // register m % 4; f64 MFMA lane n + 16 (m % 4), register m / 4.
          const int m = MODE == PM_F64 ? row + 4 * i : 4 * row + i;
          const int e = t * 256 + m * 16 + c16;
          red[e] = (w == 0 ? 0.0 : red[e]) + dacc[t][i];
        }
    }
    __syncthreads();
  }
  for (int e = tid; e < T * 256; e += kBlock) out[e] = red[e];
}

// ---------------------------------------------------------------------------
// stream pass (no Gram): alpha only (PM_NONE) or alpha plus the vector moments
// of the low-rank form (PM_VEC).  One pixel per lane: each wave copies a
// 64-pixel chunk of its work item into its own LDS tile with fully coalesced
// loads (the next chunk is in flight while the current one is scored), then
// every lane scores its own pixel from LDS with the column's constants as
// wave-uniform scalar operands.  m = sum c (L - mean L) is accumulated
// band-per-lane from the same tile, and skipped when the chunk has no
// nonzero c (the enhancement is sparse).

constexpr int kChunk = 32;                 // pixels per wave chunk (adjoint streaming pass)
constexpr int kSW = 4;                     // waves per workgroup (adjoint streaming pass)
constexpr int kSBlock = 64 * kSW;
constexpr int kCopyGroup = 10;             // 16-byte loads in flight per lane while copying

// Tile shape of the forward streaming pass: CHUNK pixels per wave chunk (32:
// lanes l and l + 32 share pixel l, each running half of its bands; 64: one
// pixel per lane) and SW waves per workgroup.
template <int CHUNK, int SW>
struct StreamTile {
  static_assert(CHUNK == 32 || CHUNK == 64, "32 or 64 pixels per wave chunk");
  static_assert(SW >= 1 && SW <= 4, "1 to 4 waves per workgroup");
  static constexpr int kThreads = 64 * SW;
  static constexpr int kGroups = (CHUNK * 80 / 4 + 63) / 64;   // 16-byte loads per lane per chunk
  static constexpr int kTileFloats = kGroups * 64 * 4;         // floats per wave tile
  static constexpr bool kSplit = CHUNK == 32;
  // dynamic LDS bytes: c per pixel, moment partials, column constants, tiles
  static constexpr size_t kLds = (size_t)SW * CHUNK * sizeof(double) + SW * (kPad + 3) * sizeof(double) +
                                 4 * kPad * sizeof(double) + (size_t)SW * kTileFloats * sizeof(float);
  static_assert(kLds + 16 <= 64 * 1024, "within the default dynamic LDS of a workgroup");
};

// Synchronous copy of one chunk (contiguous in memory) into a wave's LDS tile.
__device__ __forceinline__ void copy_chunk(const float* g, int nfl, float* my, int lane) {
  const uintptr_t ga = reinterpret_cast<uintptr_t>(g);
  if ((ga & 15) == 0 && (nfl & 3) == 0) {
    const float4* g4 = reinterpret_cast<const float4*>(g);
    float4* t4 = reinterpret_cast<float4*>(my);
    const int n4 = nfl / 4;
    for (int base = 0; base < n4; base += 64 * kCopyGroup) {
      float4 r[kCopyGroup];
#pragma unroll
      for (int q = 0; q < kCopyGroup; ++q) {
        const int e = base + lane + 64 * q;
        r[q] = e < n4 ? g4[e] : float4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int q = 0; q < kCopyGroup; ++q) {
        const int e = base + lane + 64 * q;
        if (e < n4) t4[e] = r[q];
      }
    }
  } else if ((ga & 7) == 0 && (nfl & 1) == 0) {
    const float2* g2 = reinterpret_cast<const float2*>(g);
    float2* t2 = reinterpret_cast<float2*>(my);
    const int n2 = nfl / 2;
    for (int e = lane; e < n2; e += 64) t2[e] = g2[e];
  } else {
    for (int e = lane; e < nfl; e += 64) my[e] = g[e];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wave's radiance tile (adjoint pass): kF4 16-byte groups per lane (a whole
// chunk of up to 80 bands), so the fast path writes it without bounds tests.
constexpr int kF4 = (kChunk * 80 / 4 + 63) / 64;     // 10
constexpr int kTileF = kF4 * 64 * 4;                  // floats per wave tile

// Wave-uniform copies (scalar registers) of values every lane loaded alike.
__device__ __forceinline__ int uni32(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uni64(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double unif64(double x) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x)),
                          __builtin_amdgcn_readfirstlane(__double2loint(x)));
}

// One work item of the forward streaming pass.  The work item and the
// column's scalars are read once and made wave-uniform: in the persistent
// loop the compiler cannot prove them unchanged by earlier stores, so it
// would keep them as vector loads and wait for every load in flight (the
// next chunk's prefetch included) where the score first uses them.
template <int MODE, int CHUNK, int SW>
__device__ __forceinline__ void stream_item(const PassArgs& a, int item, double* dyn) {
  using T = StreamTile<CHUNK, SW>;
  constexpr int kChunk = CHUNK, kSW = SW, kSBlock = T::kThreads, kF4 = T::kGroups, kTileF = T::kTileFloats;
  WorkItem it;
  {
    const WorkItem w = a.items[item];
    it.px_begin = uni64(w.px_begin);
    it.col = uni32(w.col);
    it.n_px = uni32(w.n_px);
  }
  const ColState* __restrict__ st = a.state + it.col;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  const int B = a.B;
  const int64_t begin = it.px_begin, end = begin + it.n_px;
  double* cbuf = dyn;                                   // [kSW][kChunk]
  double* redm = cbuf + kSW * kChunk;                   // [kSW][kPad + 3]
  double* cst = redm + kSW * (kPad + 3);                // [kPad] v, m0, lbar; mu . v
  float* my = reinterpret_cast<float*>(cst + 4 * kPad) + wid * kTileF;   // [kChunk][B]

  const int64_t step = (int64_t)kSW * kChunk;
  int64_t c0 = begin + (int64_t)kChunk * wid;
  // A chunk is loaded from the 16-byte boundary at or below its first float,
  // so its tile starts `shift` floats into the LDS buffer; shift is the same
  // for every chunk of this wave (a chunk step is a multiple of 4 floats).
  // The loaded span, rounded out to 16 bytes, must lie inside the radiance
  // array: true for every chunk but possibly the first and last ones of the
  // array, which are copied synchronously.
  const int shift = (int)((reinterpret_cast<uintptr_t>(a.L + c0 * B) & 15) >> 2);
  const int n4 = (shift + kChunk * B + 3) / 4;        // 16-byte groups per chunk span
  auto span_ok = [&](int64_t c) {
    return c * B - shift >= 0 && (c * B - shift) + 4 * (int64_t)n4 <= a.n_floats;
  };
  const float* tile = my + shift;

  // The first chunk is requested before the column state: its loads do not
  // depend on it, and the two latencies overlap.
  float4 pre[kF4];
  uint32_t vld_n = 1;
  double ap_n = 0.0, rp_n = 0.0;
  const bool fast = c0 < end && span_ok(c0);
  // lane l and l + 32 load pixel l of the chunk (only lanes < kChunk score),
  // so no load reaches past the chunk
  const int pl = lane & (kChunk - 1);
  if (fast) {
    vld_n = a.valid ? (uint32_t)ntl(a.valid + c0 + pl) : 1u;
    ap_n = a.alpha_prev ? ntl(a.alpha_prev + c0 + pl) : 0.0;
    rp_n = a.r_in ? ntl(a.r_in + c0 + pl) : 0.0;
    const __amdgpu_buffer_rsrc_t rs = chunk_rsrc(a.L + (c0 * B - shift), n4 * 16);
#pragma unroll
    for (int k = 0; k < kF4; ++k) pre[k] = load16(rs, (lane + 64 * k) * 16);
  }

  if (uni32(st->status) != MF_COL_OK) {    // failed column: alpha = 0, no moments
    for (int64_t px = begin + tid; px < end; px += kSBlock) {
      if (a.alpha_out) a.alpha_out[px] = 0.0;
      if (a.alpha_final) a.alpha_final[px] = 0.f;
    }
    return;
  }
  const double q = unif64(st->q);
  for (int b = tid; b < kPad; b += kSBlock) {
    cst[b] = st->v[b];
    cst[kPad + b] = st->m0[b];
    cst[2 * kPad + b] = st->lbar[b];
  }
  if (wid == 0) {          // mu . v (fixed summation order); p = L . v - mu . v
    double d = 0.0;
    if (lane < B) d = st->mu[lane] * st->v[lane];
    if (lane + 64 < B) d = fma(st->mu[lane + 64], st->v[lane + 64], d);
    for (int off = 32; off >= 1; off >>= 1) d += __shfl_xor(d, off, 64);
    if (lane == 0) cst[3 * kPad] = d;
  }
  __syncthreads();
  const double muv = unif64(cst[3 * kPad]);
  const double lam = a.lam, eps = a.eps;
  const int j = a.j;

  [[maybe_unused]] double m_lo = 0.0, m_hi = 0.0, s1 = 0.0, s2 = 0.0;
  double se = 0.0;                       // pixel part of E^{j-1} (R14)

  // Scores the chunk at c0 (n pixels, tile in LDS): alpha^{j-1}, and for the
  // low-rank form the moment contributions of the pixels with c != 0.
  // r = L . m0 does not change between iterations: the low-rank form computes
  // it in pass 1 and later passes read it (r_in), so their band loop reads
  // only v.  p = L . v - mu . v, with even and odd bands on two FMA chains.
  const bool own_r = a.r_in == nullptr;
  // Lanes l and l + 32 share pixel l of the chunk: the lower lane runs the
  // bands [0, h), the upper one [h, B), and the two partial dot products are
  // added across the halves; every later step of the score is the lower
  // lane's (the upper lanes hold the same values and store nothing).
  const int hsplit = T::kSplit ? ((B + 3) / 4) * 2 : B;   // even, so both halves start on a pair
  const int upper = T::kSplit ? lane >> 5 : 0;
  auto score = [&](int64_t c0, int n, uint32_t vld, double ap, double rp, const float* tl) {
    const int pxl = lane & (kChunk - 1);
    const int64_t px = c0 + pxl;
    const bool inb = pxl < n;
    const bool ok = inb && vld != 0;
    double pe = 0.0, po = 0.0, re = 0.0, ro = 0.0;
    if (ok) {
      const float* rowp = tl + pxl * B;
      const double2* v2 = reinterpret_cast<const double2*>(cst);
      const double2* m2 = reinterpret_cast<const double2*>(cst + kPad);
      int b = upper ? hsplit : 0;
      const int bend = upper ? B : hsplit;
      // pairs of bands need 8-byte aligned rows (B even, tile 8-byte aligned)
      const bool pairs = (B & 1) == 0 && (reinterpret_cast<uintptr_t>(tl) & 7) == 0;
      if (own_r) {
        if (pairs) {                          // 8-byte tile reads
#pragma unroll 4
          for (; b + 1 < bend; b += 2) {
            const float2 l2 = *reinterpret_cast<const float2*>(rowp + b);
            const double2 cv = v2[b >> 1], cm = m2[b >> 1];
            const double l0 = (double)l2.x, l1 = (double)l2.y;
            pe = fma(l0, cv.x, pe);
            re = fma(l0, cm.x, re);
            po = fma(l1, cv.y, po);
            ro = fma(l1, cm.y, ro);
          }
        }
        for (; b < bend; ++b) {
          const double l = (double)rowp[b];
          pe = fma(l, cst[b], pe);
          re = fma(l, cst[kPad + b], re);
        }
      } else {
        if (pairs) {
          double2 cv = v2[b >> 1];
#pragma unroll 4
          for (; b + 1 < bend; b += 2) {
            const double2 nv = v2[(b >> 1) + 1];   // next pair, in flight (kPad > B)
            const float2 l2 = *reinterpret_cast<const float2*>(rowp + b);
            pe = fma((double)l2.x, cv.x, pe);
            po = fma((double)l2.y, cv.y, po);
            cv = nv;
          }
        }
        for (; b < bend; ++b) pe = fma((double)rowp[b], cst[b], pe);
      }
    }
    double pp = pe + po, rr = re + ro;
    if constexpr (T::kSplit) {
      pp += __shfl_xor(pp, 32, 64);             // both halves of the pixel's bands
      if (own_r) rr += __shfl_xor(rr, 32, 64);
    }
    pp -= muv;
    double c = 0.0;
    if (j >= 1) {
      const double r = own_r ? (a.albedo ? rr : 1.0) : rp;
      const double num = (j == 1) ? pp : pp - lam / (ap + eps);
      double al = num / (r * q);
      const bool dark = !(r > 0.0);
      if (!a.unclamped) al = al > 0.0 ? al : 0.0;
      if (!ok || dark) al = 0.0;
      if (inb && !upper) {
        if (a.alpha_out) a.alpha_out[px] = al;
        if (a.alpha_final) a.alpha_final[px] = (float)al;
        if (a.p_save) a.p_save[px] = ok ? pp : 0.0;
        if (a.r_out) a.r_out[px] = ok ? r : 0.0;
      }
      c = (ok && !dark && al > 0.0 && !upper) ? r * al : 0.0;
      if (a.track_energy && ok && !dark && !upper) {
        // -r a p + 1/2 r^2 a^2 q + r w a, with w^0 = 0
        const double w = (j == 1) ? 0.0 : lam / (ap + eps);
        se += r * al * (0.5 * r * al * q - pp + w);
      }
    }
    if constexpr (MODE == PM_VEC) {
      s1 += c;
      s2 = fma(c, c, s2);
      if (__ballot(c != 0.0)) {                 // wave-uniform
        if (lane < kChunk) cbuf[wid * kChunk + lane] = c;
        wave_sync_lds();
        const int b0 = lane, b1 = lane + 64;
        const double lb0 = b0 < B ? cst[2 * kPad + b0] : 0.0;
        const double lb1 = b1 < B ? cst[2 * kPad + b1] : 0.0;
        for (int p = 0; p < n; ++p) {
          const double cp = cbuf[wid * kChunk + p];
          if (cp != 0.0) {                      // wave-uniform; skips invalid pixels too
            if (b0 < B) m_lo = fma(cp, (double)tl[p * B + b0] - lb0, m_lo);
            if (b1 < B) m_hi = fma(cp, (double)tl[p * B + b1] - lb1, m_hi);
          }
        }
      }
    }
    // the tile is rewritten by this wave only after every lane is done with it
    wave_sync_lds();
  };

  // Fast path: each chunk (a ragged last one of the item too) is loaded one
  // chunk ahead, 16 bytes per load, into registers.  Lanes past the item's
  // end load pixels of the next column, which stay unused (the span check
  // keeps every such read inside the arrays).  The loads of a chunk's
  // per-pixel inputs (valid flag, alpha^{j-2}, r) are issued before its tile:
  // vector loads retire in order, so waiting for them never waits for the
  // tile in flight.  When there is no next chunk the resource covers 16 bytes
  // of the current chunk, so the loop body has no branch around a load.
  if (fast) {
    while (true) {
      const int n = (int)min<int64_t>(kChunk, end - c0);
      const uint32_t vld = vld_n;
      const double ap = ap_n, rp = rp_n;
      float4* t4 = reinterpret_cast<float4*>(my);
#pragma unroll
      for (int k = 0; k < kF4; ++k) t4[lane + 64 * k] = pre[k];
      wave_sync_lds();
      const int64_t nx = c0 + step;
      const bool more = nx < end && span_ok(nx);
      {                                       // in flight while this chunk is scored
        const int64_t cn = more ? nx : c0;
        const int64_t pn = cn + (more ? pl : 0);
        vld_n = a.valid ? (uint32_t)ntl(a.valid + pn) : 1u;
        ap_n = a.alpha_prev ? ntl(a.alpha_prev + pn) : 0.0;
        rp_n = a.r_in ? ntl(a.r_in + pn) : 0.0;
        const __amdgpu_buffer_rsrc_t rs = chunk_rsrc(a.L + (cn * B - shift), more ? n4 * 16 : 16);
#pragma unroll
        for (int k = 0; k < kF4; ++k) pre[k] = load16(rs, (lane + 64 * k) * 16);
      }
      score(c0, n, vld, ap, rp, tile);
      c0 = nx;
      if (!more) break;
    }
  }
  // the rest (the last chunk of the array, when its span would pass the end):
  // synchronous copies
  for (; c0 < end; c0 += step) {
    const int n = (int)min<int64_t>(kChunk, end - c0);
    const int64_t px = c0 + pl;
    const bool inb = pl < n;
    const uint32_t vld = (inb && a.valid) ? (uint32_t)a.valid[px] : 1u;
    const double ap = (inb && a.alpha_prev) ? a.alpha_prev[px] : 0.0;
    const double rp = (inb && a.r_in) ? a.r_in[px] : 0.0;
    copy_chunk(a.L + c0 * B, n * B, my, lane);
    score(c0, n, vld, ap, rp, my);
  }

  if (a.track_energy)
    for (int off = 32; off >= 1; off >>= 1) se += __shfl_xor(se, off, 64);
  if constexpr (MODE == PM_VEC) {
    for (int off = 32; off >= 1; off >>= 1) {
      s1 += __shfl_xor(s1, off, 64);
      s2 += __shfl_xor(s2, off, 64);
    }
    double* rw = redm + wid * (kPad + 3);
    if (lane < kPad) rw[lane] = lane < B ? m_lo : 0.0;
    if (lane + 64 < kPad) rw[lane + 64] = lane + 64 < B ? m_hi : 0.0;
    if (lane == 0) {
      rw[kVecS1] = s1;
      rw[kVecS2] = s2;
      rw[kVecE] = se;
    }
    __syncthreads();
    double* out = a.partials + (int64_t)item * a.partial_stride;
    for (int e = tid; e < kPad + 3; e += kSBlock) {
      double sum = 0.0;
      for (int w = 0; w < kSW; ++w) sum += redm[w * (kPad + 3) + e];
      out[e] = sum;
    }
  } else {
    if (a.track_energy) {                // last pass: only the energy slot
      if (lane == 0) redm[wid] = se;
      __syncthreads();
      if (tid == 0) {
        double sum = 0.0;
        for (int w = 0; w < kSW; ++w) sum += redm[w];
        a.partials[(int64_t)item * a.partial_stride + kVecE] = sum;
      }
    }
  }
}

// Work items of a persistent pass come from the pass's queue counter:
// thread 0 takes a ticket, the workgroup reads it through LDS, and every
// workgroup stops once the counter passes the item count, so the grid
// drains without waiting on another workgroup.  The ticket for the next
// item is requested when an item starts and read when it ends, so the
// atomic's latency overlaps the item's work.  Tickets map to items through
// `order` (longest first) and are marked wave-uniform (readfirstlane), so
// the work item, column state and buffer resources derived from them stay in
// scalar registers.
__device__ __forceinline__ int share_ticket(int mine, int* slot) {
  if (threadIdx.x == 0) *slot = mine;
  __syncthreads();
  const int t = __builtin_amdgcn_readfirstlane(*slot);
  __syncthreads();                       // every thread has read it before it is reused
  return t;
}
__device__ __forceinline__ int ticket_item(const PassArgs& a, int t) {
  return a.order ? __builtin_amdgcn_readfirstlane(a.order[t]) : t;
}

// PERSIST: a persistent grid taking work items from the pass's queue; else
// one workgroup per work item (blockIdx.x).
// The dynamic LDS holds everything (the ticket slot after the tiles): a
// static LDS variable would move the dynamic buffer off the 16-byte alignment
// that the tiles' 16-byte stores and the constants' paired reads need.
template <int MODE, int CHUNK, int SW, bool PERSIST>
__global__ void __launch_bounds__(64 * SW) stream_kernel(PassArgs a) {
  extern __shared__ __align__(16) double dyn[];
  if constexpr (!PERSIST) {
    stream_item<MODE, CHUNK, SW>(a, (int)blockIdx.x, dyn);
  } else {
    int* slot = reinterpret_cast<int*>(reinterpret_cast<char*>(dyn) + StreamTile<CHUNK, SW>::kLds);
    int t = share_ticket(threadIdx.x == 0 ? atomicAdd(a.queue, 1) : 0, slot);
    while (t < a.n_items) {
      const int next = threadIdx.x == 0 ? atomicAdd(a.queue, 1) : 0;   // read after the item
      stream_item<MODE, CHUNK, SW>(a, ticket_item(a, t), dyn);
      t = share_ticket(next, slot);
    }
  }
}

// The Gram passes run one workgroup per work item (their registers leave
// no room for the persistent loop).
template <int NB, bool WIDE, int MODE, bool SCORE, bool RIN>
__global__ void __launch_bounds__(kBlock, (MODE == PM_F64 && SCORE) ? 1 : 2) pass_kernel(PassArgs a) {
  pass_item<NB, WIDE, MODE, SCORE, RIN>(a, (int)blockIdx.x);
}

// ---------------------------------------------------------------------------
// solve: per column, FP64 combine of the partial Grams, the covariance of
// Eq. 11 (or the sample covariance for j = 0), Cholesky, v = C^-1 t with
// iterative refinement, q = t^T v.

// Register block and lane column holding band b (inverse of band_of).
template <int NB, bool WIDE>
__device__ __forceinline__ void block_of(int b, int& blk, int& m) {
  if (WIDE) {
    blk = b < 64 ? (b & 3) : 4;
    m = b < 64 ? (b >> 2) : b - 64;
  } else {
    blk = b >> 4;
    m = b & 15;
  }
}


// One workgroup per column.  The symmetric matrix is split in 4x4 blocks of
// the lower triangle; thread t < 210 keeps block (bi, bj), t = bi(bi+1)/2 + bj,
// in registers through assembly and a right-looking Cholesky (two barriers
// per column of the factor).
constexpr int kBlk = 4;
constexpr int kNBlkRows = kPad / kBlk;                            // 20
constexpr int kNBlk = kNBlkRows * (kNBlkRows + 1) / 2;            // 210
// Per-column C^0 and P = (C^0)^-1 in HBM: 16 doubles per 4x4 block, stored
// element-major (element e of every block contiguous), so the owner threads
// of a workgroup read and write them with coalesced accesses.
__device__ __forceinline__ int blk_at(int blk, int x, int y) { return (x * kBlk + y) * kNBlk + blk; }

// Dot product of two LDS vectors (length B) on one wave; every lane gets it.
__device__ __forceinline__ double wave_dot(const double* x, const double* y, int B, int lane) {
  double s = 0.0;
  for (int i = lane; i < B; i += 64) s += x[i] * y[i];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

// R x C dot products d[r * C + c] = x_r . y_c of LDS vectors (x_r at x + r
// kPad, y_c at y + c kPad, length B) on one wave, every lane getting all of
// them; the same order of additions as wave_dot, with one butterfly for all.
template <int R, int C>
__device__ __forceinline__ void wave_dots(const double* x, const double* y, int B, int lane,
                                          double (&d)[R * C]) {
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < C; ++c) {
      double s = 0.0;
      for (int i = lane; i < B; i += 64) s += x[r * kPad + i] * y[c * kPad + i];
      d[r * C + c] = s;
    }
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int e = 0; e < R * C; ++e) d[e] += __shfl_xor(d[e], off, 64);
}

// Block of the lower triangle owned by thread t (t = bi(bi+1)/2 + bj).
__device__ __forceinline__ void block_coords(int t, int& bi, int& bj) {
  bi = 0;
  while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
  bj = t - bi * (bi + 1) / 2;
}

// y_r = M b_r (r < R) for a symmetric M held as lower 4x4 register blocks:
// block (bi, bj) of thread t < kNBlk holds M[i][jj] for jj <= i; entries of
// diagonal blocks above the diagonal and rows or columns >= B are zero, and
// so are b_r[i >= B].  Vectors are LDS arrays of stride kPad.  q is LDS
// scratch of R * kPad * kNBlkRows doubles: q[r][i][k] is the product of row i
// with block k of b_r (from block (i/4, k) for k <= i/4, from the transpose of
// block (k, i/4) above it), so every slot is written once and row i is the
// sum of its kNBlkRows contiguous partials in a fixed order (deterministic).
// Contains two barriers.
constexpr int kSymvScratch = kPad * kNBlkRows;
template <int R>
__device__ void block_symv(const double (&M)[kBlk][kBlk], bool owner, int bi, int bj, int tid,
                           int B, const double* bv, double* yv, double* q) {
  if (owner) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double* b = bv + r * kPad;
      double* qr = q + r * kSymvScratch;
      if (bi == bj) {                 // diagonal block: the full symmetric product
#pragma unroll
        for (int x = 0; x < kBlk; ++x) {
          double s = 0.0;
#pragma unroll
          for (int y = 0; y < kBlk; ++y) s += (x >= y ? M[x][y] : M[y][x]) * b[kBlk * bj + y];
          qr[(kBlk * bi + x) * kNBlkRows + bi] = s;
        }
      } else {
#pragma unroll
        for (int x = 0; x < kBlk; ++x) {
          double s = 0.0;
#pragma unroll
          for (int y = 0; y < kBlk; ++y) s += M[x][y] * b[kBlk * bj + y];
          qr[(kBlk * bi + x) * kNBlkRows + bj] = s;
        }
#pragma unroll
        for (int y = 0; y < kBlk; ++y) {
          double s = 0.0;
#pragma unroll
          for (int x = 0; x < kBlk; ++x) s += M[x][y] * b[kBlk * bi + x];
          qr[(kBlk * bj + y) * kNBlkRows + bi] = s;
        }
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < R * kPad; idx += kBlock) {
    const int r = idx / kPad, i = idx - r * kPad;
    const double2* p2 = reinterpret_cast<const double2*>(q + r * kSymvScratch + i * kNBlkRows);
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k < kNBlkRows / 2; ++k) {
      const double2 v = p2[k];
      s0 += v.x;
      s1 += v.y;
    }
    yv[r * kPad + i] = i < B ? s0 + s1 : 0.0;
  }
  __syncthreads();
}

// v = X^T X x = C^-1 x with the inverse Cholesky factor X = L^-1 in the
// owner threads' register blocks (X_ij, i >= j; diagonal blocks lower
// triangular; blocks of row blocks >= nkb unused): y = X x, then v = X^T y.
// Each product writes one partial per (row, block) slot of q ([kPad][kNBlkRows]
// doubles) and sums each row's slots in a fixed order (deterministic).  x must
// be zero beyond B; y is scratch; v gets zeros beyond B.  Four barriers.
__device__ void block_inv_solve(const double (&X)[kBlk][kBlk], bool owner, int bi, int bj, int tid,
                                int B, int nkb, const double* x, double* y, double* v, double* q) {
  const bool use = owner && bi < nkb;
  if (use) {                                       // y_i += X_ij x_j into slot j of row i
#pragma unroll
    for (int r = 0; r < kBlk; ++r) {
      double t = 0.0;
#pragma unroll
      for (int c = 0; c < kBlk; ++c) t = fma(X[r][c], x[kBlk * bj + c], t);
      q[(kBlk * bi + r) * kNBlkRows + bj] = t;
    }
  }
  __syncthreads();
  for (int e = tid; e < kPad; e += kBlock) {
    const int rb = e / kBlk;
    double t = 0.0;
    if (e < B)
      for (int k = 0; k <= rb; ++k) t += q[e * kNBlkRows + k];
    y[e] = t;
  }
  __syncthreads();
  if (use) {                                       // v_j += X_ij^T y_i into slot i of row j
#pragma unroll
    for (int c = 0; c < kBlk; ++c) {
      double t = 0.0;
#pragma unroll
      for (int r = 0; r < kBlk; ++r) t = fma(X[r][c], y[kBlk * bi + r], t);
      q[(kBlk * bj + c) * kNBlkRows + bi] = t;
    }
  }
  __syncthreads();
  for (int e = tid; e < kPad; e += kBlock) {
    const int cb = e / kBlk;
    double t = 0.0;
    if (e < B)
      for (int k = cb; k < nkb; ++k) t += q[e * kNBlkRows + k];
    v[e] = t;
  }
  __syncthreads();
}

// Cholesky factor L (lower) of a symmetric 4x4 block D (row-major, lower part
// read) and W = L^-1 (lower); only the lower triangles of L and W are set.
// False if a pivot is not positive (or not finite).
// 1 / sqrt(d) for a normal d > 0: the hardware estimate refined by two
// Newton-Raphson steps y <- y + y (1 - d y^2) / 2, each of which doubles the
// number of correct bits (the pivot chain of a 4x4 factor is ~8 dependent
// operations per column instead of a square root and a division).
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

template <typename Get>
__device__ __forceinline__ bool chol4g(Get D, double (&Lc)[kBlk][kBlk], double (&W)[kBlk][kBlk]) {
  bool spd = true;
  double rl[kBlk];                             // 1 / L_cc
#pragma unroll
  for (int c = 0; c < kBlk; ++c) {
    double d = D(c, c);
#pragma unroll
    for (int z = 0; z < c; ++z) d = fma(-Lc[c][z], Lc[c][z], d);
    spd = spd && d > 0.0 && isfinite(d);
    rl[c] = rsqrt_nr(d);
    Lc[c][c] = d * rl[c];
#pragma unroll
    for (int r = c + 1; r < kBlk; ++r) {
      double e = D(r, c);
#pragma unroll
      for (int z = 0; z < c; ++z) e = fma(-Lc[r][z], Lc[c][z], e);
      Lc[r][c] = e * rl[c];
    }
  }
#pragma unroll
  for (int c = 0; c < kBlk; ++c) {
    W[c][c] = rl[c];
#pragma unroll
    for (int r = c + 1; r < kBlk; ++r) {
      double e = 0.0;
#pragma unroll
      for (int z = c; z < r; ++z) e = fma(Lc[r][z], W[z][c], e);
      W[r][c] = -e * rl[r];
    }
  }
  return spd;
}
__device__ __forceinline__ bool chol4(const double* D, double (&Lc)[kBlk][kBlk], double (&W)[kBlk][kBlk]) {
  return chol4g([&](int r, int c) { return D[r * 4 + c]; }, Lc, W);
}

// Y = C W^T for a 4x4 block C (row-major) and lower W.
__device__ __forceinline__ void mul_wt(const double* C, const double (&W)[kBlk][kBlk], double (&Y)[kBlk][kBlk]) {
#pragma unroll
  for (int x = 0; x < kBlk; ++x) {
    double c[kBlk];
#pragma unroll
    for (int z = 0; z < kBlk; ++z) c[z] = C[x * 4 + z];
#pragma unroll
    for (int y = 0; y < kBlk; ++y) {
      double t = 0.0;
#pragma unroll
      for (int z = 0; z <= y; ++z) t = fma(c[z], W[y][z], t);
      Y[x][y] = t;
    }
  }
}

// The 4x4 register block of thread tid (< kNBlk) of a per-column matrix
// stored element-major (C^0 or P).  Every thread loads (threads past the
// owners read block 0 and never use it), so the 16 loads issue back to back.
__device__ __forceinline__ void load_block(const double* m, bool owner, int tid, double (&Mb)[kBlk][kBlk]) {
  const int blk = owner ? tid : 0;
#pragma unroll
  for (int x = 0; x < kBlk; ++x)
#pragma unroll
    for (int y = 0; y < kBlk; ++y) Mb[x][y] = m[blk_at(blk, x, y)];
}

// S of the rank-3 identity:  N C^j = N C^0 + N a^2 D D^T + (S2 - N a^2) t t^T - (m t^T + t m^T)
// for U = [D, t, m].
__device__ void rank3_S(double* S3, double abar, double S2, double N) {
  S3[0] = abar * abar; S3[1] = 0.0;                     S3[2] = 0.0;
  S3[3] = 0.0;         S3[4] = S2 / N - abar * abar;    S3[5] = -1.0 / N;
  S3[6] = 0.0;         S3[7] = -1.0 / N;                S3[8] = 0.0;
}

// Column checkpoint of iteration k (save_for_backward): mu, t, v, m, a, S2, q, N.
constexpr int kCkMu = 0, kCkT = kPad, kCkV = 2 * kPad, kCkM = 3 * kPad, kCkScal = 4 * kPad;
constexpr int kCk = 4 * kPad + 8;

template <int NB, bool WIDE>
__global__ void __launch_bounds__(kBlock, 3) solve_kernel(SolveArgs a) {
  const int col = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  ColState& st = a.state[col];
  if (st.status != MF_COL_OK) return;
  const ColInfo ci = a.cols[col];
  const int B = a.B;
  const int j = a.j;
  constexpr int T = n_tiles(NB);
  const int64_t pstride = a.partial_stride;
  const double* P = a.partials + (int64_t)ci.first_item * pstride;
  const bool xref = a.exact_ref && j >= 1;
  double* c0 = a.c0 + (int64_t)col * (kNBlk * 16);
  double* pinv = a.pinv + (int64_t)col * (kNBlk * 16);

  __shared__ double Lf[kMaxTri];     // the column's Gram, then pivot-block buffers
  __shared__ double g1[kPad], g2[kPad], D[kPad], E[kPad], tn[kPad], mun[kPad];
  __shared__ double colk[kPad], vbuf[kPad], rbuf[kPad], dvec[kPad];
  double* wbuf = Lf + 2 * kNBlkRows * 16;   // Gram forms: L_KK^-1 of every pivot block
  __shared__ __align__(16) double qsym[kSymvScratch];
  __shared__ double sc[4];
  __shared__ int fail;
  // exact refinement (rounded forms): U = [t^{j-1} - t^j, t^j, m] and S of the
  // rank-3 identity, sum c L and sum c, sum c^2 of the pass (FP64)
  __shared__ double U3[3 * kPad];
  __shared__ double xmom[kXMom];
  __shared__ double S3[9], zb[4];

  // block owned by this thread
  int bi = 0, bj = 0;
  const bool owner = tid < kNBlk;
  if (owner) block_coords(tid, bi, bj);

  // The column's Gram of [y, 1, c], summed over its work items into LDS as
  // a packed lower triangle (Lf is free until the factor is stored).  Thread
  // t sums element t of every tile, so all of its loads of an item are in
  // flight together; items are added in order, as before.
  {
    static_assert(kBlock == 256, "one tile element per thread");
    double g[T];
#pragma unroll
    for (int u = 0; u < T; ++u) g[u] = 0.0;
    for (int it = 0; it < ci.n_items; ++it) {
      const double* Pi = P + (int64_t)it * pstride + tid;
#pragma unroll
      for (int u = 0; u < T; ++u) g[u] += Pi[256 * u];
    }
    const int mi = tid >> 4, mj = tid & 15;
#pragma unroll
    for (int u = 0; u < T; ++u) {
      const int I = tile_row(u), J = u - n_tiles(I);
      const int bi = band_of<NB, WIDE>(I, mi), bj = band_of<NB, WIDE>(J, mj);
      // off-diagonal tiles hold each band pair once; diagonal tiles twice
      if (bi < B + 2 && bj < B + 2 && (I != J || bi >= bj))
        Lf[bi >= bj ? tri(bi, bj) : tri(bj, bi)] = g[u];
    }
  }
  if (xref) {
    // the exact moments of the column, items in order
    for (int e = tid; e < kXMom; e += kBlock) {
      double acc = 0.0;
      for (int it = 0; it < ci.n_items; ++it) acc += P[(int64_t)it * pstride + T * 256 + e];
      xmom[e] = acc;
    }
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  if (tid == 0) {
    sc[0] = Lf[tri(B, B)];                     // N
    sc[1] = Lf[tri(B + 1, B)];                 // S1 = sum c
    sc[2] = Lf[tri(B + 1, B + 1)];             // S2 = sum c^2
  }
  for (int b = tid; b < B; b += kBlock) {
    g1[b] = Lf[tri(B, b)];
    g2[b] = Lf[tri(B + 1, b)];
  }
  __syncthreads();
  const double N = sc[0], S1 = sc[1], S2 = sc[2];
  for (int b = tid; b < B; b += kBlock) {
    const double mu_used = st.mu[b];           // what the pass subtracted
    const double t_used = st.t[b];
    const double sb = (double)a.s[b];
    double m;
    if (j == 0) {
      m = mu_used + g1[b] / N;                 // mu^0 = z + mean(L - z)
    } else {
      // Eq. 10: mean(L) - mean(c) t^{j-1}, with the exact sum c in the rounded forms
      m = st.lbar[b] - ((xref ? xmom[kXS1] : S1) / N) * st.t[b];
    }
    mun[b] = m;
    tn[b] = m * sb;                            // Eq. 9
    D[b] = mu_used - m;
    E[b] = j == 0 ? 0.0 : t_used - tn[b];
    if (xref) {
      U3[b] = t_used - tn[b];
      U3[kPad + b] = tn[b];
      U3[2 * kPad + b] = xmom[b] - xmom[kXS1] * st.lbar[b];   // m = sum c (L - mean L)
    }
  }
  for (int b = B + tid; b < kPad; b += kBlock) {
    U3[b] = 0.0;
    U3[kPad + b] = 0.0;
    U3[2 * kPad + b] = 0.0;
  }
  if (xref && tid == 0) rank3_S(S3, xmom[kXS1] / N, xmom[kXS2], N);
  __syncthreads();

  // ---- assembly of C (Eq. 11) into the register blocks
  double A_[kBlk][kBlk], C_[kBlk][kBlk];
  int myfail = 0;
#pragma unroll
  for (int x = 0; x < kBlk; ++x)
#pragma unroll
    for (int y = 0; y < kBlk; ++y) {
      const int i = kBlk * bi + x, jj = kBlk * bj + y;
      double c = (i == jj) ? 1.0 : 0.0;        // padding keeps the factor regular
      if (owner && i < B && jj < B && i >= jj) {
        c = Lf[tri(i, jj)];
        c += g1[i] * D[jj] + D[i] * g1[jj] + g2[i] * E[jj] + E[i] * g2[jj] +
             N * D[i] * D[jj] + S1 * (D[i] * E[jj] + E[i] * D[jj]) + S2 * E[i] * E[jj];
        c /= N;
        if (!isfinite(c)) myfail = 1;
      } else if (owner && i < B && jj < B) {
        c = 0.0;                               // upper half of a diagonal block: unused
      }
      A_[x][y] = c;
      C_[x][y] = c;
    }
  if (owner && (a.lowrank || a.exact_ref) && j == 0) {
#pragma unroll
    for (int x = 0; x < kBlk; ++x)
#pragma unroll
      for (int y = 0; y < kBlk; ++y) c0[blk_at(tid, x, y)] = A_[x][y];
  }

  if (myfail) fail = 1;
  __syncthreads();
  if (N <= (double)B) {
    if (tid == 0) st.status = MF_COL_FEW_PIXELS;
    return;
  }
  if (fail) {
    if (tid == 0) st.status = j == 0 ? MF_COL_NONFINITE : MF_COL_NOT_SPD;
    return;
  }

  if (a.lowrank) {
    // ---- low-rank form, pass 0: invert C^0 by a blocked symmetric sweep on
    // the 4x4 register blocks (A <- -A^-1 after all pivot blocks) and keep
    // C^0 and its inverse for the rank-3 solves of later iterations.  For
    // pivot block K with D = A_KK = L L^T and Y_i = A_iK L^-T:
    //   A_ij -= Y_i Y_j^T,  A_iK <- Y_i L^-1 (= A_iK D^-1),  A_KK <- -L^-T L^-1,
    // the four scalar sweeps of the block in one step; going through the
    // Cholesky factor of D (not D^-1) keeps the accuracy of the scalar
    // sweeps when adjacent bands make D ill-conditioned.  Block column K is
    // published by its owners right after their update of pivot block K - 1,
    // into alternating LDS buffers: one barrier per pivot block.  Padding
    // rows (>= B) are decoupled with unit diagonal.
    if (owner && bi == bj) {                // full symmetric diagonal blocks
#pragma unroll
      for (int x = 0; x < kBlk; ++x)
#pragma unroll
        for (int y = x + 1; y < kBlk; ++y) A_[x][y] = A_[y][x];
    }
    double* cb0 = Lf;                       // two [kNBlkRows][4][4] buffers
    double* cb1 = Lf + kNBlkRows * 16;
    auto publish = [&](int K, double* cb) {
      if (owner && bj == K) {               // A_iK, i >= K
#pragma unroll
        for (int x = 0; x < kBlk; ++x)
#pragma unroll
          for (int y = 0; y < kBlk; ++y) cb[bi * 16 + x * 4 + y] = A_[x][y];
      } else if (owner && bi == K) {        // A_jK = A_Kj^T, j < K
#pragma unroll
        for (int x = 0; x < kBlk; ++x)
#pragma unroll
          for (int y = 0; y < kBlk; ++y) cb[bj * 16 + y * 4 + x] = A_[x][y];
      }
    };
    const int nkb = (B + kBlk - 1) / kBlk;
    publish(0, cb0);
    __syncthreads();
    for (int K = 0; K < nkb; ++K) {
      const double* cb = (K & 1) ? cb1 : cb0;
      // D = L L^T and W = L^-1 (lower), every thread (same result)
      double Lc[kBlk][kBlk], W[kBlk][kBlk];
      if (!chol4(cb + K * 16, Lc, W)) {      // uniform
        if (tid == 0) st.status = MF_COL_NOT_SPD;
        return;
      }
      if (owner) {
        // Y = C W^T for the block rows this thread needs (C = A_iK from LDS)
        if (bi != K && bj != K) {
          double Yi[kBlk][kBlk], Yj[kBlk][kBlk];
          mul_wt(cb + bi * 16, W, Yi);
          mul_wt(cb + bj * 16, W, Yj);
#pragma unroll
          for (int x = 0; x < kBlk; ++x)
#pragma unroll
            for (int y = 0; y < kBlk; ++y) {
              double t = A_[x][y];
#pragma unroll
              for (int z = 0; z < kBlk; ++z) t = fma(-Yi[x][z], Yj[y][z], t);
              A_[x][y] = t;
            }
        } else if (bi == K && bj == K) {     // -W^T W (W lower: z >= max(x, y))
#pragma unroll
          for (int x = 0; x < kBlk; ++x)
#pragma unroll
            for (int y = 0; y < kBlk; ++y) {
              double t = 0.0;
#pragma unroll
              for (int z = (x > y ? x : y); z < kBlk; ++z) t = fma(W[z][x], W[z][y], t);
              A_[x][y] = -t;
            }
        } else {
          // column block (bj == K): A_iK <- Y_i W;  row block (bi == K):
          // A_Kj <- (Y_j W)^T
          double Y[kBlk][kBlk];
          mul_wt(cb + (bj == K ? bi : bj) * 16, W, Y);
          double R[kBlk][kBlk];
#pragma unroll
          for (int x = 0; x < kBlk; ++x)
#pragma unroll
            for (int y = 0; y < kBlk; ++y) {
              double t = 0.0;
#pragma unroll
              for (int z = y; z < kBlk; ++z) t = fma(Y[x][z], W[z][y], t);
              R[x][y] = t;
            }
          const bool colblk = bj == K;
#pragma unroll
          for (int x = 0; x < kBlk; ++x)
#pragma unroll
            for (int y = 0; y < kBlk; ++y) A_[x][y] = colblk ? R[x][y] : R[y][x];
        }
      }
      if (K + 1 < nkb) publish(K + 1, (K & 1) ? cb0 : cb1);
      __syncthreads();
    }
    // P = (C^0)^-1; rows/columns >= B zero
#pragma unroll
    for (int x = 0; x < kBlk; ++x)
#pragma unroll
      for (int y = 0; y < kBlk; ++y) {
        const int i = kBlk * bi + x, jj = kBlk * bj + y;
        A_[x][y] = (owner && i < B && jj <= i) ? -A_[x][y] : 0.0;
        if (!(owner && i < B && jj <= i)) C_[x][y] = 0.0;
      }
    if (owner) {
#pragma unroll
      for (int x = 0; x < kBlk; ++x)
#pragma unroll
        for (int y = 0; y < kBlk; ++y) pinv[blk_at(tid, x, y)] = A_[x][y];
    }
    for (int b = tid; b < kPad; b += kBlock) rbuf[b] = b < B ? tn[b] : 0.0;
    __syncthreads();
    block_symv<1>(A_, owner, bi, bj, tid, B, rbuf, vbuf, qsym);   // v = P t
    for (int step = 0; step < a.refine; ++step) {
      block_symv<1>(C_, owner, bi, bj, tid, B, vbuf, colk, qsym);  // C v
      for (int b = tid; b < kPad; b += kBlock) rbuf[b] = b < B ? tn[b] - colk[b] : 0.0;
      __syncthreads();
      block_symv<1>(A_, owner, bi, bj, tid, B, rbuf, colk, qsym);  // P r
      for (int b = tid; b < B; b += kBlock) vbuf[b] += colk[b];
      __syncthreads();
    }
  } else {
  // ---- blocked right-looking Cholesky on the register blocks, forming the
  // inverse factor X = L^-1 alongside.  For pivot block K with
  // D = A_KK = L_KK L_KK^T (W = L_KK^-1): the panel A_iK <- A_iK W^T = L_iK
  // (i > K), then A_ij -= L_iK L_jK^T (i >= j > K).  X comes from the same
  // steps applied to [L | I] (right-looking forward substitution): with R the
  // right-hand side, row block K of X is X_KJ = W R_KJ (J <= K), and then
  // R_iJ -= L_iK X_KJ (i > K >= J).  A thread's block becomes R once its L
  // block is published (as a panel), so X uses the registers and threads
  // that the factorisation leaves idle: two barriers per pivot block, as
  // for the factor alone.  At the end thread (i, j) holds X_ij.  Padding
  // rows (>= B) are decoupled with unit diagonal.
  const int nkb = (B + kBlk - 1) / kBlk;
  {
    double* lpan = Lf;                      // [kNBlkRows][4][4]: L_iK of block column K
    double* xrow = Lf + kNBlkRows * 16;     // [kNBlkRows][4][4]: X_KJ of block row K
    for (int K = 0; K < nkb; ++K) {
      if (owner && bi == K && bj == K) {
        double Lc[kBlk][kBlk], W[kBlk][kBlk];
        if (!chol4g([&](int r, int c) { return A_[r][c]; }, Lc, W)) fail = 1;
#pragma unroll
        for (int x = 0; x < kBlk; ++x)
#pragma unroll
          for (int y = 0; y < kBlk; ++y) {
            A_[x][y] = y <= x ? W[x][y] : 0.0;      // X_KK = W
            wbuf[K * 16 + x * 4 + y] = y <= x ? W[x][y] : 0.0;
          }
      }
      __syncthreads();
      if (fail) {                            // uniform
        if (tid == 0) st.status = MF_COL_NOT_SPD;
        return;
      }
      if (owner && ((bj == K && bi > K) || (bi == K && bj < K))) {
        double W[kBlk][kBlk], Y[kBlk][kBlk];
#pragma unroll
        for (int x = 0; x < kBlk; ++x)
#pragma unroll
          for (int y = 0; y < kBlk; ++y) W[x][y] = wbuf[K * 16 + x * 4 + y];
        if (bj == K) {
          // panel: L_iK = A_iK W^T, published; the block becomes
          // R_iK = -L_iK X_KK = -L_iK W
#pragma unroll
          for (int x = 0; x < kBlk; ++x)
#pragma unroll
            for (int y = 0; y < kBlk; ++y) {
              double t = 0.0;
#pragma unroll
              for (int z = 0; z <= y; ++z) t = fma(A_[x][z], W[y][z], t);
              Y[x][y] = t;
            }
#pragma unroll
          for (int x = 0; x < kBlk; ++x)
#pragma unroll
            for (int y = 0; y < kBlk; ++y) {
              lpan[bi * 16 + x * 4 + y] = Y[x][y];
              double t = 0.0;
#pragma unroll
              for (int z = y; z < kBlk; ++z) t = fma(Y[x][z], W[z][y], t);
              A_[x][y] = -t;
            }
        } else {
          // row block K of X: X_KJ = W R_KJ, published
#pragma unroll
          for (int x = 0; x < kBlk; ++x)
#pragma unroll
            for (int y = 0; y < kBlk; ++y) {
              double t = 0.0;
#pragma unroll
              for (int z = 0; z <= x; ++z) t = fma(W[x][z], A_[z][y], t);
              Y[x][y] = t;
            }
#pragma unroll
          for (int x = 0; x < kBlk; ++x)
#pragma unroll
            for (int y = 0; y < kBlk; ++y) {
              A_[x][y] = Y[x][y];
              xrow[bj * 16 + x * 4 + y] = Y[x][y];
            }
        }
      }
      __syncthreads();
      if (owner && bi > K && bj != K) {
        // trailing factor update (bj > K): A_ij -= L_iK L_jK^T;
        // right-hand side (bj < K): R_iJ -= L_iK X_KJ
        const bool trail = bj > K;
        double Li[kBlk][kBlk], M[kBlk][kBlk];
#pragma unroll
        for (int x = 0; x < kBlk; ++x)
#pragma unroll
          for (int z = 0; z < kBlk; ++z) {
            Li[x][z] = lpan[bi * 16 + x * 4 + z];
            M[x][z] = trail ? lpan[bj * 16 + x * 4 + z] : xrow[bj * 16 + x * 4 + z];
          }
#pragma unroll
        for (int x = 0; x < kBlk; ++x)
#pragma unroll
          for (int y = 0; y < kBlk; ++y) {
            double t = A_[x][y];
#pragma unroll
            for (int z = 0; z < kBlk; ++z) t = fma(-Li[x][z], trail ? M[y][z] : M[z][y], t);
            A_[x][y] = t;
          }
      }
    }
    __syncthreads();
  }
  // rounded forms: the refinement's residual matrix is C^0 (+ the rank-3
  // term), not the C assembled from the rounded Gram
  if (xref) load_block(c0, owner, tid, C_);
  // residual matrix: zero outside the lower triangle of the first B rows
#pragma unroll
  for (int x = 0; x < kBlk; ++x)
#pragma unroll
    for (int y = 0; y < kBlk; ++y) {
      const int i = kBlk * bi + x, jj = kBlk * bj + y;
      if (!(owner && i < B && jj <= i)) C_[x][y] = 0.0;
    }
  for (int b = tid; b < kPad; b += kBlock) {
    rbuf[b] = b < B ? tn[b] : 0.0;
    vbuf[b] = 0.0;
    dvec[b] = 0.0;
  }
  __syncthreads();

  // ---- v = C^-1 t, then refinement.  The exact forms refine against the C
  // they assembled.  The rounded forms' factor only preconditions: their
  // residual t - C^j v takes C^j = C^0 + U S U^T exactly (the rank-3
  // identity, from the FP64 C^0 of pass 0 and this pass's FP64 moments), so
  // each step contracts the error by about |I - C_f^-1 C^j| (1e-3 for the
  // FP32 Gram, 2e-2 for BF16) down to FP64 rounding.
  {
    block_inv_solve(A_, owner, bi, bj, tid, B, nkb, rbuf, colk, vbuf, qsym);
    for (int step = 0; step < a.refine; ++step) {
      if (xref && wid == 0) {
        double u[3];
        wave_dots<3, 1>(U3, vbuf, B, lane, u);
        if (lane == 0)
          for (int r = 0; r < 3; ++r) zb[r] = S3[r * 3] * u[0] + S3[r * 3 + 1] * u[1] + S3[r * 3 + 2] * u[2];
      }
      block_symv<1>(C_, owner, bi, bj, tid, B, vbuf, rbuf, qsym);   // C v (C^0 v)
      for (int b = tid; b < kPad; b += kBlock) {
        double cv = rbuf[b];
        if (xref) cv += U3[b] * zb[0] + U3[kPad + b] * zb[1] + U3[2 * kPad + b] * zb[2];
        rbuf[b] = b < B ? tn[b] - cv : 0.0;
      }
      __syncthreads();
      block_inv_solve(A_, owner, bi, bj, tid, B, nkb, rbuf, colk, dvec, qsym);
      for (int b = tid; b < B; b += kBlock) vbuf[b] += dvec[b];
      __syncthreads();
    }
  }
  }
  if (wid == 0) {
    const double q = wave_dot(tn, vbuf, B, lane);
    const double m2 = wave_dot(mun, mun, B, lane);
    if (lane == 0) {
      sc[3] = m2;
      st.q = q;
      if (j == 0) st.n_valid = N;
      if (!(q > 0.0) || !isfinite(q)) st.status = MF_COL_NOT_SPD;
      // column part of E^0 (R14): the sample covariance gives sum_i
      // (L_i - mu^0)^T C^0^-1 (L_i - mu^0) = N B
      else if (j == 0 && a.energy) a.energy[col] = 0.5 * N * (double)B;
    }
  }
  __syncthreads();
  for (int b = tid; b < kPad; b += kBlock) {
    const bool in = b < B;
    st.mu[b] = in ? mun[b] : 0.0;
    st.t[b] = in ? tn[b] : 0.0;
    st.v[b] = in ? vbuf[b] : 0.0;
    if (j == 0) {
      st.lbar[b] = in ? mun[b] : 0.0;
      st.m0[b] = in ? mun[b] / sc[3] : 0.0;
    }
  }
  if (a.ck && j == 0) {                          // checkpoint of iteration 0
    double* ck = a.ck + (int64_t)col * kCk;
    for (int b = tid; b < kPad; b += kBlock) {
      const bool in = b < B;
      ck[kCkMu + b] = in ? mun[b] : 0.0;
      ck[kCkT + b] = in ? tn[b] : 0.0;
      ck[kCkV + b] = in ? vbuf[b] : 0.0;
      ck[kCkM + b] = 0.0;
    }
    if (tid == 0) {
      ck[kCkScal + 0] = 0.0;
      ck[kCkScal + 1] = 0.0;
      ck[kCkScal + 2] = st.q;
      ck[kCkScal + 3] = N;
    }
  }
}

// ---------------------------------------------------------------------------
// Rank-3 solves.  C = C^0 + U S U^T (U = three LDS vectors, S a 3x3 matrix)
// with P = (C^0)^-1 and C^0 held in the 4x4 register blocks.  Woodbury:
//   C^-1 b = P b - X (I + S W)^-1 S U^T P b,   X = P U,  W = U^T X,
// then refinement steps against C applied exactly.  Everything is
// matrix-vector products on the register blocks (no factorisation).

struct R3Smem {
  double U3[3 * kPad];
  double X3[3 * kPad];
  double vbuf[kPad], rbuf[kPad], wbuf[kPad];
  alignas(16) double qsym[3 * kSymvScratch];
  double S3[9], Ginv[9], W3[9], zbuf[8];
  int bad;
};

// X = P U and Ginv = (I + S U^T X)^-1 (partial pivoting); sm.bad on failure.
__device__ void r3_prepare(const double (&Pb)[kBlk][kBlk], bool owner, int bi, int bj, int tid,
                           int B, R3Smem& sm) {
  const int lane = tid & 63, wid = tid >> 6;
  if (tid == 0) sm.bad = 0;
  block_symv<3>(Pb, owner, bi, bj, tid, B, sm.U3, sm.X3, sm.qsym);
  if (wid == 0) {
    double W[9];
    wave_dots<3, 3>(sm.U3, sm.X3, B, lane, W);
    if (lane == 0) {
      // Gauss-Jordan with partial pivoting on [M | I]; rows are exchanged by
      // selects, so every index is a compile-time constant (registers only)
      double A[3][6];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double s = (r == c) ? 1.0 : 0.0;
#pragma unroll
          for (int k = 0; k < 3; ++k) s += sm.S3[r * 3 + k] * W[k * 3 + c];
          A[r][c] = s;
          A[r][3 + c] = (r == c) ? 1.0 : 0.0;
        }
      bool ok = true;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int r = k + 1; r < 3; ++r) {
          const bool sw = fabs(A[r][k]) > fabs(A[k][k]);
#pragma unroll
          for (int c = 0; c < 6; ++c) {
            const double x = A[k][c], y = A[r][c];
            A[k][c] = sw ? y : x;
            A[r][c] = sw ? x : y;
          }
        }
        ok = ok && fabs(A[k][k]) > 0.0;
        const double inv = 1.0 / A[k][k];
#pragma unroll
        for (int c = 0; c < 6; ++c) A[k][c] *= inv;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          if (r == k) continue;
          const double f = A[r][k];
#pragma unroll
          for (int c = 0; c < 6; ++c) A[r][c] -= f * A[k][c];
        }
      }
      if (!ok) sm.bad = 1;
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) sm.Ginv[r * 3 + c] = A[r][3 + c];
#pragma unroll
      for (int e = 0; e < 9; ++e) sm.W3[e] = W[e];
    }
  }
  __syncthreads();
}

// sm.vbuf = C^-1 b (b: LDS vector, zero beyond B), with `refine` refinement
// steps.  pb, if not null, already holds P b (an LDS vector).
__device__ void r3_solve(const double (&Pb)[kBlk][kBlk], const double (&Cb)[kBlk][kBlk], bool owner,
                         int bi, int bj, int tid, int B, int refine, const double* b, R3Smem& sm,
                         const double* pb = nullptr) {
  const int lane = tid & 63, wid = tid >> 6;
  if (pb) {
    for (int e = tid; e < kPad; e += kBlock) sm.wbuf[e] = pb[e];
    __syncthreads();
  } else {
    block_symv<1>(Pb, owner, bi, bj, tid, B, b, sm.wbuf, sm.qsym);   // y = P b
  }
  for (int step = 0; step <= refine; ++step) {
    if (wid == 0) {
      double u[3];
      wave_dots<3, 1>(sm.U3, sm.wbuf, B, lane, u);
      if (lane == 0) {
        double su[3];
        for (int r = 0; r < 3; ++r)
          su[r] = sm.S3[r * 3] * u[0] + sm.S3[r * 3 + 1] * u[1] + sm.S3[r * 3 + 2] * u[2];
        for (int r = 0; r < 3; ++r)
          sm.zbuf[r] = sm.Ginv[r * 3] * su[0] + sm.Ginv[r * 3 + 1] * su[1] + sm.Ginv[r * 3 + 2] * su[2];
      }
    }
    __syncthreads();
    for (int e = tid; e < kPad; e += kBlock) {
      const double corr = e < B ? sm.wbuf[e] - (sm.X3[e] * sm.zbuf[0] + sm.X3[kPad + e] * sm.zbuf[1] +
                                                sm.X3[2 * kPad + e] * sm.zbuf[2]) : 0.0;
      if (step == 0) sm.vbuf[e] = corr;
      else if (e < B) sm.vbuf[e] += corr;
    }
    __syncthreads();
    if (step == refine) break;
    // residual r = b - C v, C v = C^0 v + U S U^T v
    block_symv<1>(Cb, owner, bi, bj, tid, B, sm.vbuf, sm.rbuf, sm.qsym);
    if (wid == 0) {
      double u[3];
      wave_dots<3, 1>(sm.U3, sm.vbuf, B, lane, u);
      if (lane == 0)
        for (int r = 0; r < 3; ++r)
          sm.zbuf[4 + r] = sm.S3[r * 3] * u[0] + sm.S3[r * 3 + 1] * u[1] + sm.S3[r * 3 + 2] * u[2];
    }
    __syncthreads();
    for (int e = tid; e < kPad; e += kBlock)
      sm.rbuf[e] = e < B ? b[e] - sm.rbuf[e] -
                               (sm.U3[e] * sm.zbuf[4] + sm.U3[kPad + e] * sm.zbuf[5] +
                                sm.U3[2 * kPad + e] * sm.zbuf[6])
                         : 0.0;
    __syncthreads();
    block_symv<1>(Pb, owner, bi, bj, tid, B, sm.rbuf, sm.wbuf, sm.qsym);   // P r
  }
}




// Low-rank form, iterations j >= 1: mu^j (Eq. 10), t^j (Eq. 9), C^j by the
// rank-3 identity, v^j = C^j^-1 t^j by the rank-3 solve, q^j.
__global__ void __launch_bounds__(kBlock) lowrank_kernel(SolveArgs a) {
  const int col = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  ColState& st = a.state[col];
  if (st.status != MF_COL_OK) return;
  const ColInfo ci = a.cols[col];
  const int B = a.B;
  const int64_t stride = (int64_t)a.partial_stride;
  const double* P = a.partials + (int64_t)ci.first_item * stride;

  __shared__ R3Smem sm;
  __shared__ double mun[kPad];
  __shared__ double sc[4];

  int bi = 0, bj = 0;
  const bool owner = tid < kNBlk;
  if (owner) block_coords(tid, bi, bj);
  // the column's moments: m (kPad), S1, S2 summed over its work items (and
  // the pixel part of E^{j-1} when the energy is tracked)
  const int nsum = kPad + (a.energy ? 3 : 2);
  for (int e = tid; e < nsum; e += kBlock) {
    double acc = 0.0;
#pragma unroll 8
    for (int it = 0; it < ci.n_items; ++it) acc += P[it * stride + e];
    sm.X3[e] = acc;                              // scratch until r3_prepare
  }
  __syncthreads();
  // P first, then the column's scalars and per-band state, then C^0: loads
  // retire in order, so waiting for the state waits for P but not for C^0,
  // which only the refinement needs.
  static_assert(kBlock >= kPad, "one band per thread");
  double Cb[kBlk][kBlk], Pb[kBlk][kBlk];
  load_block(a.pinv + (int64_t)col * (kNBlk * 16), owner, tid, Pb);
  const double nv = st.n_valid;
  double* eprev = a.energy ? a.energy + (int64_t)(a.j - 1) * a.n_cols + col : nullptr;
  const double e_old = eprev ? *eprev : 0.0;
  double lbar_b = 0.0, t_b = 0.0, s_b = 0.0;
  if (tid < B) {
    lbar_b = st.lbar[tid];
    t_b = st.t[tid];
    s_b = (double)a.s[tid];
  }
  load_block(a.c0 + (int64_t)col * (kNBlk * 16), owner, tid, Cb);
  if (tid == 0) {
    const double s1 = sm.X3[kVecS1], s2 = sm.X3[kVecS2];
    sc[0] = nv;
    sc[1] = s1;
    sc[2] = s2;
    rank3_S(sm.S3, s1 / nv, s2, nv);
    if (eprev) *eprev = e_old + sm.X3[kVecE];
  }
  __syncthreads();
  const double N = sc[0], S1 = sc[1], S2 = sc[2];
  const double abar = S1 / N;
  if (tid < kPad) {
    const int b = tid;
    double m = 0.0, mu = 0.0, t = 0.0, d = 0.0;
    if (b < B) {
      m = sm.X3[b];
      mu = lbar_b - abar * t_b;                  // Eq. 10
      t = mu * s_b;                              // Eq. 9
      d = t_b - t;
    }
    mun[b] = mu;
    sm.U3[b] = d;
    sm.U3[kPad + b] = t;
    sm.U3[2 * kPad + b] = m;
  }
  __syncthreads();
  r3_prepare(Pb, owner, bi, bj, tid, B, sm);
  if (sm.bad) {
    if (tid == 0) st.status = MF_COL_NOT_SPD;
    return;
  }
  if (a.energy && tid == 0) {
    // column part of E^j (R14): 1/2 sum_i (L_i - mu^j)^T C^j^-1 (L_i - mu^j)
    //   = N/2 (B - tr(S M)) + N abar^2 / 2 e^T M e,  M = U^T C^j^-1 U = W - W G S W
    //   (Woodbury with P = C^0^-1, W = U^T P U, G = (I + S W)^-1), e = (1, 1, 0):
    // mean(L) - mu^j = abar t^{j-1} = abar U e  (Eq. 10)
    double SW[9], GSW[9], M[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double x = 0.0;
        for (int k = 0; k < 3; ++k) x += sm.S3[r * 3 + k] * sm.W3[k * 3 + c];
        SW[r * 3 + c] = x;
      }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double x = 0.0;
        for (int k = 0; k < 3; ++k) x += sm.Ginv[r * 3 + k] * SW[k * 3 + c];
        GSW[r * 3 + c] = x;
      }
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double x = sm.W3[r * 3 + c];
        for (int k = 0; k < 3; ++k) x -= sm.W3[r * 3 + k] * GSW[k * 3 + c];
        M[r * 3 + c] = x;
      }
    double trSM = 0.0;
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) trSM += sm.S3[r * 3 + k] * M[k * 3 + r];
    const double eMe = M[0] + M[1] + M[3] + M[4];
    a.energy[(int64_t)a.j * a.n_cols + col] = 0.5 * N * ((double)B - trSM) + 0.5 * N * abar * abar * eMe;
  }
  // b = t^j is the second column of U, so P b is the second column of X = P U
  r3_solve(Pb, Cb, owner, bi, bj, tid, B, a.refine, sm.U3 + kPad, sm, sm.X3 + kPad);
  if (wid == 0) {
    const double q = wave_dot(sm.U3 + kPad, sm.vbuf, B, lane);
    if (lane == 0) {
      st.q = q;
      if (!(q > 0.0) || !isfinite(q)) {
        st.status = MF_COL_NOT_SPD;
        if (a.energy) a.energy[(int64_t)a.j * a.n_cols + col] = __builtin_nan("");
      }
    }
  }
  for (int b = tid; b < kPad; b += kBlock) {
    st.mu[b] = mun[b];
    st.t[b] = sm.U3[kPad + b];
    st.v[b] = sm.vbuf[b];
  }
  if (a.ck) {                                    // checkpoint of iteration j
    double* ck = a.ck + ((int64_t)a.j * a.n_cols + col) * kCk;
    for (int b = tid; b < kPad; b += kBlock) {
      ck[kCkMu + b] = mun[b];
      ck[kCkT + b] = sm.U3[kPad + b];
      ck[kCkV + b] = sm.vbuf[b];
      ck[kCkM + b] = sm.U3[2 * kPad + b];
    }
    __syncthreads();
    if (tid == 0) {
      ck[kCkScal + 0] = abar;
      ck[kCkScal + 1] = S2;
      ck[kCkScal + 2] = st.q;
      ck[kCkScal + 3] = N;
    }
  }
}

// ===========================================================================
// Adjoint: reverse mode through the K unrolled iterations (J = sum alpha^K
// weighted by the caller's grad_alpha).  Per iteration k = K..0, with
// abar_i the adjoint of alpha_i^k and zeta_i = abar_i [z_i > 0]:
//  pass A  pbar = zeta / (r q);  rbar += -zeta z / r;
//          adjoint of alpha^{k-1} through w (Eq. 5): zeta lam / (r q (a^{k-1} + eps)^2);
//          sums  Q1 = sum zeta z,  P1 = sum pbar,  V = sum pbar (L - mu^k)
//  col A   qbar = -Q1 / q,  vbar = V + qbar t,  u = C^-1 vbar (rank-3 solve),
//          tbar = tbar_in + qbar v + u,  mubar = -P1 v
//  pass B  with d_i = L_i - c_i t - mu (Eq. 11), c_i = r_i a_i^{k-1}:
//          alpha_i = v.d_i = p - c q,  beta_i = u.d_i,  dbar_i = -(alpha_i u + beta_i v) / N;
//          radiance-gradient coefficients  cv = pbar - beta / N (of v^k), cu = -alpha / N (of u^k);
//          cbar = -t.dbar = (alpha t.u + beta q) / N:  abar += r cbar,  rbar += a^{k-1} cbar;
//          sums  A0 = sum alpha, B0 = sum beta, A1 = sum c alpha, B1 = sum c beta
//  col B   mubar += (u A0 + v B0) / N,  tbar += (u A1 + v B1) / N,
//          mubar += tbar (.) s,  sbar += tbar (.) mu   (t = mu (.) s, Eq. 9);
//          k >= 1 (mu^k = mean L - a_k t^{k-1}, Eq. 10): Mbar += mubar,
//            gamma = -(mubar . t^{k-1}) / N is the uniform part of cbar, applied by the
//            next pass A as abar += r gamma, rbar += a^{k-1} gamma;  tbar_in = -a_k mubar
//          k = 0: Mbar += mubar + (sum rbar L) / |mu0|^2 - 2 (sum rbar r) mu0 / |mu0|^2  (Eq. 7)
// Finally G_i = sum_k (cv_i^k v^k + cu_i^k u^k) + rbar_i mu0 / |mu0|^2 + Mbar / N.

constexpr int kBwTbarIn = 0, kBwTbar = kPad, kBwMubar = 2 * kPad, kBwMbar = 3 * kPad,
              kBwSbar = 4 * kPad, kBwScal = 5 * kPad;          // scal: gamma, t.u, mu.u
constexpr int kBw = 5 * kPad + 8;
constexpr int kBwQ1 = 80, kBwP1 = 81;                          // pass A partial scalars
constexpr int kBwA0 = 80, kBwB0 = 81, kBwA1 = 82, kBwB1 = 83, kBwRR = 84;   // pass B

struct BwArgs {
  const float* L;
  int64_t n_floats;          // floats of the radiance array (max_px * B)
  const uint8_t* valid;
  const WorkItem* items;
  const ColState* state;
  const double* ck_k;        // checkpoints of iteration k, [n_cols][kCk]
  const double* a_k;         // alpha^k (FP64 checkpoint)
  const double* a_km1;       // alpha^{k-1}, or null for k = 0
  const double* p_k;         // p^k = (L - mu^k) . v^k per pixel (forward pass)
  const double* r_px;        // r per pixel (forward pass), 0 off valid pixels
  const float* grad_alpha;   // adjoint of alpha^K (k = K)
  double* abar;
  double* rbar;
  double* pbar;
  double* coef_v;            // coefficient of v^k in G, per pixel
  double* coef_u;            // coefficient of u^k in G, per pixel
  const double* bwcol;       // per-column backward state [n_cols][kBw]
  const double* u_k;         // u^k [n_cols][kPad]
  double* partials;
  int partial_stride;
  int B, k, K;
  double lam, eps;
  int albedo;
};

// Pass A is light per pixel; four waves per work item measured best (8 and 16
// waves per workgroup were slower, 2 about the same).
constexpr int kAW = 4;
constexpr int kABlock = 64 * kAW;
constexpr int kAChunk = 64;                // pixels per wave chunk in pass A
constexpr int kG = 8;                      // active pixels per radiance gather in pass A (4: 14.53,
                                           // 8: 14.35, 16: 14.31 ms forward + backward, 598x4000)

// Dynamic LDS of bwd_passA_kernel: per-pixel weights, partial rows, mu^k.
__host__ __device__ constexpr size_t bwdA_lds_bytes(int B) {
  return (size_t)kAW * kAChunk * sizeof(double) + kAW * (kPad + 8) * sizeof(double) +
         kPad * sizeof(double);
}

// Reverse pass A of iteration k.  p^k = (L - mu^k) . v^k and r per pixel come
// from the forward pass, so the radiance is read only for the pixels that
// carry a nonzero pbar (alpha^k > 0), row by row, for V = sum pbar (L - mu^k).
__global__ void __launch_bounds__(kABlock) bwd_passA_kernel(BwArgs a) {
  const WorkItem it = a.items[blockIdx.x];
  const ColState* __restrict__ st = a.state + it.col;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  const int B = a.B, k = a.k;
  const int64_t begin = it.px_begin, end = begin + it.n_px;
  extern __shared__ double dyn[];
  double* cbuf = dyn;                                   // [kAW][kAChunk]
  double* redm = cbuf + kAW * kAChunk;                   // [kAW][kPad + 8]
  double* mu = redm + kAW * (kPad + 8);                 // [kPad]

  if (st->status != MF_COL_OK) return;       // failed column: gradient 0 (assembly)
  const double* ck = a.ck_k + (int64_t)it.col * kCk;
  const double* bw = a.bwcol + (int64_t)it.col * kBw;
  for (int b = tid; b < kPad; b += kABlock) mu[b] = ck[kCkMu + b];
  __syncthreads();
  const double q = ck[kCkScal + 2];
  const double gamma = bw[kBwScal + 0];
  const double lam = a.lam, eps = a.eps;
  double m_lo = 0.0, m_hi = 0.0, s0 = 0.0, s1 = 0.0;
  // Per-pixel inputs of a chunk, through buffer resources sized to its pixels
  // (zero size past the work item, for a null pointer, or for an input this
  // iteration does not use, so those read zeros): no load is conditional, and
  // the next chunk's loads are in flight while the current one is processed.
  struct PxIn {
    uint32_t v;
    double pp, r, g, ab, rb, ak, am1;
  };
  const bool last = k == a.K;
  auto load_px = [&](int64_t c) {
    const int n = __builtin_amdgcn_readfirstlane((int)max<int64_t>(0, min<int64_t>(kAChunk, end - c)));
    PxIn x;
    x.v = load1(chunk_rsrc(a.valid ? a.valid + c : nullptr, a.valid ? n : 0), lane);
    x.pp = load8(chunk_rsrc(a.p_k + c, n * 8), lane * 8);
    x.r = load8(chunk_rsrc(a.r_px + c, n * 8), lane * 8);
    x.g = (double)load4(chunk_rsrc(a.grad_alpha + c, last ? n * 4 : 0), lane * 4);
    x.ab = load8(chunk_rsrc(a.abar + c, last ? 0 : n * 8), lane * 8);
    x.rb = load8(chunk_rsrc(a.rbar + c, last ? 0 : n * 8), lane * 8);
    x.ak = load8(chunk_rsrc(a.a_k + c, last ? 0 : n * 8), lane * 8);
    x.am1 = load8(chunk_rsrc(k >= 1 ? a.a_km1 + c : nullptr, k >= 1 ? n * 8 : 0), lane * 8);
    return x;
  };
  int64_t c0 = begin + (int64_t)kAChunk * wid;
  PxIn cur = load_px(c0);
  for (; c0 < end; c0 += kAW * kAChunk) {
    const PxIn nxt = load_px(c0 + kAW * kAChunk);
    const int n = (int)min<int64_t>(kAChunk, end - c0);
    const int64_t px = c0 + lane;
    const bool inb = lane < n;
    const bool ok = inb && (a.valid == nullptr || cur.v != 0u);
    const double pp = ok ? cur.pp : 0.0;
    const double r = ok ? cur.r : 0.0;          // 0 off valid pixels
    const bool live = ok && (r > 0.0);          // dark pixels keep alpha = 0
    double ab = 0.0, rb = 0.0;
    if (inb) {
      if (last) {
        ab = cur.g;
      } else {
        ab = cur.ab + r * gamma;
        rb = cur.rb + cur.ak * gamma;
      }
    }
    const double am1 = (k >= 1 && inb) ? cur.am1 : 0.0;
    const double w = k >= 1 ? lam / (am1 + eps) : 0.0;
    const double z = live ? (pp - w) / (r * q) : 0.0;
    const bool pos = (a.K == 0) || (z > 0.0);   // K = 0 returns alpha^0 unclamped
    const double zeta = (live && pos) ? ab : 0.0;
    const double pb = zeta != 0.0 ? zeta / (r * q) : 0.0;
    if (zeta != 0.0) rb -= zeta * z / r;
    const double abm1 = (k >= 1 && zeta != 0.0) ? zeta * lam / (r * q * (am1 + eps) * (am1 + eps)) : 0.0;
    if (inb) {
      a.abar[px] = ok ? abm1 : 0.0;
      a.pbar[px] = ok ? pb : 0.0;
      a.rbar[px] = ok ? rb : 0.0;
    }
    s0 += zeta != 0.0 ? zeta * z : 0.0;
    s1 += pb;
    uint64_t mask = __ballot(pb != 0.0);        // wave-uniform; sparse weights
    if (mask) {
      cbuf[wid * kAChunk + lane] = pb;
      wave_sync_lds();
      const float* Lc = a.L + c0 * B;
      const int b0 = lane, b1 = lane + 64;
      const double o0 = b0 < B ? mu[b0] : 0.0;
      const double o1 = b1 < B ? mu[b1] : 0.0;
      // rows of kG pixels in flight, through a resource over the chunk's
      // radiance: absent pixels and bands past B read zeros, so the loads
      // of a group issue together (no branch, no wait between them)
      const __amdgpu_buffer_rsrc_t rl = chunk_rsrc(Lc, __builtin_amdgcn_readfirstlane(n * B * 4));
      while (mask) {
        int pi[kG];
#pragma unroll
        for (int u = 0; u < kG; ++u) {
          pi[u] = mask ? (int)__builtin_ctzll(mask) : -1;
          mask &= mask - 1;
        }
        float l0[kG], l1[kG];
#pragma unroll
        for (int u = 0; u < kG; ++u) {
          const bool h = pi[u] >= 0;
          l0[u] = load4(rl, (h && b0 < B) ? (pi[u] * B + b0) * 4 : kOffNone);
          l1[u] = load4(rl, (h && b1 < B) ? (pi[u] * B + b1) * 4 : kOffNone);
        }
#pragma unroll
        for (int u = 0; u < kG; ++u) {
          if (pi[u] >= 0) {
            const double cp = cbuf[wid * kAChunk + pi[u]];
            m_lo = fma(cp, (double)l0[u] - o0, m_lo);
            m_hi = fma(cp, (double)l1[u] - o1, m_hi);
          }
        }
      }
      wave_sync_lds();
    }
    cur = nxt;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    s0 += __shfl_xor(s0, off, 64);
    s1 += __shfl_xor(s1, off, 64);
  }
  double* rw = redm + wid * (kPad + 8);
  if (lane < kPad) rw[lane] = lane < B ? m_lo : 0.0;
  if (lane + 64 < kPad) rw[lane + 64] = lane + 64 < B ? m_hi : 0.0;
  if (lane == 0) {
    rw[80] = s0;
    rw[81] = s1;
    rw[82] = 0.0;
    rw[83] = 0.0;
    rw[84] = 0.0;
  }
  __syncthreads();
  double* out = a.partials + (int64_t)blockIdx.x * a.partial_stride;
  for (int e = tid; e < kPad + 5; e += kABlock) {
    double sum = 0.0;
    for (int w = 0; w < kAW; ++w) sum += redm[w * (kPad + 8) + e];
    out[e] = sum;
  }
}

// Dynamic LDS of bwd_passB_kernel: per-pixel weights, partial rows, u^k, tiles.
__host__ __device__ constexpr size_t bwd_lds_bytes(int B) {
  return (size_t)kSW * kChunk * sizeof(double) + kSW * (kPad + 8) * sizeof(double) +
         kPad * sizeof(double) + (size_t)kSW * kTileF * sizeof(float);
}

// Reverse pass B of iteration k: streams the radiance for L . u^k; p^k and r
// come from the forward pass.  Same chunk pipeline as stream_kernel.
__global__ void __launch_bounds__(kSBlock) bwd_passB_kernel(BwArgs a) {
  const WorkItem it = a.items[blockIdx.x];
  const ColState* __restrict__ st = a.state + it.col;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  const int B = a.B, k = a.k;
  const int64_t begin = it.px_begin, end = begin + it.n_px;
  extern __shared__ double dyn[];
  double* cbuf = dyn;                                   // [kSW][kChunk]
  double* redm = cbuf + kSW * kChunk;                   // [kSW][kPad + 8]
  double* ucs = redm + kSW * (kPad + 8);                // [kPad] u^k
  float* my = reinterpret_cast<float*>(ucs + kPad) + wid * kTileF;

  const int64_t step = (int64_t)kSW * kChunk;
  int64_t c0 = begin + (int64_t)kChunk * wid;
  const int shift = (int)((reinterpret_cast<uintptr_t>(a.L + c0 * B) & 15) >> 2);
  const int n4 = (shift + kChunk * B + 3) / 4;
  auto span_ok = [&](int64_t c) {
    return c * B - shift >= 0 && (c * B - shift) + 4 * (int64_t)n4 <= a.n_floats;
  };
  const float* tile = my + shift;

  // per-pixel inputs, one chunk ahead: valid, p^k, r, alpha^{k-1}, pbar, abar, rbar
  float4 pre[kF4];
  uint32_t vld_n = 1;
  double pp_n = 0.0, r_n = 0.0, am_n = 0.0, pb_n = 0.0, ab_n = 0.0, rb_n = 0.0;
  const bool fast = c0 < end && span_ok(c0);
  const int pl = lane & (kChunk - 1);     // only lanes < kChunk score
  if (fast) {
    const int64_t px = c0 + pl;
    vld_n = a.valid ? (uint32_t)a.valid[px] : 1u;
    pp_n = a.p_k[px];
    r_n = a.r_px[px];
    am_n = k >= 1 ? a.a_km1[px] : 0.0;
    pb_n = a.pbar[px];
    ab_n = a.abar[px];
    rb_n = a.rbar[px];
    const __amdgpu_buffer_rsrc_t rs = chunk_rsrc(a.L + (c0 * B - shift), n4 * 16);
#pragma unroll
    for (int q = 0; q < kF4; ++q) pre[q] = load16(rs, (lane + 64 * q) * 16);
  }

  if (st->status != MF_COL_OK) return;       // failed column: gradient 0 (assembly)
  const double* ck = a.ck_k + (int64_t)it.col * kCk;
  const double* bw = a.bwcol + (int64_t)it.col * kBw;
  for (int b = tid; b < kPad; b += kSBlock) ucs[b] = a.u_k[(int64_t)it.col * kPad + b];
  __syncthreads();
  const double q = ck[kCkScal + 2], N = ck[kCkScal + 3];
  const double tu = bw[kBwScal + 1], muu = bw[kBwScal + 2];
  // weighted band sum (k = 0 only): sum rbar L
  const bool vec = k == 0;
  double m_lo = 0.0, m_hi = 0.0;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;

  // lanes l and l + 32 split pixel l's bands for L . u (as in the forward
  // streaming pass); everything after the dot product is the lower lane's
  const int hsplit = ((B + 3) / 4) * 2;
  const int upper = lane >> 5;
  auto score = [&](int64_t c0, int n, uint32_t vld, double pp, double r, double am1_in,
                   double pb_in, double ab_in, double rb_in, const float* tl) {
    const int pxl = lane & (kChunk - 1);
    const int64_t px = c0 + pxl;
    const bool okd = pxl < n && vld != 0;       // both halves of the pixel
    double le = 0.0, lo = 0.0;
    if (okd) {
      const float* rowp = tl + pxl * B;
      const double2* u2 = reinterpret_cast<const double2*>(ucs);
      int b = upper ? hsplit : 0;
      const int bend = upper ? B : hsplit;
      if ((B & 1) == 0 && (reinterpret_cast<uintptr_t>(tl) & 7) == 0) {
#pragma unroll 4
        for (; b + 1 < bend; b += 2) {
          const float2 l2 = *reinterpret_cast<const float2*>(rowp + b);
          const double2 cu = u2[b >> 1];
          le = fma((double)l2.x, cu.x, le);
          lo = fma((double)l2.y, cu.y, lo);
        }
      }
      for (; b < bend; ++b) le = fma((double)rowp[b], ucs[b], le);
    }
    double lu = le + lo;
    lu += __shfl_xor(lu, 32, 64);
    const bool inb = pxl < n && !upper;
    const bool ok = okd && !upper;
    if (!ok) {
      pp = 0.0;
      r = 0.0;
    }
    const bool live = ok && (r > 0.0);          // dark pixels keep alpha = 0
    double wgt = 0.0;
    const double am1 = (k >= 1 && live) ? am1_in : 0.0;
    const double c = r * am1;
    const double al = ok ? pp - c * q : 0.0;
    const double be = ok ? lu - c * tu - muu : 0.0;
    const double pb = inb ? pb_in : 0.0;
    const double cbar = (al * tu + be * q) / N;
    if (inb) {
      a.coef_v[px] = ok ? pb - be / N : 0.0;
      a.coef_u[px] = ok ? -al / N : 0.0;
      if (k >= 1 && live) {
        a.abar[px] = ab_in + r * cbar;
        a.rbar[px] = rb_in + am1 * cbar;
      }
    }
    s0 += al;
    s1 += be;
    s2 += c * al;
    s3 += c * be;
    if (k == 0) {
      const double rb = ok ? rb_in : 0.0;
      s4 += rb * r;
      wgt = rb;
    }
    if (vec && __ballot(wgt != 0.0)) {             // wave-uniform; sparse weights
      if (lane < kChunk) cbuf[wid * kChunk + lane] = wgt;
      wave_sync_lds();
      const int b0 = lane, b1 = lane + 64;
      for (int p = 0; p < n; ++p) {
        const double cp = cbuf[wid * kChunk + p];
        if (cp != 0.0) {
          if (b0 < B) m_lo = fma(cp, (double)tl[p * B + b0], m_lo);
          if (b1 < B) m_hi = fma(cp, (double)tl[p * B + b1], m_hi);
        }
      }
    }
    wave_sync_lds();
  };

  if (fast) {
    while (true) {
      const int n = (int)min<int64_t>(kChunk, end - c0);
      const uint32_t vld = vld_n;
      const double pp = pp_n, r = r_n, am = am_n, pb = pb_n, ab = ab_n, rb = rb_n;
      float4* t4 = reinterpret_cast<float4*>(my);
#pragma unroll
      for (int q = 0; q < kF4; ++q) t4[lane + 64 * q] = pre[q];
      wave_sync_lds();
      const int64_t nx = c0 + step;
      const bool more = nx < end && span_ok(nx);
      {                                       // in flight while this chunk is scored
        const int64_t cn = more ? nx : c0;
        const int64_t pn = cn + (more ? pl : 0);
        vld_n = a.valid ? (uint32_t)a.valid[pn] : 1u;
        pp_n = a.p_k[pn];
        r_n = a.r_px[pn];
        am_n = k >= 1 ? a.a_km1[pn] : 0.0;
        pb_n = a.pbar[pn];
        ab_n = a.abar[pn];
        rb_n = a.rbar[pn];
        const __amdgpu_buffer_rsrc_t rs = chunk_rsrc(a.L + (cn * B - shift), more ? n4 * 16 : 16);
#pragma unroll
        for (int q = 0; q < kF4; ++q) pre[q] = load16(rs, (lane + 64 * q) * 16);
      }
      score(c0, n, vld, pp, r, am, pb, ab, rb, tile);
      c0 = nx;
      if (!more) break;
    }
  }
  for (; c0 < end; c0 += step) {               // the last chunk of the array
    const int n = (int)min<int64_t>(kChunk, end - c0);
    const int64_t px = c0 + pl;
    const bool inb = pl < n;
    const uint32_t vld = (inb && a.valid) ? (uint32_t)a.valid[px] : 1u;
    const double pp = inb ? a.p_k[px] : 0.0, r = inb ? a.r_px[px] : 0.0;
    const double am = (inb && k >= 1) ? a.a_km1[px] : 0.0, pb = inb ? a.pbar[px] : 0.0;
    const double ab = inb ? a.abar[px] : 0.0, rb = inb ? a.rbar[px] : 0.0;
    copy_chunk(a.L + c0 * B, n * B, my, lane);
    score(c0, n, vld, pp, r, am, pb, ab, rb, my);
  }
  for (int off = 32; off >= 1; off >>= 1) {
    s0 += __shfl_xor(s0, off, 64);
    s1 += __shfl_xor(s1, off, 64);
    s2 += __shfl_xor(s2, off, 64);
    s3 += __shfl_xor(s3, off, 64);
    s4 += __shfl_xor(s4, off, 64);
  }
  double* rw = redm + wid * (kPad + 8);
  if (lane < kPad) rw[lane] = (vec && lane < B) ? m_lo : 0.0;
  if (lane + 64 < kPad) rw[lane + 64] = (vec && lane + 64 < B) ? m_hi : 0.0;
  if (lane == 0) {
    rw[80] = s0;
    rw[81] = s1;
    rw[82] = s2;
    rw[83] = s3;
    rw[84] = s4;
  }
  __syncthreads();
  double* out = a.partials + (int64_t)blockIdx.x * a.partial_stride;
  for (int e = tid; e < kPad + 5; e += kSBlock) {
    double sum = 0.0;
    for (int w = 0; w < kSW; ++w) sum += redm[w * (kPad + 8) + e];
    out[e] = sum;
  }
}

struct BwColArgs {
  const ColInfo* cols;
  const ColState* state;
  const double* ck_k;        // [n_cols][kCk] of iteration k
  const double* ck_km1;      // of iteration k - 1 (k >= 1)
  const double* c0;
  const double* pinv;
  const double* partials;
  double* bwcol;
  double* u_k;
  const float* s;
  int partial_stride;
  int B, k, refine, albedo;
};

__global__ void bwd_init_kernel(double* bwcol, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) bwcol[e] = 0.0;
}

// col A: vbar, u = C^k^-1 vbar, tbar, mubar.
__global__ void __launch_bounds__(kBlock) bwd_colA_kernel(BwColArgs a) {
  const int col = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const ColState& st = a.state[col];
  if (st.status != MF_COL_OK) return;
  const ColInfo ci = a.cols[col];
  const int B = a.B, k = a.k;
  const int64_t stride = a.partial_stride;
  const double* P = a.partials + (int64_t)ci.first_item * stride;
  const double* ck = a.ck_k + (int64_t)col * kCk;
  double* bw = a.bwcol + (int64_t)col * kBw;

  __shared__ R3Smem sm;
  __shared__ double vbar[kPad];
  __shared__ double sc[2];
  int bi = 0, bj = 0;
  const bool owner = tid < kNBlk;
  if (owner) block_coords(tid, bi, bj);
  const double q = ck[kCkScal + 2], N = ck[kCkScal + 3];
  // pass A sums over the column's work items: V (kPad), Q1, P1
  for (int e = tid; e < kPad + 2; e += kBlock) {
    double acc = 0.0;
#pragma unroll 8
    for (int it = 0; it < ci.n_items; ++it) acc += P[it * stride + e];
    sm.X3[e] = acc;                              // scratch until r3_prepare
  }
  __syncthreads();
  // P first, then the checkpointed state, then C^0 (as in lowrank_kernel)
  static_assert(kBlock >= kPad, "one band per thread");
  double Cb[kBlk][kBlk], Pb[kBlk][kBlk];
  load_block(a.pinv + (int64_t)col * (kNBlk * 16), owner, tid, Pb);
  const double ab_k = ck[kCkScal + 0], s2_k = ck[kCkScal + 1];
  const double* ckm1 = k >= 1 ? a.ck_km1 + (int64_t)col * kCk : nullptr;
  double t_b = 0.0, tm1_b = 0.0, m_b = 0.0;
  if (tid < kPad) {
    t_b = ck[kCkT + tid];
    if (k >= 1 && tid < B) {
      tm1_b = ckm1[kCkT + tid];
      m_b = ck[kCkM + tid];
    }
  }
  load_block(a.c0 + (int64_t)col * (kNBlk * 16), owner, tid, Cb);
  if (tid == 0) {
    sc[0] = sm.X3[kBwQ1];
    sc[1] = sm.X3[kBwP1];
    if (k >= 1) rank3_S(sm.S3, ab_k, s2_k, N);
    else
      for (int e = 0; e < 9; ++e) sm.S3[e] = 0.0;
  }
  __syncthreads();
  const double qbar = -sc[0] / q, P1 = sc[1];
  if (tid < kPad) {
    const int b = tid;
    const double V = b < B ? sm.X3[b] : 0.0;
    const double t = t_b;
    vbar[b] = b < B ? V + qbar * t : 0.0;
    sm.U3[b] = (k >= 1 && b < B) ? tm1_b - t : 0.0;
    sm.U3[kPad + b] = (k >= 1 && b < B) ? t : 0.0;
    sm.U3[2 * kPad + b] = (k >= 1 && b < B) ? m_b : 0.0;
  }
  __syncthreads();
  r3_prepare(Pb, owner, bi, bj, tid, B, sm);
  r3_solve(Pb, Cb, owner, bi, bj, tid, B, a.refine, vbar, sm);      // u in sm.vbuf
  for (int b = tid; b < kPad; b += kBlock) {
    const double u = b < B ? sm.vbuf[b] : 0.0;
    const double v = ck[kCkV + b];
    a.u_k[(int64_t)col * kPad + b] = u;
    bw[kBwTbar + b] = b < B ? bw[kBwTbarIn + b] + qbar * v + u : 0.0;
    bw[kBwMubar + b] = b < B ? -P1 * v : 0.0;
    sm.rbuf[b] = u;
  }
  __syncthreads();
  if (wid == 0) {
    double tu = 0.0, muu = 0.0;
    for (int b = lane; b < B; b += 64) {
      tu += ck[kCkT + b] * sm.rbuf[b];
      muu += ck[kCkMu + b] * sm.rbuf[b];
    }
    for (int off = 32; off >= 1; off >>= 1) {
      tu += __shfl_xor(tu, off, 64);
      muu += __shfl_xor(muu, off, 64);
    }
    if (lane == 0) {
      bw[kBwScal + 1] = tu;
      bw[kBwScal + 2] = muu;
    }
  }
}

// col B: finish mubar and tbar of iteration k, sbar, and hand over to k - 1.
__global__ void __launch_bounds__(128) bwd_colB_kernel(BwColArgs a) {
  const int col = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const ColState& st = a.state[col];
  if (st.status != MF_COL_OK) return;
  const ColInfo ci = a.cols[col];
  const int B = a.B, k = a.k;
  const int64_t stride = a.partial_stride;
  const double* P = a.partials + (int64_t)ci.first_item * stride;
  const double* ck = a.ck_k + (int64_t)col * kCk;
  const double* u = a.u_k + (int64_t)col * kPad;
  double* bw = a.bwcol + (int64_t)col * kBw;
  __shared__ double mub[kPad], sc[8];
  if (tid == 0) {
    double A0 = 0.0, B0 = 0.0, A1 = 0.0, B1 = 0.0, RR = 0.0;
    for (int it = 0; it < ci.n_items; ++it) {
      A0 += P[it * stride + kBwA0];
      B0 += P[it * stride + kBwB0];
      A1 += P[it * stride + kBwA1];
      B1 += P[it * stride + kBwB1];
      RR += P[it * stride + kBwRR];
    }
    sc[0] = A0; sc[1] = B0; sc[2] = A1; sc[3] = B1; sc[4] = RR;
  }
  __syncthreads();
  const double N = ck[kCkScal + 3];
  for (int b = tid; b < kPad; b += 128) {
    double mubar = 0.0, tbar = 0.0;
    if (b < B) {
      const double v = ck[kCkV + b];
      mubar = bw[kBwMubar + b] + (u[b] * sc[0] + v * sc[1]) / N;
      tbar = bw[kBwTbar + b] + (u[b] * sc[2] + v * sc[3]) / N;
      mubar += tbar * (double)a.s[b];                 // t = mu (.) s
      bw[kBwSbar + b] += tbar * ck[kCkMu + b];
    }
    mub[b] = mubar;
  }
  __syncthreads();
  if (k >= 1) {
    const double* ckm1 = a.ck_km1 + (int64_t)col * kCk;
    if (wid == 0) {
      double d = 0.0;
      for (int b = lane; b < B; b += 64) d += mub[b] * ckm1[kCkT + b];
      for (int off = 32; off >= 1; off >>= 1) d += __shfl_xor(d, off, 64);
      if (lane == 0) bw[kBwScal + 0] = -d / N;       // gamma for pass A(k-1)
    }
    const double ak = ck[kCkScal + 0];
    for (int b = tid; b < kPad; b += 128) {
      bw[kBwMbar + b] += mub[b];
      bw[kBwTbarIn + b] = -ak * mub[b];
    }
  } else {
    // albedo factor r_i = L_i . mu0 / |mu0|^2 (Eq. 7), mu0 = mean L
    if (wid == 0) {
      double m2 = 0.0;
      for (int b = lane; b < B; b += 64) m2 += st.lbar[b] * st.lbar[b];
      for (int off = 32; off >= 1; off >>= 1) m2 += __shfl_xor(m2, off, 64);
      if (lane == 0) sc[5] = m2;
    }
    __syncthreads();
    const double m2 = sc[5];
    for (int b = tid; b < B; b += 128) {
      double RL = 0.0;
      for (int it = 0; it < ci.n_items; ++it) RL += P[it * stride + b];
      double alb = 0.0;
      if (a.albedo) alb = RL / m2 - 2.0 * sc[4] * st.lbar[b] / m2;
      bw[kBwMbar + b] += mub[b] + alb;
    }
  }
}

// G_i = sum_k (cv_i^k v^k + cu_i^k u^k) + rbar_i mu0 / |mu0|^2 + Mbar / N.
struct BwAsmArgs {
  const WorkItem* items;
  const ColState* state;
  const uint8_t* valid;
  const double* ck;          // [K+1][n_cols][kCk]
  const double* u_hist;      // [K+1][n_cols][kPad]
  const double* coef;        // [2(K+1)][max_px]
  const double* rbar;
  const double* bwcol;
  float* grad_L;
  int64_t max_px;
  int n_cols, B, K, albedo;
};

// Gradient assembly as one FP64 product per column: the pixel's coefficient
// row (2 (K+1) slots, then rbar and 1) times the column's basis (v^k and u^k
// rows, then m0 and Mbar / N), both padded to 64 rows.
constexpr int kAsmRows = 64;
constexpr int kAsmTiles = kPad / 16;

__host__ __device__ constexpr size_t asm_lds_bytes(int B, int K) {
  return (size_t)kAsmRows * kPad * sizeof(double);
}

// Four waves share the column's basis in LDS; each wave takes 16 pixels at a
// time on v_mfma_f64_16x16x4f64 (A: pixels x coefficient slots from global,
// B: slots x bands from LDS), 16 slot steps x 5 band tiles.
__global__ void __launch_bounds__(256) bwd_assemble_kernel(BwAsmArgs a) {
  const WorkItem it = a.items[blockIdx.x];
  const ColState& st = a.state[it.col];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int row = lane & 15, kq = lane >> 4;
  const int B = a.B, nb = 2 * (a.K + 1);
  const int64_t begin = it.px_begin, end = begin + it.n_px;
  extern __shared__ double dyn[];
  double* basis = dyn;                                // [kAsmRows][kPad]
  const bool good = st.status == MF_COL_OK;
  const double N = good ? (double)st.n_valid : 1.0;
  const double* bw = a.bwcol + (int64_t)it.col * kBw;
  for (int e = tid; e < kAsmRows * kPad; e += 256) {
    const int j = e / kPad, b = e - j * kPad;
    double v = 0.0;
    if (good && b < B) {
      if (j < nb) {
        const int kk = j >> 1;
        v = (j & 1) ? a.u_hist[((int64_t)kk * a.n_cols + it.col) * kPad + b]
                    : a.ck[((int64_t)kk * a.n_cols + it.col) * kCk + kCkV + b];
      } else if (j == kAsmRows - 2) {
        v = a.albedo ? st.m0[b] : 0.0;
      } else if (j == kAsmRows - 1) {
        v = bw[kBwMbar + b] / N;
      }
    }
    basis[e] = v;
  }
  __syncthreads();
  for (int64_t p0 = begin + 16 * wid; p0 < end; p0 += 64) {
    const int64_t px = p0 + row;                       // A row of this lane
    bool ok = good && px < end;
    if (ok && a.valid) ok = a.valid[px] != 0;
    double cf[kAsmRows / 4];
#pragma unroll
    for (int s = 0; s < kAsmRows / 4; ++s) {
      const int j = 4 * s + kq;
      double v = 0.0;
      if (ok) {
        if (j < nb) v = a.coef[(int64_t)j * a.max_px + px];
        else if (j == kAsmRows - 2) v = a.rbar[px];
        else if (j == kAsmRows - 1) v = 1.0;
      }
      cf[s] = v;
    }
    doublex4 acc[kAsmTiles];
#pragma unroll
    for (int t = 0; t < kAsmTiles; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
    // an opaque zero keeps the basis reads inside the loop (hoisted out of
    // it they would hold 160 registers per lane)
    int off = (kq * kPad + row);
    asm volatile("" : "+v"(off));
#pragma unroll
    for (int s = 0; s < kAsmRows / 4; ++s) {
      const double* brow = basis + 4 * s * kPad + off;
#pragma unroll
      for (int t = 0; t < kAsmTiles; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(cf[s], brow[16 * t], acc[t], 0, 0, 0);
    }
    // D layout: register i of this lane holds pixel p0 + 4 i + kq, band 16 t + row
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t q = p0 + 4 * i + kq;
      if (q < end) {
        float* g = a.grad_L + q * B;
#pragma unroll
        for (int t = 0; t < kAsmTiles; ++t)
          if (16 * t + row < B) g[16 * t + row] = (float)acc[t][i];
      }
    }
  }
}

// grad_s[b] = sum over healthy columns of sbar (one workgroup per band).
__global__ void __launch_bounds__(256) bwd_sbar_kernel(const ColState* state, const double* bwcol,
                                                       int n_cols, double* grad_s) {
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  __shared__ double red[4];
  double s = 0.0;
  for (int c = tid; c < n_cols; c += 256)
    if (state[c].status == MF_COL_OK) s += bwcol[(int64_t)c * kBw + kBwSbar + b];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) grad_s[b] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Plain streaming read: the achievable HBM read bandwidth for this access
// size, used as the measured ceiling next to the nominal 8 TB/s.
__global__ void __launch_bounds__(kBlock) stream_read_kernel(const float* __restrict__ src, int64_t nfl,
                                                             int64_t per_blk, float* __restrict__ sink) {
  // each workgroup reads its own contiguous span (per_blk floats, a multiple
  // of 4) with 8 non-temporal 16-byte loads in flight per lane
  const int64_t b0 = (int64_t)blockIdx.x * per_blk;
  if (b0 >= nfl) return;
  const int64_t len = b0 + per_blk <= nfl ? per_blk : nfl - b0;
  const __amdgpu_buffer_rsrc_t rs = chunk_rsrc(src + b0, (int)(len * 4));
  float acc = 0.f;
  for (int off = threadIdx.x * 16; off < (int)(len * 4); off += kBlock * 16 * 8) {
    float4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = load16(rs, off + u * kBlock * 16);
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  if (acc == 1.2345e-30f) sink[blockIdx.x] = acc;   // keeps the loads alive
}

// ---------------------------------------------------------------------------
// Ingest: band-interleaved-by-line cube [line][band][sample] (the ENVI "BIL"
// layout of imaging-spectrometer radiance files) to the column-contiguous
// [sample][line][band] layout of the retrieval, optionally with the valid mask
// (0 where a band is non-finite or equals the no-data value).  A workgroup
// moves a tile of kRpS samples x kRpL lines through LDS: rows of kRpS samples
// are read coalesced, and each sample's kRpL x B floats are written as one
// contiguous run.  The LDS rows are padded by one float (no bank conflicts
// when a sample's bands are gathered).
constexpr int kRpS = 64;
constexpr int kRpL = 2;
constexpr int kRpRow = kRpS + 1;

__global__ void __launch_bounds__(256) repack_bil_kernel(const float* __restrict__ bil, int64_t n_lines,
                                                         int B, int n_samples, float* __restrict__ out,
                                                         uint8_t* __restrict__ valid, int64_t first_px,
                                                         int use_nodata, float nodata) {
  extern __shared__ float tile[];                      // [kRpL][B][kRpRow]
  const int tid = threadIdx.x;
  const int64_t l0 = (int64_t)blockIdx.x * kRpL;       // lines on x (no 64 K limit)
  const int s0 = blockIdx.y * kRpS;
  const int ns = min(kRpS, n_samples - s0);
  const int nl = (int)min<int64_t>(kRpL, n_lines - l0);
  // read: rows (line l, band b) of ns samples
  const int nrows = nl * B;
  for (int e = tid; e < nrows * kRpS; e += 256) {
    const int r = e / kRpS, s = e - r * kRpS;
    if (s < ns) {
      const int l = r / B, b = r - l * B;
      tile[(l * B + b) * kRpRow + s] = bil[((l0 + l) * B + b) * (int64_t)n_samples + s0 + s];
    }
  }
  __syncthreads();
  // write: for each sample, nl consecutive pixels of B floats (one run)
  const int run = nl * B;
  for (int e = tid; e < ns * run; e += 256) {
    const int s = e / run, k = e - s * run;
    const int l = k / B, b = k - l * B;
    out[((first_px + (int64_t)(s0 + s) * n_lines + l0) * B) + k] = tile[(l * B + b) * kRpRow + s];
  }
  if (valid) {
    for (int e = tid; e < ns * nl; e += 256) {
      const int s = e / nl, l = e - s * nl;
      bool ok = true;
      for (int b = 0; b < B; ++b) {
        const float x = tile[(l * B + b) * kRpRow + s];
        ok = ok && isfinite(x) && !(use_nodata && x == nodata);
      }
      valid[first_px + (int64_t)(s0 + s) * n_lines + l0 + l] = ok ? 1 : 0;
    }
  }
}

// Adds the pixel part of E^K (the last streaming pass, partial slot kVecE of
// each work item) to the column part the last solve wrote, for the columns
// that finished healthy.
__global__ void energy_last_kernel(const ColInfo* __restrict__ cols, const ColState* __restrict__ state,
                                   const double* __restrict__ partials, int64_t stride,
                                   double* __restrict__ energy_k, int64_t n_cols) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= n_cols || state[col].status != MF_COL_OK) return;
  const ColInfo ci = cols[col];
  double acc = 0.0;
  for (int it = 0; it < ci.n_items; ++it) acc += partials[(int64_t)(ci.first_item + it) * stride + kVecE];
  energy_k[col] += acc;
}

__global__ void status_kernel(const ColState* __restrict__ state, int32_t* __restrict__ out,
                              int64_t n) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) out[c] = state[c].status;
}

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
  ColInfo* cols_d = nullptr;
  WorkItem* items_d = nullptr;
  size_t off_state = 0, off_partials = 0, off_c0 = 0, off_pinv = 0, off_alpha0 = 0, off_alpha1 = 0;
  // save_for_backward: checkpoints and adjoint buffers
  size_t off_r = 0, off_ck_alpha = 0, off_ck_col = 0, off_ck_p = 0, off_bw_px = 0, off_bw_coef = 0, off_bw_u = 0,
         off_bw_col = 0;
  size_t off_energy = 0;     // track_energy: E^k per partition [K+1][n_cols]
  size_t ws_bytes = 0;
  void* scratch_d = nullptr; // this device's `scratch` (mf_retrieve_noalloc)
  // launch shape of the passes (mf_plan_set_launch)
  int stream_tile = 0;       // MF_TILE_*
  int wgs_per_cu = 0;        // 0: one workgroup per work item; n: persistent grid
  int n_cu = 0;
  int32_t* order_d = nullptr; // work items, longest first (persistent launches)
  size_t off_queue = 0;      // K + 2 queue counters
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
  if (!a.queue) return (unsigned)p->n_items;
  return (unsigned)std::min<int64_t>(p->n_items, (int64_t)p->wgs_per_cu * p->n_cu);
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
  const dim3 g((unsigned)p->n_items), b(kBlock);
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
    default:
      if (rin) hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_BF16, true, true>), g, b, 0, s, a);
      else hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_BF16, true, false>), g, b, 0, s, a);
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

void dispatch_solve(const mf_plan_s* p, const SolveArgs& a, hipStream_t s) {
  const dim3 g((unsigned)p->n_cols), b(kBlock);
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

// Doubles per work item in the partial buffer: the item's partial Gram (T
// tiles of 16 x 16; the low-rank form's vector moments fit in it), plus the
// exact moments of the rounded Gram forms.
int64_t partial_stride(const mf_plan_s* p) {
  const bool rounded = p->opt.cov == MF_COV_GRAM_FP32 || p->opt.cov == MF_COV_GRAM_BF16;
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
    case MF_COV_GRAM_FP64: return PM_F64;
    default: return j == 0 ? PM_F64 : PM_VEC;   // MF_COV_LOWRANK
  }
}


}  // namespace

namespace {
// The launch sequence of one retrieval (also what a graph captures).
void enqueue_retrieve(mf_plan_s* p, const float* radiance, const uint8_t* valid, const float* s,
                      float* alpha, int32_t* column_status, void* workspace, hipStream_t st) {
  char* ws = (char*)workspace;
  ColState* state = (ColState*)(ws + p->off_state);
  double* partials = (double*)(ws + p->off_partials);
  double* abuf[2] = {(double*)(ws + p->off_alpha0), (double*)(ws + p->off_alpha1)};
  double* ck_alpha = p->opt.save_for_backward ? (double*)(ws + p->off_ck_alpha) : nullptr;
  double* ck_p = p->opt.save_for_backward ? (double*)(ws + p->off_ck_p) : nullptr;
  const int B = p->opt.n_bands;
  const int K = p->opt.n_iter;
  double* energy = p->opt.track_energy ? (double*)(ws + p->off_energy) : nullptr;
  int* queue = p->wgs_per_cu > 0 ? (int*)(ws + p->off_queue) : nullptr;

  {
    LaunchTimer tm(p, MF_KERNEL_OTHER, st);
    hipLaunchKernelGGL(setup_kernel, dim3((unsigned)p->n_cols), dim3(64), 0, st, radiance, valid,
                       p->cols_d, state, B, energy, K + 1, p->n_cols, queue, K + 2);
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
  sa.exact_ref = p->opt.cov == MF_COV_GRAM_FP32 || p->opt.cov == MF_COV_GRAM_BF16;
  sa.ck = p->opt.save_for_backward ? (double*)(ws + p->off_ck_col) : nullptr;
  sa.n_cols = (int)p->n_cols;
  sa.energy = energy;
  pa.order = p->order_d;
  pa.n_items = (int)p->n_items;
  for (int j = 0; j <= K + 1; ++j) {
    pa.j = j;
    pa.queue = queue ? queue + j : nullptr;
    pa.track_energy = (energy && j >= 1) ? 1 : 0;
    pa.unclamped = (j == 1 && K == 0) ? 1 : 0;
    if (ck_alpha) {          // save_for_backward: keep alpha^0..alpha^K
      pa.alpha_prev = j >= 2 ? ck_alpha + (int64_t)(j - 2) * p->max_px : nullptr;
      pa.alpha_out = j >= 1 ? ck_alpha + (int64_t)(j - 1) * p->max_px : nullptr;
    } else {
      pa.alpha_prev = j >= 2 ? abuf[(j - 2) & 1] : nullptr;
      pa.alpha_out = (j >= 1 && j <= K) ? abuf[(j - 1) & 1] : nullptr;
    }
    pa.alpha_final = j == K + 1 ? alpha : nullptr;
    pa.p_save = (ck_p && j >= 1) ? ck_p + (int64_t)(j - 1) * p->max_px : nullptr;
    // r per pixel: written by pass 1, read by every later scored pass
    double* rbuf = (double*)(ws + p->off_r);
    pa.r_out = j == 1 ? rbuf : nullptr;
    pa.r_in = j >= 2 ? rbuf : nullptr;
    const bool mom = j <= K;
    const int mode = pass_mode(p->opt.cov, j, K);
    {
      LaunchTimer tm(p, j == 0 ? MF_KERNEL_PASS_INIT
                        : mode == PM_NONE ? MF_KERNEL_PASS_LAST
                        : mode == PM_VEC ? MF_KERNEL_PASS_VEC : MF_KERNEL_PASS_GRAM, st);
      dispatch_pass(p, pa, mode, st);
    }
    if (mom) {
      sa.j = j;
      LaunchTimer tm(p, MF_KERNEL_SOLVE, st);
      if (sa.lowrank && j >= 1)
        hipLaunchKernelGGL(lowrank_kernel, dim3((unsigned)p->n_cols), dim3(kBlock), 0, st, sa);
      else
        dispatch_solve(p, sa, st);
    }
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
  if (opt->cov < MF_COV_LOWRANK || opt->cov > MF_COV_GRAM_BF16)
    return fail_with(MF_E_ARG, "cov must be one of MF_COV_*");
  if (opt->refine_steps < -1 || opt->refine_steps > 8)
    return fail_with(MF_E_ARG, "refine_steps must be -1 (the form's default) or in [0, 8]");
  if (opt->save_for_backward != 0 && opt->save_for_backward != 1)
    return fail_with(MF_E_ARG, "save_for_backward must be 0 or 1");
  if (opt->save_for_backward && opt->cov != MF_COV_LOWRANK)
    return fail_with(MF_E_UNSUPPORTED, "save_for_backward needs the low-rank covariance form");
  if (opt->save_for_backward && opt->n_iter > 30)
    return fail_with(MF_E_UNSUPPORTED, "save_for_backward supports n_iter <= 30");
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
  int64_t n_px = 0, max_px = 0;
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
        w.col = (int32_t)cols.size();
        w.n_px = std::min(per, npart - done);
        done += w.n_px;
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
  p->off_r = off;                              // r per pixel (written by pass 1)
  off = align256(off + (size_t)max_px * sizeof(double));
  if (opt->save_for_backward) {
    const size_t K1 = (size_t)opt->n_iter + 1;
    p->off_ck_alpha = off;
    off = align256(off + K1 * (size_t)max_px * sizeof(double));
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
  }
  if (opt->track_energy) {
    p->off_energy = off;
    off = align256(off + ((size_t)opt->n_iter + 1) * (size_t)p->n_cols * sizeof(double));
  }
  p->off_queue = off;                          // persistent launches' queue counters
  off = align256(off + ((size_t)opt->n_iter + 2) * sizeof(int));
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
  const size_t lds = bwd_lds_bytes(B), ldsA = bwdA_lds_bytes(B);
  for (int k = K; k >= 0; --k) {
    ba.k = ca.k = k;
    ba.ck_k = ca.ck_k = ck_col + (int64_t)k * p->n_cols * kCk;
    ca.ck_km1 = k >= 1 ? ck_col + (int64_t)(k - 1) * p->n_cols * kCk : nullptr;
    ba.a_k = ck_alpha + (int64_t)k * mp;
    ba.a_km1 = k >= 1 ? ck_alpha + (int64_t)(k - 1) * mp : nullptr;
    ba.p_k = ck_p + (int64_t)k * mp;
    ba.coef_v = coef + (int64_t)(2 * k) * mp;
    ba.coef_u = coef + (int64_t)(2 * k + 1) * mp;
    ba.u_k = ca.u_k = u_hist + (int64_t)k * p->n_cols * kPad;
    {
      LaunchTimer tm(p, MF_KERNEL_PASS_VEC, st);
      hipLaunchKernelGGL(bwd_passA_kernel, dim3((unsigned)p->n_items), dim3(kABlock), ldsA, st, ba);
    }
    {
      LaunchTimer tm(p, MF_KERNEL_SOLVE, st);
      hipLaunchKernelGGL(bwd_colA_kernel, dim3((unsigned)p->n_cols), dim3(kBlock), 0, st, ca);
    }
    {
      LaunchTimer tm(p, MF_KERNEL_PASS_VEC, st);
      hipLaunchKernelGGL(bwd_passB_kernel, dim3((unsigned)p->n_items), dim3(kSBlock), lds, st, ba);
    }
    {
      LaunchTimer tm(p, MF_KERNEL_SOLVE, st);
      hipLaunchKernelGGL(bwd_colB_kernel, dim3((unsigned)p->n_cols), dim3(128), 0, st, ca);
    }
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
  {
    LaunchTimer tm(p, MF_KERNEL_PASS_LAST, st);
    hipLaunchKernelGGL(bwd_assemble_kernel, dim3((unsigned)p->n_items), dim3(256), asm_lds_bytes(B, K),
                       st, aa);
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
  if (p->cols_d) (void)hipFree(p->cols_d);
  if (p->items_d) (void)hipFree(p->items_d);
  if (p->order_d) (void)hipFree(p->order_d);
  delete p;
}

}  // extern "C"

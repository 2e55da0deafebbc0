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

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mf.h"

namespace {

constexpr int kBlock = 256;      // 4 waves of 64
constexpr int kPad = 80;         // bands of the per-column state (5 x 16)
constexpr int kMaxTri = 80 * 81 / 2;
constexpr int kDefaultChunk = 2048;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// What a pass accumulates besides alpha.
enum PassMode {
  PM_NONE = 0,   // last pass: alpha only
  PM_VEC = 1,    // m = sum c (L - mean L), S1, S2 in FP64 (low-rank form)
  PM_F64 = 2,    // Gram of [y, 1, c] on v_mfma_f64_16x16x4_f64 (exact)
  PM_F32 = 3,    // Gram on v_mfma_f32_16x16x4_f32, FP64 flush every 64 px
  PM_BF16 = 4    // Gram on v_mfma_f32_16x16x32_bf16, FP64 flush every 256 px
};
constexpr int kVecM = 80, kVecS1 = 80, kVecS2 = 81;   // PM_VEC partial layout

struct ColInfo {
  int64_t first_px;
  int32_t n_lines;
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
  int B;
  int j;
  int albedo;
  int unclamped;             // K == 0: return alpha^0 without the clamp
  double lam;
  double eps;
  int partial_stride;        // doubles per work item in the partial buffer
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
  int partial_stride;        // doubles per work item in the partial buffer
};

__host__ __device__ constexpr int n_tiles(int nb) { return nb * (nb + 1) / 2; }
__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }  // j <= i

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(
      0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

// Sum over the 16 lanes of a DPP row (one pixel per row in the pass layout).
__device__ __forceinline__ float row_sum16(float x) {
  x += dpp<0xB1>(x);    // quad_perm [1,0,3,2]
  x += dpp<0x4E>(x);    // quad_perm [2,3,0,1]
  x += dpp<0x124>(x);   // row_ror:4
  x += dpp<0x128>(x);   // row_ror:8
  return x;
}

// ---------------------------------------------------------------------------
// setup: per column, the shift point z (first valid pixel) and a clean state.

__global__ void __launch_bounds__(64) setup_kernel(const float* __restrict__ L,
                                                   const uint8_t* __restrict__ valid,
                                                   const ColInfo* __restrict__ cols,
                                                   ColState* __restrict__ state, int B) {
  const int col = blockIdx.x;
  const int lane = threadIdx.x;
  const ColInfo ci = cols[col];
  int64_t z = -1;
  if (valid == nullptr) {
    z = ci.n_lines > 0 ? ci.first_px : -1;
  } else {
    for (int64_t l0 = 0; l0 < ci.n_lines; l0 += 64) {
      const bool v = (l0 + lane < ci.n_lines) && valid[ci.first_px + l0 + lane] != 0;
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
// as unpacked FP32 on CDNA.

template <int NB, bool WIDE>
__host__ __device__ constexpr int band_of(int k, int c) {
  return WIDE ? (k < 4 ? 4 * c + k : 64 + c) : c + 16 * k;
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

template <int NB, bool WIDE, int S8>
__device__ __forceinline__ void load_super(const PassArgs& a, int64_t base, int64_t end,
                                           int row, int c16, float (&Lv)[S8][NB],
                                           double (&ap)[S8], unsigned& okmask) {
  static_assert(S8 == 8, "a super-step is 8 sub-steps");
  okmask = 0;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int64_t px = base + 4 * s + row;
    const bool inb = px < end;
    const float* pl = a.L + px * a.B;
    if constexpr (WIDE) {
      float4 v4 = float4{0.f, 0.f, 0.f, 0.f};
      if (inb) v4 = *reinterpret_cast<const float4*>(pl + 4 * c16);   // 4-byte aligned rows
      Lv[s][0] = v4.x;
      Lv[s][1] = v4.y;
      Lv[s][2] = v4.z;
      Lv[s][3] = v4.w;
      Lv[s][4] = (inb && 64 + c16 < a.B) ? pl[64 + c16] : 0.f;
    } else {
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const int b = band_of<NB, WIDE>(k, c16);
        Lv[s][k] = (inb && b < a.B) ? pl[b] : 0.f;
      }
    }
    ap[s] = (inb && a.alpha_prev) ? a.alpha_prev[px] : 0.0;
    bool ok = inb;
    if (inb && a.valid) ok = a.valid[px] != 0;
    okmask |= (ok ? 1u : 0u) << s;
  }
}

template <int NB, bool WIDE, int MODE>
__global__ void __launch_bounds__(kBlock, 1) pass_kernel(PassArgs a) {
  constexpr int T = n_tiles(NB);
  constexpr bool GRAM = MODE >= PM_F64;
  constexpr bool F32ACC = MODE == PM_F32 || MODE == PM_BF16;
  constexpr int FLUSH = MODE == PM_BF16 ? 8 : 2;   // super-steps between FP64 flushes
  const WorkItem it = a.items[blockIdx.x];
  const ColState& st = a.state[it.col];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
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

  double mu[NB], vv[NB], tt[NB], m0[NB], lb[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int b = band_of<NB, WIDE>(k, c16);
    const bool in = b < B;
    mu[k] = in ? st.mu[b] : 0.0;
    vv[k] = in ? st.v[b] : 0.0;
    tt[k] = in ? st.t[b] : 0.0;
    m0[k] = in ? st.m0[b] : 0.0;
    lb[k] = in ? st.lbar[b] : 0.0;
  }
  const double q = st.q;
  const double lam = a.lam, eps = a.eps;
  const int j = a.j;

  [[maybe_unused]] floatx4 acc[F32ACC ? T : 1];
  [[maybe_unused]] doublex4 dacc[GRAM ? T : 1];
  [[maybe_unused]] double md[NB], s1d = 0.0, s2d = 0.0;
  if constexpr (GRAM) {
#pragma unroll
    for (int t = 0; t < T; ++t) dacc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
  }
  if constexpr (F32ACC) {
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  }
  if constexpr (MODE == PM_VEC) {
#pragma unroll
    for (int k = 0; k < NB; ++k) md[k] = 0.0;
  }

  // The MFMA-bound Gram passes run one wave per SIMD and prefetch the next
  // super-step explicitly; the streaming passes keep fewer registers and
  // hide latency with more waves instead.
  constexpr bool PREFETCH = GRAM;
  float Lc[8][NB];
  double apc[8];
  unsigned okc = 0;
  int64_t base = begin + 32 * wid;
  if (PREFETCH && base < end) load_super<NB, WIDE, 8>(a, base, end, row, c16, Lc, apc, okc);
  int nsuper = 0;

  for (; base < end; base += 128) {
    [[maybe_unused]] float Ln[PREFETCH ? 8 : 1][NB];
    [[maybe_unused]] double apn[PREFETCH ? 8 : 1];
    [[maybe_unused]] unsigned okn = 0;
    if constexpr (PREFETCH) {
      if (base + 128 < end) load_super<NB, WIDE, 8>(a, base + 128, end, row, c16, Ln, apn, okn);
    } else {
      load_super<NB, WIDE, 8>(a, base, end, row, c16, Lc, apc, okc);
    }

    [[maybe_unused]] bf16x8 ybf[NB];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int64_t px = base + 4 * s + row;
      const bool ok = (okc >> s) & 1u;
      double x[NB], l[NB];
      double pp = 0.0, rr = 0.0;
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        const bool in = ok && band_of<NB, WIDE>(k, c16) < B;
        l[k] = in ? (double)Lc[s][k] : 0.0;
        x[k] = in ? l[k] - mu[k] : 0.0;
        pp = fma(x[k], vv[k], pp);
        rr = fma(l[k], m0[k], rr);
      }
      pp = row_sum16_f64(pp);
      rr = row_sum16_f64(rr);
      double c = 0.0;
      if (j >= 1) {
        const double r = a.albedo ? rr : 1.0;
        const double num = (j == 1) ? pp : pp - lam / (apc[s] + eps);
        double al = num / (r * q);
        const bool dark = !(r > 0.0);
        if (!a.unclamped) al = al > 0.0 ? al : 0.0;
        if (!ok || dark) al = 0.0;
        if (c16 == 0 && px < end) {
          if (a.alpha_out) a.alpha_out[px] = al;
          if (a.alpha_final) a.alpha_final[px] = (float)al;
        }
        c = (ok && !dark && al > 0.0) ? r * al : 0.0;
      }
      if constexpr (MODE == PM_VEC) {
#pragma unroll
        for (int k = 0; k < NB; ++k)
          md[k] = fma(c, l[k] - lb[k], md[k]);   // c = 0 off valid pixels
        s1d += c;
        s2d = fma(c, c, s2d);
      }
      if constexpr (GRAM) {
        double y[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          const int b = band_of<NB, WIDE>(k, c16);
          y[k] = fma(-c, tt[k], x[k]);
          if (b == B) y[k] = ok ? 1.0 : 0.0;
          if (b == B + 1) y[k] = c;
        }
        if constexpr (MODE == PM_F64) {
#pragma unroll
          for (int I = 0; I < NB; ++I)
#pragma unroll
            for (int J = 0; J <= I; ++J)
              dacc[n_tiles(I) + J] =
                  __builtin_amdgcn_mfma_f64_16x16x4f64(y[I], y[J], dacc[n_tiles(I) + J], 0, 0, 0);
        } else if constexpr (MODE == PM_F32) {
          float yf[NB];
#pragma unroll
          for (int k = 0; k < NB; ++k) yf[k] = (float)y[k];
#pragma unroll
          for (int I = 0; I < NB; ++I)
#pragma unroll
            for (int J = 0; J <= I; ++J)
              acc[n_tiles(I) + J] =
                  __builtin_amdgcn_mfma_f32_16x16x4f32(yf[I], yf[J], acc[n_tiles(I) + J], 0, 0, 0);
        } else {
#pragma unroll
          for (int k = 0; k < NB; ++k) ybf[k][s] = (__bf16)(float)y[k];
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
    if constexpr (F32ACC) {
      if (++nsuper == FLUSH) {
        nsuper = 0;
#pragma unroll
        for (int t = 0; t < T; ++t) {
#pragma unroll
          for (int i = 0; i < 4; ++i) dacc[t][i] += (double)acc[t][i];
          acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
      }
    }
    if constexpr (PREFETCH) {
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        apc[s] = apn[s];
#pragma unroll
        for (int k = 0; k < NB; ++k) Lc[s][k] = Ln[s][k];
      }
      okc = okn;
    }
  }

  double* out = a.partials + (int64_t)blockIdx.x * (T * 256);
  if constexpr (GRAM) {
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
  } else if constexpr (MODE == PM_VEC) {
    // 16 (wave, row) partials per band, summed in a fixed order.
    __shared__ double redv[16 * 82];
    const int slot = (wid * 4 + row) * 82;
    for (int b = c16; b < kVecM; b += 16) redv[slot + b] = 0.0;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int b = band_of<NB, WIDE>(k, c16);
      if (b < B) redv[slot + b] = md[k];
    }
    if (c16 == 0) {           // every lane of a row holds the same c
      redv[slot + kVecS1] = s1d;
      redv[slot + kVecS2] = s2d;
    }
    __syncthreads();
    for (int e = tid; e < 82; e += kBlock) {
      double sum = 0.0;
      for (int w = 0; w < 16; ++w) sum += redv[w * 82 + e];
      out[e] = sum;
    }
  }
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

constexpr int kChunk = 64;                 // pixels per wave chunk
constexpr int kSW = 2;                     // waves per stream workgroup
constexpr int kSBlock = 64 * kSW;
constexpr int kCopyGroup = 10;             // 16-byte loads in flight per lane while copying

// Dynamic LDS bytes of stream_kernel for B bands (about 42 KB at 74 bands).
__host__ __device__ constexpr size_t stream_lds_bytes(int B) {
  return (size_t)kSW * kChunk * B * sizeof(float) + kSW * kChunk * sizeof(double) +
         kSW * (kPad + 2) * sizeof(double) + 4 * kPad * sizeof(double);
}

template <int MODE>
__global__ void __launch_bounds__(kSBlock) stream_kernel(PassArgs a) {
  const WorkItem it = a.items[blockIdx.x];
  const ColState* __restrict__ st = a.state + it.col;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int B = a.B;
  const int64_t begin = it.px_begin, end = begin + it.n_px;
  extern __shared__ double dyn[];
  double* cbuf = dyn;                                   // [kSW][kChunk]
  double* redm = cbuf + kSW * kChunk;                   // [kSW][kPad + 2]
  double* cst = redm + kSW * (kPad + 2);                // [kPad][4]: mu, v, m0, lbar
  float* my = reinterpret_cast<float*>(cst + 4 * kPad) + wid * kChunk * B;   // [kChunk][B]

  if (st->status != MF_COL_OK) {           // failed column: alpha = 0, no moments
    for (int64_t px = begin + tid; px < end; px += kSBlock) {
      if (a.alpha_out) a.alpha_out[px] = 0.0;
      if (a.alpha_final) a.alpha_final[px] = 0.f;
    }
    return;
  }
  for (int b = tid; b < kPad; b += kSBlock) {
    cst[4 * b + 0] = st->mu[b];
    cst[4 * b + 1] = st->v[b];
    cst[4 * b + 2] = st->m0[b];
    cst[4 * b + 3] = st->lbar[b];
  }
  __syncthreads();
  const double q = st->q;
  const double lam = a.lam, eps = a.eps;
  const int j = a.j;
  const uintptr_t lp = reinterpret_cast<uintptr_t>(a.L);

  [[maybe_unused]] double m_lo = 0.0, m_hi = 0.0, s1 = 0.0, s2 = 0.0;

  // Whole chunks whose bytes start on a 16-byte boundary are streamed with
  // 16-byte loads, one chunk ahead in registers; other chunks are copied
  // synchronously with 8- or 4-byte loads (never past the chunk).
  constexpr int kF4 = (kChunk * 78 / 4 + 63) / 64;     // float4 per lane per chunk (20)
  float4 pre[kF4];
  auto fast = [&](int64_t c) {          // a whole, 16-byte aligned chunk
    return c + kChunk <= end && ((lp + (uintptr_t)(c * B) * 4) & 15) == 0;
  };
  auto prefetch = [&](int64_t c) {
    const float4* g4 = reinterpret_cast<const float4*>(a.L + c * B);
    const int n4 = kChunk * B / 4;
#pragma unroll
    for (int k = 0; k < kF4; ++k) {
      const int e = lane + 64 * k;
      pre[k] = e < n4 ? g4[e] : float4{0.f, 0.f, 0.f, 0.f};
    }
  };
  int64_t c0 = begin + (int64_t)kChunk * wid;
  bool have = c0 < end && fast(c0);
  if (have) prefetch(c0);

  for (; c0 < end; c0 += kSW * kChunk) {
    const int n = (int)min<int64_t>(kChunk, end - c0);
    const int nfl = n * B;
    const float* g = a.L + c0 * B;
    if (have) {
      float4* t4 = reinterpret_cast<float4*>(my);
      const int n4 = kChunk * B / 4;
#pragma unroll
      for (int k = 0; k < kF4; ++k) {
        const int e = lane + 64 * k;
        if (e < n4) t4[e] = pre[k];
      }
    } else {
      const uintptr_t ga = lp + (uintptr_t)(c0 * B) * 4;
      if ((ga & 7) == 0 && (nfl & 1) == 0) {
        const float2* g2 = reinterpret_cast<const float2*>(g);
        float2* t2 = reinterpret_cast<float2*>(my);
        const int n2 = nfl / 2;
        for (int base = 0; base < n2; base += 64 * kCopyGroup) {
          float2 r[kCopyGroup];
#pragma unroll
          for (int k = 0; k < kCopyGroup; ++k) {
            const int e = base + lane + 64 * k;
            r[k] = e < n2 ? g2[e] : float2{0.f, 0.f};
          }
#pragma unroll
          for (int k = 0; k < kCopyGroup; ++k) {
            const int e = base + lane + 64 * k;
            if (e < n2) t2[e] = r[k];
          }
        }
      } else {
        for (int e = lane; e < nfl; e += 64) my[e] = g[e];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    {
      const int64_t nx = c0 + kSW * kChunk;
      have = nx < end && fast(nx);
      if (have) prefetch(nx);                 // in flight while this chunk is scored
    }

    // score this lane's pixel
    const int64_t px = c0 + lane;
    const bool inb = lane < n;
    bool ok = inb;
    if (inb && a.valid) ok = a.valid[px] != 0;
    const double ap = (inb && a.alpha_prev) ? a.alpha_prev[px] : 0.0;
    double pp = 0.0, rr = 0.0;
    if (ok) {
      const float* rowp = my + lane * B;
      int b = 0;
      if ((B & 1) == 0) {                     // pairs of bands: 8-byte tile reads
#pragma unroll 4
        for (; b < B; b += 2) {
          const float2 l2 = *reinterpret_cast<const float2*>(rowp + b);
          const double4 c0v = *reinterpret_cast<const double4*>(cst + 4 * b);
          const double4 c1v = *reinterpret_cast<const double4*>(cst + 4 * b + 4);
          const double l0 = (double)l2.x, l1 = (double)l2.y;
          pp = fma(l0 - c0v.x, c0v.y, pp);
          rr = fma(l0, c0v.z, rr);
          pp = fma(l1 - c1v.x, c1v.y, pp);
          rr = fma(l1, c1v.z, rr);
        }
      }
      for (; b < B; ++b) {
        const double l = (double)rowp[b];
        pp = fma(l - cst[4 * b], cst[4 * b + 1], pp);
        rr = fma(l, cst[4 * b + 2], rr);
      }
    }
    double c = 0.0;
    if (j >= 1) {
      const double r = a.albedo ? rr : 1.0;
      const double num = (j == 1) ? pp : pp - lam / (ap + eps);
      double al = num / (r * q);
      const bool dark = !(r > 0.0);
      if (!a.unclamped) al = al > 0.0 ? al : 0.0;
      if (!ok || dark) al = 0.0;
      if (inb) {
        if (a.alpha_out) a.alpha_out[px] = al;
        if (a.alpha_final) a.alpha_final[px] = (float)al;
      }
      c = (ok && !dark && al > 0.0) ? r * al : 0.0;
    }
    if constexpr (MODE == PM_VEC) {
      s1 += c;
      s2 = fma(c, c, s2);
      if (__ballot(c != 0.0)) {                 // wave-uniform
        cbuf[wid * kChunk + lane] = c;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int b0 = lane, b1 = lane + 64;
        const double lb0 = b0 < B ? cst[4 * b0 + 3] : 0.0;
        const double lb1 = b1 < B ? cst[4 * b1 + 3] : 0.0;
        for (int p = 0; p < n; ++p) {
          const double cp = cbuf[wid * kChunk + p];
          if (cp != 0.0) {                      // wave-uniform; skips invalid pixels too
            if (b0 < B) m_lo = fma(cp, (double)my[p * B + b0] - lb0, m_lo);
            if (b1 < B) m_hi = fma(cp, (double)my[p * B + b1] - lb1, m_hi);
          }
        }
      }
    }
    // the tile is rewritten by this wave only after every lane is done with it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }

  if constexpr (MODE == PM_VEC) {
    for (int off = 32; off >= 1; off >>= 1) {
      s1 += __shfl_xor(s1, off, 64);
      s2 += __shfl_xor(s2, off, 64);
    }
    double* rw = redm + wid * (kPad + 2);
    if (lane < kPad) rw[lane] = lane < B ? m_lo : 0.0;
    if (lane + 64 < kPad) rw[lane + 64] = lane + 64 < B ? m_hi : 0.0;
    if (lane == 0) {
      rw[kVecS1] = s1;
      rw[kVecS2] = s2;
    }
    __syncthreads();
    double* out = a.partials + (int64_t)blockIdx.x * a.partial_stride;
    for (int e = tid; e < kPad + 2; e += kSBlock) {
      double sum = 0.0;
      for (int w = 0; w < kSW; ++w) sum += redm[w * (kPad + 2) + e];
      out[e] = sum;
    }
  }
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

// G[i][j] summed over the column's work items (tiles hold block I >= J).
template <int NB, bool WIDE>
__device__ __forceinline__ double gram_elem(const double* __restrict__ P, int n_items,
                                            int i, int j) {
  constexpr int T = n_tiles(NB);
  int I, mi, J, mj;
  block_of<NB, WIDE>(i, I, mi);
  block_of<NB, WIDE>(j, J, mj);
  if (I < J) {
    const int t0 = I, t1 = mi;
    I = J; mi = mj; J = t0; mj = t1;
  }
  const int e = (n_tiles(I) + J) * 256 + mi * 16 + mj;
  double g = 0.0;
  for (int it = 0; it < n_items; ++it) g += P[(int64_t)it * T * 256 + e];
  return g;
}

__device__ __forceinline__ double readlane_f64(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// Wave-synchronous solve of L L^T v = y on one wave (64 lanes); the factor
// is packed lower-triangular in LDS with inverse diagonal invd; the vector
// lives in registers, lane l holding entries l and l + 64.
__device__ void wave_chol_solve(const double* __restrict__ Lf, double invd_lo, double invd_hi,
                                double& y_lo, double& y_hi, int B, int lane) {
  const int i0 = lane, i1 = lane + 64;
  for (int k = 0; k < B; ++k) {                     // forward: L y' = y
    const bool lo = k < 64;
    const double yk = readlane_f64(lo ? y_lo : y_hi, k & 63) *
                      readlane_f64(lo ? invd_lo : invd_hi, k & 63);
    if (i0 == k) y_lo = yk;
    if (i1 == k) y_hi = yk;
    if (i0 > k && i0 < B) y_lo -= Lf[tri(i0, k)] * yk;
    if (i1 > k && i1 < B) y_hi -= Lf[tri(i1, k)] * yk;
  }
  for (int k = B - 1; k >= 0; --k) {                // backward: L^T v = y'
    const bool lo = k < 64;
    const double vk = readlane_f64(lo ? y_lo : y_hi, k & 63) *
                      readlane_f64(lo ? invd_lo : invd_hi, k & 63);
    if (i0 == k) y_lo = vk;
    if (i1 == k) y_hi = vk;
    if (i0 < k) y_lo -= Lf[tri(k, i0)] * vk;
    if (i1 < k) y_hi -= Lf[tri(k, i1)] * vk;
  }
}

// One workgroup per column.  The symmetric matrix is split in 4x4 blocks of
// the lower triangle; thread t < 210 keeps block (bi, bj), t = bi(bi+1)/2 + bj,
// in registers through assembly and a right-looking Cholesky (two barriers
// per column of the factor).
constexpr int kBlk = 4;
constexpr int kNBlkRows = kPad / kBlk;                            // 20
constexpr int kNBlk = kNBlkRows * (kNBlkRows + 1) / 2;            // 210

// Dot product of two LDS vectors (length B) on one wave; every lane gets it.
__device__ __forceinline__ double wave_dot(const double* x, const double* y, int B, int lane) {
  double s = 0.0;
  for (int i = lane; i < B; i += 64) s += x[i] * y[i];
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
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
// so are b_r[i >= B].  Vectors are LDS arrays of stride kPad; prow/pcol are
// LDS scratch of R * kNBlk * kBlk doubles each.  Each row sums its blocks in
// a fixed order (deterministic).  Contains two barriers.
template <int R>
__device__ void block_symv(const double (&M)[kBlk][kBlk], bool owner, int bi, int bj, int tid,
                           int B, const double* bv, double* yv, double* prow, double* pcol) {
  if (owner) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double* b = bv + r * kPad;
#pragma unroll
      for (int x = 0; x < kBlk; ++x) {
        double s = 0.0;
#pragma unroll
        for (int y = 0; y < kBlk; ++y) s += M[x][y] * b[kBlk * bj + y];
        prow[(r * kNBlk + tid) * kBlk + x] = s;
      }
#pragma unroll
      for (int y = 0; y < kBlk; ++y) {
        double s = 0.0;
#pragma unroll
        for (int x = 0; x < kBlk; ++x)
          if (kBlk * bi + x > kBlk * bj + y) s += M[x][y] * b[kBlk * bi + x];
        pcol[(r * kNBlk + tid) * kBlk + y] = s;
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < R * kPad; idx += kBlock) {
    const int r = idx / kPad, i = idx - r * kPad;
    if (i >= B) {
      yv[r * kPad + i] = 0.0;
      continue;
    }
    const int ib = i / kBlk, ix = i % kBlk;
    double acc = 0.0;
    for (int c = 0; c <= ib; ++c) acc += prow[(r * kNBlk + ib * (ib + 1) / 2 + c) * kBlk + ix];
    for (int rr = ib; rr < kNBlkRows; ++rr)
      acc += pcol[(r * kNBlk + rr * (rr + 1) / 2 + ib) * kBlk + ix];
    yv[r * kPad + i] = acc;
  }
  __syncthreads();
}

template <int NB, bool WIDE>
__global__ void __launch_bounds__(kBlock) solve_kernel(SolveArgs a) {
  const int col = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  ColState& st = a.state[col];
  if (st.status != MF_COL_OK) return;
  const ColInfo ci = a.cols[col];
  const int B = a.B;
  const int j = a.j;
  constexpr int T = n_tiles(NB);
  const double* P = a.partials + (int64_t)ci.first_item * T * 256;
  const bool rank3 = a.lowrank && j >= 1;
  double* c0 = a.c0 + (int64_t)col * (kNBlk * 16);
  double* pinv = a.pinv + (int64_t)col * (kNBlk * 16);

  __shared__ double Lf[kMaxTri];     // the factor, packed lower triangle
  __shared__ double g1[kPad], g2[kPad], D[kPad], E[kPad], tn[kPad], mun[kPad];
  __shared__ double colk[kPad], vbuf[kPad], rbuf[kPad], invd[kPad];
  __shared__ double prow[kNBlk * kBlk], pcol[kNBlk * kBlk];
  __shared__ double sc[4];
  __shared__ double sdiag;
  __shared__ int fail;

  // block owned by this thread
  int bi = 0, bj = 0;
  const bool owner = tid < kNBlk;
  if (owner) block_coords(tid, bi, bj);

  if (tid == 0) {
    if (rank3) {
      double s1 = 0.0, s2 = 0.0;
      for (int it = 0; it < ci.n_items; ++it) {
        s1 += P[(int64_t)it * T * 256 + kVecS1];
        s2 += P[(int64_t)it * T * 256 + kVecS2];
      }
      sc[0] = st.n_valid;
      sc[1] = s1;
      sc[2] = s2;
    } else {
      sc[0] = gram_elem<NB, WIDE>(P, ci.n_items, B, B);          // N
      sc[1] = gram_elem<NB, WIDE>(P, ci.n_items, B + 1, B);      // S1 = sum c
      sc[2] = gram_elem<NB, WIDE>(P, ci.n_items, B + 1, B + 1);  // S2 = sum c^2
    }
    fail = 0;
  }
  for (int b = tid; b < B; b += kBlock) {
    if (rank3) {
      double m = 0.0;
      for (int it = 0; it < ci.n_items; ++it) m += P[(int64_t)it * T * 256 + b];
      g1[b] = m;
      g2[b] = 0.0;
    } else {
      g1[b] = gram_elem<NB, WIDE>(P, ci.n_items, B, b);
      g2[b] = gram_elem<NB, WIDE>(P, ci.n_items, B + 1, b);
    }
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
      m = st.lbar[b] - (S1 / N) * st.t[b];     // Eq. 10: mean(L) - mean(c) t^{j-1}
    }
    mun[b] = m;
    tn[b] = m * sb;                            // Eq. 9
    if (rank3) {
      D[b] = st.t[b] - tn[b];                  // t^{j-1} - t^j
      E[b] = 0.0;
    } else {
      D[b] = mu_used - m;
      E[b] = j == 0 ? 0.0 : t_used - tn[b];
    }
  }
  __syncthreads();

  // ---- assembly of C (Eq. 11) into the register blocks
  double A_[kBlk][kBlk], C_[kBlk][kBlk];
  const double abar = S1 / N;
  int myfail = 0;
#pragma unroll
  for (int x = 0; x < kBlk; ++x)
#pragma unroll
    for (int y = 0; y < kBlk; ++y) {
      const int i = kBlk * bi + x, jj = kBlk * bj + y;
      double c = (i == jj) ? 1.0 : 0.0;        // padding keeps the factor regular
      if (owner && i < B && jj < B && i >= jj) {
        if (rank3) {
          c = c0[tid * 16 + x * kBlk + y] + abar * abar * D[i] * D[jj] +
              (S2 / N - abar * abar) * tn[i] * tn[jj] - (g1[i] * tn[jj] + tn[i] * g1[jj]) / N;
        } else {
          c = gram_elem<NB, WIDE>(P, ci.n_items, i, jj);
          c += g1[i] * D[jj] + D[i] * g1[jj] + g2[i] * E[jj] + E[i] * g2[jj] +
               N * D[i] * D[jj] + S1 * (D[i] * E[jj] + E[i] * D[jj]) + S2 * E[i] * E[jj];
          c /= N;
        }
        if (!isfinite(c)) myfail = 1;
      } else if (owner && i < B && jj < B) {
        c = 0.0;                               // upper half of a diagonal block: unused
      }
      A_[x][y] = c;
      C_[x][y] = c;
    }
  if (owner && a.lowrank && j == 0) {
#pragma unroll
    for (int x = 0; x < kBlk; ++x)
#pragma unroll
      for (int y = 0; y < kBlk; ++y) c0[tid * 16 + x * kBlk + y] = A_[x][y];
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
    // ---- low-rank form, pass 0: invert C^0 by symmetric sweeps on the
    // register blocks (A <- -A^-1 after all pivots) and keep C^0 and its
    // inverse for the rank-3 solves of later iterations.
    for (int k = 0; k < B; ++k) {
      const int kb = k >> 2, ka = k & 3;
      if (owner && bi == kb && bj == kb) {
        double dkk = 0.0;
#pragma unroll
        for (int x = 0; x < kBlk; ++x)
          if (x == ka) dkk = A_[x][x];
        sdiag = dkk;
      }
      __syncthreads();
      const double d = sdiag;
      if (!(d > 0.0) || !isfinite(d)) {      // uniform
        if (tid == 0) st.status = MF_COL_NOT_SPD;
        return;
      }
      if (owner) {                           // publish row/column k
#pragma unroll
        for (int x = 0; x < kBlk; ++x)
#pragma unroll
          for (int y = 0; y < kBlk; ++y) {
            const int i = kBlk * bi + x, jj = kBlk * bj + y;
            if (jj == k && i > k && i < B) colk[i] = A_[x][y];
            if (i == k && jj < k) colk[jj] = A_[x][y];
          }
      }
      __syncthreads();
      const double inv = 1.0 / d;
      if (owner) {
#pragma unroll
        for (int x = 0; x < kBlk; ++x)
#pragma unroll
          for (int y = 0; y < kBlk; ++y) {
            const int i = kBlk * bi + x, jj = kBlk * bj + y;
            if (i >= B || jj > i) continue;
            if (i == k && jj == k) A_[x][y] = -inv;
            else if (jj == k) A_[x][y] = colk[i] * inv;
            else if (i == k) A_[x][y] = colk[jj] * inv;
            else A_[x][y] -= colk[i] * colk[jj] * inv;
          }
      }
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
        for (int y = 0; y < kBlk; ++y) pinv[tid * 16 + x * kBlk + y] = A_[x][y];
    }
    for (int b = tid; b < kPad; b += kBlock) rbuf[b] = b < B ? tn[b] : 0.0;
    __syncthreads();
    block_symv<1>(A_, owner, bi, bj, tid, B, rbuf, vbuf, prow, pcol);   // v = P t
    for (int step = 0; step < a.refine; ++step) {
      block_symv<1>(C_, owner, bi, bj, tid, B, vbuf, colk, prow, pcol);  // C v
      for (int b = tid; b < kPad; b += kBlock) rbuf[b] = b < B ? tn[b] - colk[b] : 0.0;
      __syncthreads();
      block_symv<1>(A_, owner, bi, bj, tid, B, rbuf, colk, prow, pcol);  // P r
      for (int b = tid; b < B; b += kBlock) vbuf[b] += colk[b];
      __syncthreads();
    }
  } else {
  // ---- right-looking Cholesky on the register blocks
  for (int k = 0; k < B; ++k) {
    const int kb = k >> 2, ka = k & 3;
    if (owner && bi == kb && bj == kb) {
      double dkk = 0.0;
#pragma unroll
      for (int x = 0; x < kBlk; ++x)
        if (x == ka) dkk = A_[x][x];
      sdiag = dkk;
    }
    __syncthreads();
    const double dkk = sdiag;
    if (!(dkk > 0.0) || !isfinite(dkk)) {      // uniform
      if (tid == 0) st.status = MF_COL_NOT_SPD;
      return;
    }
    const double d = sqrt(dkk);
    if (owner && bj == kb) {
      const double inv = 1.0 / d;
#pragma unroll
      for (int x = 0; x < kBlk; ++x) {
        const int i = kBlk * bi + x;
#pragma unroll
        for (int y = 0; y < kBlk; ++y) {
          if (y != ka) continue;
          if (i == k) A_[x][y] = d;
          if (i > k) {
            A_[x][y] *= inv;
            colk[i] = A_[x][y];
          }
        }
      }
    }
    __syncthreads();
    if (owner && kBlk * bi + 3 > k) {
      double cI[kBlk], cJ[kBlk];
#pragma unroll
      for (int x = 0; x < kBlk; ++x) {
        cI[x] = colk[kBlk * bi + x];
        cJ[x] = colk[kBlk * bj + x];
      }
#pragma unroll
      for (int x = 0; x < kBlk; ++x)
#pragma unroll
        for (int y = 0; y < kBlk; ++y) {
          const int i = kBlk * bi + x, jj = kBlk * bj + y;
          if (jj > k && i >= jj && i < B) A_[x][y] -= cI[x] * cJ[y];
        }
    }
  }
  // factor -> LDS, inverse diagonal
  if (owner) {
#pragma unroll
    for (int x = 0; x < kBlk; ++x)
#pragma unroll
      for (int y = 0; y < kBlk; ++y) {
        const int i = kBlk * bi + x, jj = kBlk * bj + y;
        if (i < B && jj <= i) {
          Lf[tri(i, jj)] = A_[x][y];
          if (i == jj) invd[i] = 1.0 / A_[x][y];
        }
      }
  }
  // residual matrix: zero outside the lower triangle of the first B rows
#pragma unroll
  for (int x = 0; x < kBlk; ++x)
#pragma unroll
    for (int y = 0; y < kBlk; ++y) {
      const int i = kBlk * bi + x, jj = kBlk * bj + y;
      if (!(owner && i < B && jj <= i)) C_[x][y] = 0.0;
    }
  for (int b = tid; b < kPad; b += kBlock) vbuf[b] = 0.0;
  __syncthreads();

  // ---- v = C^-1 t, then refinement against the assembled C
  double y_lo = 0.0, y_hi = 0.0, id_lo = 0.0, id_hi = 0.0;
  if (wid == 0) {
    y_lo = lane < B ? tn[lane] : 0.0;
    y_hi = lane + 64 < B ? tn[lane + 64] : 0.0;
    id_lo = lane < B ? invd[lane] : 0.0;
    id_hi = lane + 64 < B ? invd[lane + 64] : 0.0;
    wave_chol_solve(Lf, id_lo, id_hi, y_lo, y_hi, B, lane);
    if (lane < B) vbuf[lane] = y_lo;
    if (lane + 64 < B) vbuf[lane + 64] = y_hi;
  }
  __syncthreads();
  for (int step = 0; step < a.refine; ++step) {
    block_symv<1>(C_, owner, bi, bj, tid, B, vbuf, rbuf, prow, pcol);   // C v
    for (int b = tid; b < B; b += kBlock) rbuf[b] = tn[b] - rbuf[b];
    __syncthreads();
    if (wid == 0) {
      double r_lo = lane < B ? rbuf[lane] : 0.0;
      double r_hi = lane + 64 < B ? rbuf[lane + 64] : 0.0;
      wave_chol_solve(Lf, id_lo, id_hi, r_lo, r_hi, B, lane);
      if (lane < B) vbuf[lane] += r_lo;
      if (lane + 64 < B) vbuf[lane + 64] += r_hi;
    }
    __syncthreads();
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
}

// Low-rank form, iterations j >= 1: C^j = C^0 + U S U^T with U = [D, t, m],
//   D = t^{j-1} - t^j, S = [[a^2, 0, 0], [0, S2/N - a^2, -1/N], [0, -1/N, 0]],
// (the rank-3 identity), solved with the stored P = (C^0)^-1 by Woodbury:
//   C^-1 b = P b - X (I + S W)^-1 S U^T P b,  X = P U,  W = U^T X,
// followed by refinement steps against C^j applied exactly.  Everything is
// matrix-vector products on the register blocks: no sequential factorisation.
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
  const double* c0 = a.c0 + (int64_t)col * (kNBlk * 16);
  const double* pinv = a.pinv + (int64_t)col * (kNBlk * 16);

  __shared__ double U3[3 * kPad];   // D, t, m
  __shared__ double X3[3 * kPad];   // P D, P t, P m
  __shared__ double mun[kPad], vbuf[kPad], rbuf[kPad], wbuf[kPad], zbuf[kPad];
  __shared__ double prow[3 * kNBlk * kBlk], pcol[3 * kNBlk * kBlk];
  __shared__ double sc[4];
  __shared__ double G3[9], S3[9], Ginv[9];
  __shared__ int bad;

  int bi = 0, bj = 0;
  const bool owner = tid < kNBlk;
  if (owner) block_coords(tid, bi, bj);
  double Cb[kBlk][kBlk], Pb[kBlk][kBlk];
#pragma unroll
  for (int x = 0; x < kBlk; ++x)
#pragma unroll
    for (int y = 0; y < kBlk; ++y) {
      Cb[x][y] = owner ? c0[tid * 16 + x * kBlk + y] : 0.0;
      Pb[x][y] = owner ? pinv[tid * 16 + x * kBlk + y] : 0.0;
    }
  if (tid == 0) {
    double s1 = 0.0, s2 = 0.0;
    for (int it = 0; it < ci.n_items; ++it) {
      s1 += P[it * stride + kVecS1];
      s2 += P[it * stride + kVecS2];
    }
    sc[0] = st.n_valid;
    sc[1] = s1;
    sc[2] = s2;
    bad = 0;
  }
  __syncthreads();
  const double N = sc[0], S1 = sc[1], S2 = sc[2];
  const double abar = S1 / N;
  for (int b = tid; b < kPad; b += kBlock) {
    double m = 0.0, mu = 0.0, t = 0.0, d = 0.0;
    if (b < B) {
      for (int it = 0; it < ci.n_items; ++it) m += P[it * stride + b];
      mu = st.lbar[b] - abar * st.t[b];          // Eq. 10
      t = mu * (double)a.s[b];                   // Eq. 9
      d = st.t[b] - t;
    }
    mun[b] = mu;
    U3[b] = d;
    U3[kPad + b] = t;
    U3[2 * kPad + b] = m;
  }
  __syncthreads();
  block_symv<3>(Pb, owner, bi, bj, tid, B, U3, X3, prow, pcol);    // X = P U
  if (wid == 0) {
    // W = U^T X, S, and (I + S W)^-1 by Gauss-Jordan with partial pivoting
    double W[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) W[r * 3 + c] = wave_dot(U3 + r * kPad, X3 + c * kPad, B, lane);
    if (lane == 0) {
      const double S[9] = {abar * abar, 0.0, 0.0, 0.0, S2 / N - abar * abar, -1.0 / N,
                           0.0, -1.0 / N, 0.0};
      double M[9], I3[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double s = (r == c) ? 1.0 : 0.0;
          for (int k = 0; k < 3; ++k) s += S[r * 3 + k] * W[k * 3 + c];
          M[r * 3 + c] = s;
          I3[r * 3 + c] = (r == c) ? 1.0 : 0.0;
          S3[r * 3 + c] = S[r * 3 + c];
        }
      for (int k = 0; k < 3; ++k) {
        int piv = k;
        for (int r = k + 1; r < 3; ++r)
          if (fabs(M[r * 3 + k]) > fabs(M[piv * 3 + k])) piv = r;
        if (!(fabs(M[piv * 3 + k]) > 0.0)) bad = 1;
        for (int c = 0; c < 3; ++c) {
          double t0 = M[k * 3 + c]; M[k * 3 + c] = M[piv * 3 + c]; M[piv * 3 + c] = t0;
          t0 = I3[k * 3 + c]; I3[k * 3 + c] = I3[piv * 3 + c]; I3[piv * 3 + c] = t0;
        }
        const double inv = 1.0 / M[k * 3 + k];
        for (int c = 0; c < 3; ++c) {
          M[k * 3 + c] *= inv;
          I3[k * 3 + c] *= inv;
        }
        for (int r = 0; r < 3; ++r) {
          if (r == k) continue;
          const double f = M[r * 3 + k];
          for (int c = 0; c < 3; ++c) {
            M[r * 3 + c] -= f * M[k * 3 + c];
            I3[r * 3 + c] -= f * I3[k * 3 + c];
          }
        }
      }
      for (int e = 0; e < 9; ++e) Ginv[e] = I3[e];
      (void)G3;
    }
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) st.status = MF_COL_NOT_SPD;
    return;
  }
  // v = Woodbury(t): P t is X3[1]
  // correction coefficients z = (I + S W)^-1 S U^T y  with y = P b
  // (computed by wave 0, applied by all threads)
  for (int step = 0; step <= a.refine; ++step) {
    const double* y = step == 0 ? (X3 + kPad) : wbuf;     // P b
    if (wid == 0) {
      double u[3];
      for (int r = 0; r < 3; ++r) u[r] = wave_dot(U3 + r * kPad, y, B, lane);
      if (lane == 0) {
        double su[3], z[3];
        for (int r = 0; r < 3; ++r) su[r] = S3[r * 3] * u[0] + S3[r * 3 + 1] * u[1] + S3[r * 3 + 2] * u[2];
        for (int r = 0; r < 3; ++r) z[r] = Ginv[r * 3] * su[0] + Ginv[r * 3 + 1] * su[1] + Ginv[r * 3 + 2] * su[2];
        sc[3] = 0.0;
        zbuf[0] = z[0];
        zbuf[1] = z[1];
        zbuf[2] = z[2];
      }
    }
    __syncthreads();
    for (int b = tid; b < kPad; b += kBlock) {
      const double corr = b < B ? y[b] - (X3[b] * zbuf[0] + X3[kPad + b] * zbuf[1] +
                                          X3[2 * kPad + b] * zbuf[2]) : 0.0;
      if (step == 0) vbuf[b] = corr;
      else if (b < B) vbuf[b] += corr;
    }
    __syncthreads();
    if (step == a.refine) break;
    // residual r = t - C^j v with C^j v = C^0 v + U S U^T v
    block_symv<1>(Cb, owner, bi, bj, tid, B, vbuf, rbuf, prow, pcol);
    if (wid == 0) {
      double u[3];
      for (int r = 0; r < 3; ++r) u[r] = wave_dot(U3 + r * kPad, vbuf, B, lane);
      if (lane == 0)
        for (int r = 0; r < 3; ++r)
          zbuf[4 + r] = S3[r * 3] * u[0] + S3[r * 3 + 1] * u[1] + S3[r * 3 + 2] * u[2];
    }
    __syncthreads();
    for (int b = tid; b < kPad; b += kBlock)
      rbuf[b] = b < B ? U3[kPad + b] - rbuf[b] -
                            (U3[b] * zbuf[4] + U3[kPad + b] * zbuf[5] + U3[2 * kPad + b] * zbuf[6])
                      : 0.0;
    __syncthreads();
    block_symv<1>(Pb, owner, bi, bj, tid, B, rbuf, wbuf, prow, pcol);  // P r
  }
  if (wid == 0) {
    const double q = wave_dot(U3 + kPad, vbuf, B, lane);
    if (lane == 0) {
      st.q = q;
      if (!(q > 0.0) || !isfinite(q)) st.status = MF_COL_NOT_SPD;
    }
  }
  for (int b = tid; b < kPad; b += kBlock) {
    st.mu[b] = mun[b];
    st.t[b] = U3[kPad + b];
    st.v[b] = vbuf[b];
  }
}

// Plain streaming read: the achievable HBM read bandwidth for this access
// size, used as the measured ceiling next to the nominal 8 TB/s.
__global__ void __launch_bounds__(kBlock) stream_read_kernel(const float4* __restrict__ src,
                                                             int64_t n4, float* __restrict__ sink) {
  float acc = 0.f;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n4; i += 4 * stride) {
    float4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = (i + u * stride < n4) ? src[i + u * stride] : float4{0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += (v[u].x + v[u].y) + (v[u].z + v[u].w);
  }
  if (acc == 1.2345e-30f) sink[blockIdx.x] = acc;   // keeps the loads alive
}

__global__ void status_kernel(const ColState* __restrict__ state, int32_t* __restrict__ out,
                              int64_t n) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) out[c] = state[c].status;
}

// ---------------------------------------------------------------------------
// Host side

thread_local std::string g_last_error;

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
  size_t ws_bytes = 0;
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

template <int NB, bool WIDE>
void launch_pass_nb(const mf_plan_s* p, const PassArgs& a, int mode, hipStream_t s) {
  const dim3 g((unsigned)p->n_items), b(kBlock);
  switch (mode) {
    case PM_F64: hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_F64>), g, b, 0, s, a); break;
    case PM_F32: hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_F32>), g, b, 0, s, a); break;
    default: hipLaunchKernelGGL((pass_kernel<NB, WIDE, PM_BF16>), g, b, 0, s, a); break;
  }
}

void dispatch_pass(const mf_plan_s* p, const PassArgs& a, int mode, hipStream_t s) {
  if (mode == PM_NONE || mode == PM_VEC) {
    const dim3 g((unsigned)p->n_items), b(kSBlock);
    const size_t lds = stream_lds_bytes(a.B);
    if (mode == PM_NONE) hipLaunchKernelGGL(stream_kernel<PM_NONE>, g, b, lds, s, a);
    else hipLaunchKernelGGL(stream_kernel<PM_VEC>, g, b, lds, s, a);
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

// Pass mode of pass j for a covariance form.
int pass_mode(int cov, int j, int K) {
  if (j == K + 1) return PM_NONE;
  switch (cov) {
    case MF_COV_GRAM_FP32: return PM_F32;
    case MF_COV_GRAM_BF16: return PM_BF16;
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
  const int B = p->opt.n_bands;
  const int K = p->opt.n_iter;

  {
    LaunchTimer tm(p, MF_KERNEL_OTHER, st);
    hipLaunchKernelGGL(setup_kernel, dim3((unsigned)p->n_cols), dim3(64), 0, st, radiance, valid,
                       p->cols_d, state, B);
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
  pa.partial_stride = n_tiles(p->nb) * 256;
  SolveArgs sa{};
  sa.cols = p->cols_d;
  sa.state = state;
  sa.partials = partials;
  sa.c0 = (double*)(ws + p->off_c0);
  sa.pinv = (double*)(ws + p->off_pinv);
  sa.partial_stride = n_tiles(p->nb) * 256;
  sa.s = s;
  sa.B = B;
  sa.refine = p->opt.refine_steps;
  sa.lowrank = p->opt.cov == MF_COV_LOWRANK;
  for (int j = 0; j <= K + 1; ++j) {
    pa.j = j;
    pa.unclamped = (j == 1 && K == 0) ? 1 : 0;
    pa.alpha_prev = j >= 2 ? abuf[(j - 2) & 1] : nullptr;
    pa.alpha_out = (j >= 1 && j <= K) ? abuf[(j - 1) & 1] : nullptr;
    pa.alpha_final = j == K + 1 ? alpha : nullptr;
    const bool mom = j <= K;
    const int mode = pass_mode(p->opt.cov, j, K);
    {
      LaunchTimer tm(p, mode == PM_NONE ? MF_KERNEL_PASS_LAST
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
  o->refine_steps = 1;
  o->save_for_backward = 0;
  o->chunk_lines = 0;
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
  if (opt->refine_steps < 0 || opt->refine_steps > 4)
    return fail_with(MF_E_ARG, "refine_steps must be in [0, 4]");
  if (opt->save_for_backward != 0)
    return fail_with(MF_E_UNSUPPORTED, "save_for_backward is not available in ABI version 1");
  if (opt->chunk_lines < 0 || opt->chunk_lines % 128 != 0)
    return fail_with(MF_E_ARG, "chunk_lines must be a non-negative multiple of 128");
  if (n_fl < 1) return fail_with(MF_E_SHAPE, "need at least one flightline");

  const int chunk = opt->chunk_lines ? opt->chunk_lines : kDefaultChunk;
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
    for (int c = 0; c < F.n_columns; ++c) {
      ColInfo ci{};
      ci.first_px = F.first_px + (int64_t)c * F.n_lines;
      ci.n_lines = F.n_lines;
      ci.first_item = (int32_t)items.size();
      const int nit = (F.n_lines + chunk - 1) / chunk;
      // split evenly, in multiples of 128 pixels
      int per = (F.n_lines + nit - 1) / nit;
      per = (per + 127) / 128 * 128;
      int done = 0;
      for (int k = 0; k < nit && done < F.n_lines; ++k) {
        WorkItem w{};
        w.px_begin = ci.first_px + done;
        w.col = (int32_t)cols.size();
        w.n_px = std::min(per, F.n_lines - done);
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
  const size_t T = (size_t)n_tiles(p->nb);
  size_t off = 0;
  p->off_state = off;
  off = align256(off + (size_t)p->n_cols * sizeof(ColState));
  p->off_partials = off;
  off = align256(off + (size_t)p->n_items * T * 256 * sizeof(double));
  p->off_c0 = off;
  if (opt->cov == MF_COV_LOWRANK) off = align256(off + (size_t)p->n_cols * kNBlk * 16 * sizeof(double));
  p->off_pinv = off;
  if (opt->cov == MF_COV_LOWRANK) off = align256(off + (size_t)p->n_cols * kNBlk * 16 * sizeof(double));
  p->off_alpha0 = off;
  off = align256(off + (size_t)max_px * sizeof(double));
  p->off_alpha1 = off;
  off = align256(off + (size_t)max_px * sizeof(double));
  p->ws_bytes = off;
  *out = p;
  g_last_error.clear();
  return MF_OK;
}

size_t mf_workspace_bytes(mf_plan p) { return p ? p->ws_bytes : 0; }
int64_t mf_plan_columns(mf_plan p) { return p ? p->n_cols : 0; }
int64_t mf_plan_pixels(mf_plan p) { return p ? p->n_px : 0; }

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

mf_status mf_plan_set_graph(mf_plan p, int enable) {
  if (!p) return fail_with(MF_E_ARG, "plan is NULL");
  p->use_graph = enable != 0;
  return MF_OK;
}

mf_status mf_stream_read(const float* src, int64_t n, float* sink, int32_t n_blocks,
                         float* ms_out, void* stream) {
  if (!src || !sink || n < 4 || n % 4 != 0 || ((uintptr_t)src & 15) != 0 || n_blocks < 1)
    return fail_with(MF_E_ARG, "src/sink NULL, n not a positive multiple of 4, or src not 16-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms_out && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    return fail_with(MF_E_DEVICE, "event creation failed");
  if (ms_out) (void)hipEventRecord(e0, st);
  hipLaunchKernelGGL(stream_read_kernel, dim3((unsigned)n_blocks), dim3(kBlock), 0, st,
                     (const float4*)src, n / 4, sink);
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

mf_status mf_plan_set_timing(mf_plan p, int enable) {
  if (!p) return fail_with(MF_E_ARG, "plan is NULL");
  p->timing = enable != 0;
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
  delete p;
}

}  // extern "C"

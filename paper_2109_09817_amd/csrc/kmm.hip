// Fused, never-materialised kernel-matrix products for gfx950.
//
//   square:  W = K_hat V = s_f M(X, X) V + sigma^2 V,  M_ab = m(r_ab)
//   cross:   W = K(Z, X) V = s_f M(Z, X) V
//
// with r_ab^2 = sum_j ((x_aj - x_bj)/l_j)^2 and m the Matern-5/2 or RBF
// profile (the kernel of Sec. 4; K_hat of Sec. 2.2; the O(N^2) product that
// CG needs, Sec. 3.1, never stored, Sec. 3.2).
//
// One workgroup = 4 wave64s, each owning 16*NA output rows a.  A wave keeps
// the MFMA fragments of its rows in registers and sweeps the b stream in
// chunks of 32 points.  Per (16-row block, 32-point chunk):
//   1. S = XR_b . XC_a^T on the matrix cores gives r^2 directly: the operands
//      carry -2 x~_b against x~_a plus the two squared norms folded into the
//      K padding, so no VALU work builds the distance.
//   2. m(r) is evaluated in registers on the S accumulator (v_sqrt, v_exp,
//      two FMAs); the accumulator layout (lane = a, 4 consecutive b per lane
//      group) is already the A-operand layout of the next product once the
//      K index of that product is permuted to match, so nothing goes through
//      LDS.
//   3. acc += M . V_b on the matrix cores.
// FP32 accumulators are flushed to FP64 every FLUSH chunks.  The diagonal
// element of the square product is masked out of the tiles and added exactly
// in FP64 by the epilogue as (s_f + sigma^2) V.
//
// Two arithmetic forms share this structure:
//   BF16X3 (the mixed form; the name is the ABI's): the distance from FP16
//           hi/lo coordinates (centred on the b stream's column means) with the
//           three products hi.hi + hi.lo + lo.hi on v_mfma_f32_16x16x32_f16; M
//           and V split x = hi + lo in FP16 as well, after power-of-two scalings
//           that keep them in FP16's normal range (2^15 M; each column of V so
//           that its largest entry lies in [2^14, 2^15)), the same three
//           products on the same instruction; FP32 accumulation, the scalings
//           undone exactly in the FP64 epilogue.
//   FP32:   v_mfma_f32_16x16x4_f32 for both products; the squared norms
//           initialise the distance accumulator.
// Row-independent BF16X3 cross products with many columns (prediction) use a
// variant that evaluates each entry once for all columns (the wide sweep), and
// the FP64 form (low-noise regime) runs both contractions on
// v_mfma_f64_16x16x4; both are described where they are defined.
#include "internal.h"
#include "mfma_bf16.h"

#include <algorithm>
#include <mutex>
#include <vector>
#include <cmath>

namespace gpk {

constexpr int kFlush = 32;  // 32-point chunks accumulated in FP32 before the FP64 flush
constexpr int kF64MaxD = 64;   // FP64 form: features held in registers
constexpr int kF64Chunk = 32;  // FP64 form: points per LDS chunk
constexpr int kF64Cols = 64;   // FP64 form: V columns per pass
constexpr int kF64Rows = 64;   // FP64 form: output rows per workgroup

// The profile m(r) from S = r^2 scaled as above.  ACCURATE replaces the raw
// v_sqrt_f32 by v_rsq_f32 plus one Newton step on the residual S - u^2.  The raw
// instruction is within 9.3e-8 relative (about 1.6 ulp; 15% of results not
// correctly rounded, slightly biased low) and the Newton form correctly rounded,
// both measured over 4.2M values in [1e-2, 1e3).  The FP32 form uses the Newton
// form (its VALU work hides behind the slower FP32 matrix cores); in the mixed
// form the hi/lo splits dominate the error.
template <int KIND, bool ACCURATE>
__device__ __forceinline__ float profile(float S) {
  if constexpr (KIND == GP_MATERN52) {
    float u;
    if constexpr (ACCURATE) {
      const float s = __builtin_fmaxf(__builtin_fabsf(S), 1e-30f);
      const float y = __builtin_amdgcn_rsqf(s);
      const float u0 = s * y;
      u = __builtin_fmaf(__builtin_fmaf(-u0, u0, s), 0.5f * y, u0);
    } else {
      u = __builtin_amdgcn_sqrtf(__builtin_fabsf(S));
    }
    const float e = __builtin_amdgcn_exp2f(-u);
    const float poly = __builtin_fmaf(__builtin_fmaf(u, kMaternC2, kMaternC1), u, 1.0f);
    return poly * e;
  } else {
    return __builtin_amdgcn_exp2f(-__builtin_fabsf(S));
  }
}

// kMScale m(r) for the mixed form's FP16 value products: the Matern scale rides in
// the polynomial's constants, the RBF one costs a multiply.
template <int KIND>
__device__ __forceinline__ float profile_scaled(float S) {
  if constexpr (KIND == GP_MATERN52) {
    const float u = __builtin_amdgcn_sqrtf(__builtin_fabsf(S));
    const float e = __builtin_amdgcn_exp2f(-u);
    return __builtin_fmaf(__builtin_fmaf(u, kMaternC2s, kMaternC1s), u, kMScale) * e;
  } else {
    return __builtin_amdgcn_exp2f(-__builtin_fabsf(S)) * kMScale;
  }
}

// ---------------------------------------------------------------- preparation
//
// Distances of the mixed form.  r^2 = n_a + n_b - 2 x'_a . x'_b runs on the FP16
// matrix cores with each centred, scaled coordinate x' = (x - c) s split as
// x' ~ h + l, h = RNE16(x'), l = RNE16(x' - h) (22 significant bits), and the
// three products h.h + h.l + l.h; n = sum (h + l)^2, so that the dropped l.l
// leaves an error of 2 l_a . l_b (about 2^-22 |x'|^2, of either sign) instead of a
// bias.  The centre c is the column mean of the b stream (the training points),
// so the coordinates, and with them the cancellation in n_a + n_b - 2 x'_a . x'_b,
// stay as small as the data's spread allows whatever its offset.  FP16 holds
// |h| <= 32752 (-2h must stay finite): a point with a scaled coordinate beyond
// that, about 10^4 lengthscales from the centre, gets a NaN norm, and every
// product involving it is NaN (never silently wrong).  The norms enter the K
// padding as three FP16 digits against the constants kNormScale (a mixed-radix
// expansion whose residual is below 1e-9 relative up to n ~ 2e9).

constexpr float kNormScale[3] = {32768.f, 16.f, 0.0078125f};  // 2^15, 2^4, 2^-7
constexpr double kMaxScaled = 32752.0;                      // largest |h| with -2h finite in FP16
constexpr double kMaxNorm = 65504.0 * 32768.0;              // largest n the top digit holds

__device__ __forceinline__ double f16_round(double x) { return (double)(_Float16)(float)x; }

// Column means of the row-major n x d matrix X (the centre of the mixed form), in
// two fixed-order passes: sums over blocks of consecutive rows, then over the
// blocks, so that repeated runs give the same bits.
constexpr int64_t kMeanBlocks = 1024;

static int64_t colmean_blocks(int64_t n) {
  return std::max<int64_t>(1, std::min<int64_t>(kMeanBlocks, (n + 255) / 256));
}

size_t colmean_scratch_doubles(int64_t n, int d) { return (size_t)colmean_blocks(n) * (size_t)d; }

__global__ void colmean_partial_kernel(const double* __restrict__ X, int64_t n, int d, int64_t rows_per_blk,
                                       double* __restrict__ part) {
  const int j = threadIdx.x;
  if (j >= d) return;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < n ? r0 + rows_per_blk : n;
  double s = 0.0;
#pragma unroll 4
  for (int64_t i = r0; i < r1; ++i) s += X[i * d + j];
  part[(int64_t)blockIdx.x * d + j] = s;
}

__global__ void colmean_final_kernel(const double* __restrict__ part, int64_t nblk, int d, int64_t n,
                                     double* __restrict__ mu) {
  const int j = threadIdx.x;
  if (j >= d) return;
  double s = 0.0;
  for (int64_t b = 0; b < nblk; ++b) s += part[b * d + j];
  mu[j] = s / (double)n;
}

hipError_t column_means(const double* X, int64_t n, int d, double* part, double* mu, hipStream_t st) {
  if (!X || !part || !mu || n < 1 || d < 1 || d > GP_MAX_D) return hipErrorInvalidValue;
  const int64_t nblk = colmean_blocks(n);
  const int64_t rpb = (n + nblk - 1) / nblk;
  colmean_partial_kernel<<<(unsigned)nblk, 128, 0, st>>>(X, n, d, rpb, part);
  colmean_final_kernel<<<1, 128, 0, st>>>(part, nblk, d, n, mu);
  return hipGetLastError();
}

// Squared norm of each prepared point (FP64).  mode 1 (mixed form): the centred
// FP16 split above, n = sum (h + l)^2, NaN out of range.  mode 0 (FP32 form):
// n = sum f^2 with f = fl32(x s), no centring.  ctr: the centre (d values, mode 1).
__global__ __launch_bounds__(256) void prep_norm_kernel(const double* __restrict__ X, int64_t n, int64_t npad,
                                                        int d, Scale sc, int mixed, const double* __restrict__ ctr,
                                                        double* __restrict__ nrm) {
  // Each wave owns 64 consecutive points.  Per slice of 16 features the wave
  // loads the 64 x 16 block of X (each load instruction covers four rows'
  // 128-byte runs), turns every element into its norm term and parks the terms
  // in LDS; lane r then adds row r's terms in feature order, the same sequence
  // of additions as a per-point loop over the features.
  constexpr int kF = 16;
  __shared__ double term[4][64][kF + 1];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * 64;
  const int fl = lane & 15;
  double s = 0.0;
  if (n > 0) {  // the same for the whole block
    for (int j0 = 0; j0 < d; j0 += kF) {
      const int f = j0 + fl < d ? j0 + fl : d - 1;
      const double scale = sc.s[f];
      const double c = mixed ? ctr[f] : 0.0;
      double x[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {  // row 4 k + lane / 16 of the wave's 64 (clamped into X)
        const int64_t pr = r0 + 4 * k + (lane >> 4);
        x[k] = X[(pr < n ? pr : n - 1) * d + f];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int i = 4 * k + (lane >> 4);
        double t;
        if (mixed) {
          const double v = (x[k] - c) * scale;
          const double h = f16_round(v);
          const double l = f16_round(v - h);
          t = __builtin_fabs(v) <= kMaxScaled ? (h + l) * (h + l) : __builtin_nan("");
        } else {
          const double fv = (float)(x[k] * scale);
          t = fv * fv;
        }
        term[wave][i][fl] = (r0 + i < n && j0 + fl < d) ? t : 0.0;
      }
      __syncthreads();
      const int nf = d - j0 < kF ? d - j0 : kF;
      for (int q = 0; q < nf; ++q) s += term[wave][lane][q];
      __syncthreads();  // the next slice overwrites the terms
    }
  }
  if (mixed && !(s <= kMaxNorm)) s = __builtin_nan("");
  const int64_t p = r0 + lane;
  if (p < npad) nrm[p] = p < n ? s : 0.0;
}

// Mixed-form point fragments.  K layout of a prepared point (length 32*KS, zero padded):
//   row side (b):    [-2h_0..-2h_{d-1}, -2h_0.., -2l_0.., D2, D1, D0, C2, C1, C0, 0..]
//   column side (a): [  h_0..  h_{d-1},   l_0..,   h_0.., C2, C1, C0, D2, D1, D0, 0..]
// with C = kNormScale and D the point's norm digits (n = sum_k D_k C_k), so that
// sum_K row*col = -2(h.h + h.l + l.h) + n_b + n_a.  FP16 values, stored as
// 16-byte units.  Fragment (blk, ks, lane) holds K = 32 ks + 8 (lane/16) + j,
// j = 0..7, of point 16 blk + lane%16.
__global__ void prep_frag_f16x3_kernel(const double* __restrict__ X, const double* __restrict__ nrm,
                                       const double* __restrict__ ctr, int64_t n, int64_t nblk, int d, int KS,
                                       Scale sc, bf16x8* __restrict__ xr, bf16x8* __restrict__ xc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nblk * KS * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;
  const int ks = (int)(rest % KS);
  const int64_t blk = rest / KS;
  const int64_t p = blk * 16 + (lane & 15);
  const int g = lane >> 4;
  f16x8 r, c;
  double dig[3] = {0.0, 0.0, 0.0};
  if (p < n) {
    double rem = nrm[p];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      dig[q] = f16_round(rem * (1.0 / (double)kNormScale[q]));  // powers of two: exact
      rem -= dig[q] * (double)kNormScale[q];
    }
  }
  for (int j = 0; j < 8; ++j) {
    const int k = 32 * ks + 8 * g + j;
    double rv = 0.0, cv = 0.0;
    if (p < n) {
      if (k < 3 * d) {
        const int seg = k / d, f = k - seg * d;
        const double v = (X[p * d + f] - ctr[f]) * sc.s[f];
        const double h = f16_round(v);
        const double l = f16_round(v - h);
        rv = -2.0 * (seg == 2 ? l : h);
        cv = (seg == 1 ? l : h);
      } else if (k < 3 * d + 3) {
        const int q = k - 3 * d;
        rv = dig[q];
        cv = kNormScale[q];
      } else if (k < 3 * d + 6) {
        const int q = k - 3 * d - 3;
        rv = kNormScale[q];
        cv = dig[q];
      }
    }
    r[j] = (_Float16)(float)rv;
    c[j] = (_Float16)(float)cv;
  }
  if (xr) xr[idx] = __builtin_bit_cast(bf16x8, r);
  if (xc) xc[idx] = __builtin_bit_cast(bf16x8, c);
}

// FP32 point fragments: float4 (blk, q, lane) = f(point 16 blk + lane%16, feature
// 16 q + 4 s + lane/16) for s = 0..3, f = -2 x~ (row side) or x~ (column side).
__global__ void prep_frag_fp32_kernel(const double* __restrict__ X, const double* __restrict__ nrm,
                                      int64_t n, int64_t nblk, int d, int KQ, Scale sc,
                                      f32x4* __restrict__ xr, f32x4* __restrict__ xc,
                                      float* __restrict__ nrm_r, float* __restrict__ nrm_c) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nblk * KQ * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;
  const int q = (int)(rest % KQ);
  const int64_t blk = rest / KQ;
  const int64_t p = blk * 16 + (lane & 15);
  const int g = lane >> 4;
  f32x4 r, c;
  for (int s = 0; s < 4; ++s) {
    const int f = 16 * q + 4 * s + g;
    float v = 0.f;
    if (p < n && f < d) v = (float)(X[p * d + f] * sc.s[f]);
    r[s] = -2.f * v;
    c[s] = v;
  }
  if (xr) xr[idx] = r;
  if (xc) xc[idx] = c;
  if (q == 0 && g == 0) {
    const float nv = p < n ? (float)nrm[p] : 0.f;
    if (nrm_r) nrm_r[p] = nv;
    if (nrm_c) nrm_c[p] = nv;
  }
}

// Column scales of the mixed form's V fragments.  vmax_partial_kernel: the
// largest |V| of each column over kVParts row ranges (NaN entries are skipped
// here and reach the products through the values themselves); vscale_kernel:
// scale[c] = 2^e with e = 15 - E, max |V_c| = f 2^E (f in [1/2, 1)), so that the
// scaled column's largest entry lies in [2^14, 2^15), and inv[c] = 2^(-e - 15),
// the factor that takes a partial sum of (kMScale m)(scale V) back to m V.  A zero
// or non-finite column keeps scale 1; e is clamped to [-1022, 1023], which only a
// column whose largest entry lies below 2^-1008 reaches (its scaled entries then stay
// below 2^15 and, down to 2^-1046 relative to that, in FP16's normal range).
constexpr int kVParts = 64;

__global__ __launch_bounds__(256) void vmax_partial_kernel(const double* __restrict__ V, int64_t ldv,
                                                           const double* __restrict__ col0, int64_t n,
                                                           double* __restrict__ part) {
  __shared__ double red[256];
  const int c = blockIdx.y;
  const int64_t per = (n + kVParts - 1) / kVParts;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < n ? r0 + per : n;
  const double* src = col0 ? (c == 0 ? col0 : V + (int64_t)(c - 1) * ldv) : V + (int64_t)c * ldv;
  double mx = 0.0;
  for (int64_t b = r0 + threadIdx.x; b < r1; b += 256) mx = fmax(mx, fabs(src[b]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)c * kVParts + blockIdx.x] = red[0];
}

__global__ void vscale_kernel(const double* __restrict__ part, int t, double* __restrict__ scale,
                              double* __restrict__ inv) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= t) return;
  double mx = 0.0;
  for (int q = 0; q < kVParts; ++q) mx = fmax(mx, part[(int64_t)c * kVParts + q]);
  int e = 0;
  if (mx > 0.0 && mx <= 1.7976931348623157e308) {
    int E = 0;
    (void)frexp(mx, &E);
    e = 15 - E;
    e = e < -1022 ? -1022 : (e > 1023 ? 1023 : e);  // 2^e and 2^(-e - 15) stay representable
  }
  scale[c] = ldexp(1.0, e);
  inv[c] = ldexp(1.0, -e - 15);
}

__global__ void colmax_final_kernel(const double* __restrict__ part, int t, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= t) return;
  double mx = 0.0;
  for (int q = 0; q < kVParts; ++q) mx = fmax(mx, part[(int64_t)c * kVParts + q]);
  out[c] = mx;
}

size_t column_absmax_scratch_doubles(int t) { return (size_t)kVParts * (size_t)t; }

hipError_t column_absmax(const double* V, int64_t ldv, int64_t n, int t, double* part, double* out, hipStream_t st) {
  if (!V || !part || !out || t < 1 || n < 1) return hipErrorInvalidValue;
  vmax_partial_kernel<<<dim3(kVParts, (unsigned)t), 256, 0, st>>>(V, ldv, nullptr, n, part);
  colmax_final_kernel<<<(unsigned)((t + 63) / 64), 64, 0, st>>>(part, t, out);
  return hipGetLastError();
}

// Mixed-form V fragments: (chunk, cb, hl, lane) -> 8 FP16 of v' = scale[c] V[b][c],
// b = 32 chunk + vperm(g, j), c = 16 cb + lane%16; hl = 0: hi = RNE16(v'),
// hl = 1: lo = RNE16(v' - hi).  Columns c >= t are zero.
__global__ void prep_v_f16x3_kernel(const double* __restrict__ V, int64_t ldv, const double* __restrict__ col0,
                                    const double* __restrict__ scale, int64_t n, int t, int64_t nchunks, int ntb,
                                    bf16x8* __restrict__ vf) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nchunks * ntb * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;
  const int cb = (int)(rest % ntb);
  const int64_t ch = rest / ntb;
  const int c = 16 * cb + (lane & 15);
  const int g = lane >> 4;
  const double sc = c < t ? scale[c] : 0.0;
  f16x8 hi, lo;
  for (int j = 0; j < 8; ++j) {
    const int64_t b = ch * 32 + vperm(g, j);
    double v = 0.0;
    if (b < n && c < t) v = sc * (col0 ? (c == 0 ? col0[b] : V[(int64_t)(c - 1) * ldv + b]) : V[(int64_t)c * ldv + b]);
    const double h = f16_round(v);
    hi[j] = (_Float16)(float)h;
    lo[j] = (_Float16)(float)(v - h);
  }
  vf[(rest * 2 + 0) * 64 + lane] = __builtin_bit_cast(bf16x8, hi);
  vf[(rest * 2 + 1) * 64 + lane] = __builtin_bit_cast(bf16x8, lo);
}

// FP32 V fragments: (chunk, cb, tile, lane) -> float4 of V[b = 32 chunk + 16 tile + 4g + i]
// [c = 16 cb + lane%16], i = 0..3.
__global__ void prep_v_fp32_kernel(const double* __restrict__ V, int64_t ldv, const double* __restrict__ col0,
                                   int64_t n, int t, int64_t nchunks, int ntb, f32x4* __restrict__ vf) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nchunks * ntb * 2 * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;  // (ch * ntb + cb) * 2 + tile
  const int tile = (int)(rest & 1);
  const int64_t cbch = rest >> 1;
  const int cb = (int)(cbch % ntb);
  const int64_t ch = cbch / ntb;
  const int c = 16 * cb + (lane & 15);
  const int g = lane >> 4;
  f32x4 o;
  for (int i = 0; i < 4; ++i) {
    const int64_t b = ch * 32 + 16 * tile + 4 * g + i;
    double v = 0.0;
    if (b < n && c < t) v = col0 ? (c == 0 ? col0[b] : V[(int64_t)(c - 1) * ldv + b]) : V[(int64_t)c * ldv + b];
    o[i] = (float)v;
  }
  vf[idx] = o;
}

// ------------------------------------------------------------------ main sweep

struct SweepArgs {
  const void* xr;
  const void* xc;
  const float* nrm_b;
  const float* nrm_a;
  const void* vf;
  double* part;
  int64_t mpad;
  int64_t nchunks;
  int64_t cps;   // chunks per split
  int ntb;       // 16-column blocks in vf
  int tpad;      // columns of the partial buffer
  int square;    // mask the diagonal (square product)
};

// 16-row blocks per wave: each staged b-stream fragment serves NA tiles and
// each V fragment NA row blocks, as far as the registers allow (two blocks
// with three or four column blocks fit only up to KS = 5).
template <int KS, int NT>
struct NAOf {
  static constexpr int value = NT == 1 ? 4 : (NT == 2 || KS <= 5 ? 2 : 1);
};

// One 32-point chunk of the b stream staged in LDS: the 2 KS point fragments
// followed by the NT (hi, lo) V fragments, 64 lanes x 16 bytes each.
template <int KS, int NT>
struct ChunkUnits {
  static constexpr int kPoint = 2 * KS * 64;
  static constexpr int kV = 2 * NT * 64;
  static constexpr int kAll = kPoint + kV;
  static constexpr int kPerThread = (kAll + 255) / 256;
};

template <int KS, int NT, int KIND>
__global__ __launch_bounds__(256, 2) void sweep_bf16x3_kernel(SweepArgs a) {
  constexpr int NA = NAOf<KS, NT>::value;
  using CU = ChunkUnits<KS, NT>;
  __shared__ bf16x8 stage[2][CU::kAll];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 4;
  const int64_t ablk0 = ((int64_t)blockIdx.x * 4 + wave) * NA;  // every wave is live: mpad % (64 NA) == 0
  const int cb0 = blockIdx.z * NT;
  const bf16x8* __restrict__ xr = (const bf16x8*)a.xr;
  const bf16x8* __restrict__ xc = (const bf16x8*)a.xc;
  const bf16x8* __restrict__ vf = (const bf16x8*)a.vf;

  bf16x8 A[NA][KS];
#pragma unroll
  for (int ab = 0; ab < NA; ++ab)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) A[ab][ks] = xc[((ablk0 + ab) * KS + ks) * 64 + lane];

  double acc64[NA][NT][4];
  f32x4 acc[NA][NT];
#pragma unroll
  for (int ab = 0; ab < NA; ++ab)
#pragma unroll
    for (int cb = 0; cb < NT; ++cb) {
      acc[ab][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < 4; ++i) acc64[ab][cb][i] = 0.0;
    }

  const int64_t c_begin = (int64_t)blockIdx.y * a.cps;
  const int64_t c_end = c_begin + a.cps < a.nchunks ? c_begin + a.cps : a.nchunks;

  // cooperative load of one chunk: unit u < kPoint comes from the point stream,
  // the rest from the V fragments of this launch's column group
  bf16x8 pre[CU::kPerThread];
  auto fetch = [&](int64_t ch) {
#pragma unroll
    for (int r = 0; r < CU::kPerThread; ++r) {
      const int u = tid + 256 * r;
      if (u < CU::kPoint) {
        pre[r] = xr[(2 * ch * KS) * 64 + u];
      } else if (u < CU::kAll) {
        pre[r] = vf[(ch * a.ntb + cb0) * 2 * 64 + (u - CU::kPoint)];
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int r = 0; r < CU::kPerThread; ++r) {
      const int u = tid + 256 * r;
      if (u < CU::kAll) stage[buf][u] = pre[r];
    }
  };
  if (c_begin < c_end) {
    fetch(c_begin);
    stash(0);
  }
  __syncthreads();
  for (int64_t ch = c_begin; ch < c_end; ++ch) {
    const int cur = (int)((ch - c_begin) & 1);
    const bool more = ch + 1 < c_end;
    if (more) fetch(ch + 1);
    bf16x8 B0[KS], B1[KS], VH[NT], VL[NT];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      B0[ks] = stage[cur][ks * 64 + lane];
      B1[ks] = stage[cur][(KS + ks) * 64 + lane];
    }
#pragma unroll
    for (int cb = 0; cb < NT; ++cb) {
      VH[cb] = stage[cur][CU::kPoint + (2 * cb) * 64 + lane];
      VL[cb] = stage[cur][CU::kPoint + (2 * cb + 1) * 64 + lane];
    }
#pragma unroll
    for (int ab = 0; ab < NA; ++ab) {
      f32x4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        s0 = mfma_dist(B0[ks], A[ab][ks], s0);
        s1 = mfma_dist(B1[ks], A[ab][ks], s1);
      }
      f32x8 mv;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        mv[i] = profile_scaled<KIND>(s0[i]);
        mv[4 + i] = profile_scaled<KIND>(s1[i]);
      }
      if (a.square) {
        const int64_t arow = (ablk0 + ab) * 16;
        if (arow == ch * 32 || arow == ch * 32 + 16) {
          const int off = arow == ch * 32 ? 0 : 4;
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if ((lane & 15) == 4 * g + i) mv[off + i] = 0.f;
        }
      }
      bf16x8 H, L;
      split_f16x8(mv, H, L);
#pragma unroll
      for (int cb = 0; cb < NT; ++cb) {
        acc[ab][cb] = mfma_val(H, VH[cb], acc[ab][cb]);
        acc[ab][cb] = mfma_val(H, VL[cb], acc[ab][cb]);
        acc[ab][cb] = mfma_val(L, VH[cb], acc[ab][cb]);
      }
    }
    if (((ch - c_begin + 1) % kFlush) == 0 || !more) {
#pragma unroll
      for (int ab = 0; ab < NA; ++ab)
#pragma unroll
        for (int cb = 0; cb < NT; ++cb) {
#pragma unroll
          for (int i = 0; i < 4; ++i) acc64[ab][cb][i] += (double)acc[ab][cb][i];
          acc[ab][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
    if (more) stash(cur ^ 1);
    __syncthreads();
  }
  // partial[(split * tpad + col) * mpad + row]
#pragma unroll
  for (int ab = 0; ab < NA; ++ab)
#pragma unroll
    for (int cb = 0; cb < NT; ++cb) {
      const int64_t col = (int64_t)(cb0 + cb) * 16 + (lane & 15);
      const int64_t row = (ablk0 + ab) * 16 + 4 * g;
      double* dst = a.part + ((int64_t)blockIdx.y * a.tpad + col) * a.mpad + row;
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[i] = acc64[ab][cb][i];
    }
}

// ------------------------------------------------------------------ wide cross sweep
//
// The prediction product K(Z, X) [alpha | R] has few query rows (a request
// batch) and many columns (1 + k_c).  The sweep above evaluates each kernel
// entry once per 64-column group; here a workgroup owns 64 query rows and all
// columns of one chunk split.  Per 32-point chunk, wave w evaluates the
// distances and the profile of row block w (16 rows) into an LDS tile (FP16
// hi / lo, two buffers so that one barrier per chunk suffices); then every
// wave multiplies the four row blocks' tiles by its own column blocks (cb = w,
// w + 4, ...).  Both operand streams run one chunk ahead in registers: the
// point fragments of chunk c + 1 are loaded during chunk c - 1 and written to
// LDS at the top of chunk c, and each wave's V fragments of chunk c + 1 are
// loaded during chunk c.  FP32 windows of kFlush chunks are added into the
// split's FP64 partials (this workgroup owns those slots) in the same order
// as the sweep above, so each output row's sums depend on n only, not on the
// batch; a split of one window stores it as FP32, which is exact and halves
// the partials' traffic.  Workgroups are numbered so that the row groups of
// one split run back to back on one XCD and share the chunk data in its L2.
constexpr int kWideNB = 5;  // column blocks per wave: 4 waves x 5 x 16 = 320 >= 1 + 256 columns

struct WideArgs {
  const void* xr;  // b stream (training points)
  const void* xc;  // query-row fragments
  const void* vf;  // V fragments, vstride 16-column blocks per chunk
  double* part;    // [split][tpad][mpad], FP64, or FP32 when f32part
  int64_t mpad, nchunks, cps, nsplit;
  int ntb, vstride, tpad, rgroups;
  int f32part;  // cps <= kFlush: each split is one FP32 window, stored exactly as FP32
};

template <int KS, int KIND>
__global__ __launch_bounds__(256, 2) void wide_cross_bf16x3_kernel(WideArgs a) {
  constexpr int kPoint = 2 * KS * 64;         // 16-byte units of one chunk's point fragments
  constexpr int kPer = (kPoint + 255) / 256;  // units per thread
  __shared__ bf16x8 stage[2][kPoint];
  __shared__ bf16x8 tile[2][4][2][64];  // [parity][row block][hi / lo][lane]
  // hardware workgroup i runs on XCD i % 8; the j-th workgroup an XCD receives
  // (j = i / 8) takes row group j % R of split 8 (j / R) + i % 8
  const int64_t hw = blockIdx.x;
  const int64_t j8 = hw >> 3;
  const int rg = (int)(j8 % a.rgroups);
  const int64_t split = (j8 / a.rgroups) * 8 + (hw & 7);
  if (split >= a.nsplit) return;  // whole workgroup, before any barrier
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t ablk = (int64_t)rg * 4 + wave;  // this wave's row block (16 rows)
  const bf16x8* __restrict__ xr = (const bf16x8*)a.xr;
  const bf16x8* __restrict__ xc = (const bf16x8*)a.xc;
  const bf16x8* __restrict__ vf = (const bf16x8*)a.vf;
  bf16x8 A[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) A[ks] = xc[(ablk * KS + ks) * 64 + lane];
  f32x4 acc[4][kWideNB];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int jb = 0; jb < kWideNB; ++jb) acc[rb][jb] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t c_begin = split * a.cps;
  const int64_t c_end = c_begin + a.cps < a.nchunks ? c_begin + a.cps : a.nchunks;

  // Loads are unconditional (indexes clamped into the chunk and to the last
  // column block) so that the number in flight is the same on every path and
  // the waits before each use cover only what that use needs.
  bf16x8 pre[kPer];
  auto fetch = [&](int64_t ch) {
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int u = tid + 256 * r < kPoint ? tid + 256 * r : kPoint - 1;
      pre[r] = xr[(2 * ch * KS) * 64 + u];
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int u = tid + 256 * r;
      if (u < kPoint) stage[buf][u] = pre[r];
    }
  };
  bf16x8 Vc[kWideNB][2], Vn[kWideNB][2];
  auto vload = [&](int64_t ch, bf16x8(&Vx)[kWideNB][2]) {
#pragma unroll
    for (int jb = 0; jb < kWideNB; ++jb) {
      const int cb = wave + 4 * jb < a.ntb ? wave + 4 * jb : a.ntb - 1;
      Vx[jb][0] = vf[((ch * a.vstride + cb) * 2 + 0) * 64 + lane];
      Vx[jb][1] = vf[((ch * a.vstride + cb) * 2 + 1) * 64 + lane];
    }
  };
  // the FP32 window into the split's FP64 partials (written by the first
  // window); later windows read a column block's 16 partials at once, then add
  bool first_window = true;
  auto flush = [&]() {
    const int64_t row0 = (int64_t)rg * 64 + 4 * (lane >> 4);
#pragma unroll
    for (int jb = 0; jb < kWideNB; ++jb) {
      const int cb = wave + 4 * jb;
      if (cb < a.ntb && a.f32part) {
        const int64_t col = (int64_t)cb * 16 + (lane & 15);
        float* dst = (float*)a.part + (split * a.tpad + col) * a.mpad + row0;
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) *(f32x4*)(dst + 16 * rb) = acc[rb][jb];
      } else if (cb < a.ntb) {
        const int64_t col = (int64_t)cb * 16 + (lane & 15);
        double* dst = a.part + (split * a.tpad + col) * a.mpad + row0;
        double old[4][4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int i = 0; i < 4; ++i) old[rb][i] = first_window ? 0.0 : dst[16 * rb + i];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
          for (int i = 0; i < 4; ++i) dst[16 * rb + i] = old[rb][i] + (double)acc[rb][jb][i];
      }
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) acc[rb][jb] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    first_window = false;
  };

  fetch(c_begin);
  stash(0);
  if (c_begin + 1 < c_end) fetch(c_begin + 1);
  vload(c_begin, Vc);
  // drain the prologue's loads: the loop then starts with nothing in flight,
  // as it does after every iteration (the V copy below waits for the loads
  // issued at its top), so no wait inside the loop covers a newer load
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int64_t ch = c_begin; ch < c_end; ++ch) {
    const int cur = (int)((ch - c_begin) & 1);
    const bool more = ch + 1 < c_end;
    // stage[cur ^ 1] was last read by every wave's phase A of the previous
    // chunk, which the previous barrier closed
    if (more) stash(cur ^ 1);
    if (ch + 2 < c_end) fetch(ch + 2);
    if (more) vload(ch + 1, Vn);
    // phase A: this wave's row block against the chunk
    {
      f32x4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        s0 = mfma_dist(stage[cur][ks * 64 + lane], A[ks], s0);
        s1 = mfma_dist(stage[cur][(KS + ks) * 64 + lane], A[ks], s1);
      }
      f32x8 mv;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        mv[i] = profile_scaled<KIND>(s0[i]);
        mv[4 + i] = profile_scaled<KIND>(s1[i]);
      }
      bf16x8 H, L;
      split_f16x8(mv, H, L);
      tile[cur][wave][0][lane] = H;
      tile[cur][wave][1][lane] = L;
    }
    // the four tiles of this chunk, and the next chunk's points, are in LDS
    __syncthreads();
    // phase B: the four row blocks against this wave's column blocks
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const bf16x8 TH = tile[cur][rb][0][lane];
      const bf16x8 TL = tile[cur][rb][1][lane];
#pragma unroll
      for (int jb = 0; jb < kWideNB; ++jb) {
        if (wave + 4 * jb < a.ntb) {
          acc[rb][jb] = mfma_val(TH, Vc[jb][0], acc[rb][jb]);
          acc[rb][jb] = mfma_val(TH, Vc[jb][1], acc[rb][jb]);
          acc[rb][jb] = mfma_val(TL, Vc[jb][0], acc[rb][jb]);
        }
      }
    }
    if (((ch - c_begin + 1) % kFlush) == 0 || !more) flush();
    if (more) {
#pragma unroll
      for (int jb = 0; jb < kWideNB; ++jb) {
        Vc[jb][0] = Vn[jb][0];
        Vc[jb][1] = Vn[jb][1];
      }
    }
  }
}

// 16-row blocks per wave of the FP32 form.
template <int NT>
struct NAOfF32 {
  static constexpr int value = NT == 1 ? 4 : (NT == 2 ? 2 : 1);
};

template <int KQ, int NT, int KIND>
__global__ __launch_bounds__(256, 2) void sweep_fp32_kernel(SweepArgs a) {
  constexpr int NA = NAOfF32<NT>::value;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4;
  const int64_t ablk0 = ((int64_t)blockIdx.x * 4 + wave) * NA;
  if (ablk0 * 16 >= a.mpad) return;
  const int cb0 = blockIdx.z * NT;
  const f32x4* __restrict__ xr = (const f32x4*)a.xr;
  const f32x4* __restrict__ xc = (const f32x4*)a.xc;
  const f32x4* __restrict__ vf = (const f32x4*)a.vf;

  f32x4 A[NA][KQ];
  float na[NA];
#pragma unroll
  for (int ab = 0; ab < NA; ++ab) {
#pragma unroll
    for (int q = 0; q < KQ; ++q) A[ab][q] = xc[((ablk0 + ab) * KQ + q) * 64 + lane];
    na[ab] = a.nrm_a[(ablk0 + ab) * 16 + (lane & 15)];
  }
  double acc64[NA][NT][4];
#pragma unroll
  for (int ab = 0; ab < NA; ++ab)
#pragma unroll
    for (int cb = 0; cb < NT; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc64[ab][cb][i] = 0.0;

  const int64_t c_begin = (int64_t)blockIdx.y * a.cps;
  const int64_t c_end = c_begin + a.cps < a.nchunks ? c_begin + a.cps : a.nchunks;
  for (int64_t c0 = c_begin; c0 < c_end; c0 += kFlush) {
    const int64_t c1 = c0 + kFlush < c_end ? c0 + kFlush : c_end;
    f32x4 acc[NA][NT];
#pragma unroll
    for (int ab = 0; ab < NA; ++ab)
#pragma unroll
      for (int cb = 0; cb < NT; ++cb) acc[ab][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t ch = c0; ch < c1; ++ch) {
      f32x4 B0[KQ], B1[KQ];
#pragma unroll
      for (int q = 0; q < KQ; ++q) {
        B0[q] = xr[((2 * ch) * KQ + q) * 64 + lane];
        B1[q] = xr[((2 * ch + 1) * KQ + q) * 64 + lane];
      }
      const f32x4 nb0 = *(const f32x4*)(a.nrm_b + ch * 32 + 4 * g);
      const f32x4 nb1 = *(const f32x4*)(a.nrm_b + ch * 32 + 16 + 4 * g);
      f32x4 V0[NT], V1[NT];
#pragma unroll
      for (int cb = 0; cb < NT; ++cb) {
        const int64_t base = ((ch * a.ntb + cb0 + cb) * 2) * 64 + lane;
        V0[cb] = vf[base];
        V1[cb] = vf[base + 64];
      }
#pragma unroll
      for (int ab = 0; ab < NA; ++ab) {
        f32x4 s0 = nb0 + na[ab];
        f32x4 s1 = nb1 + na[ab];
#pragma unroll
        for (int q = 0; q < KQ; ++q)
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            s0 = __builtin_amdgcn_mfma_f32_16x16x4f32(B0[q][s], A[ab][q][s], s0, 0, 0, 0);
            s1 = __builtin_amdgcn_mfma_f32_16x16x4f32(B1[q][s], A[ab][q][s], s1, 0, 0, 0);
          }
        f32x4 m0, m1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          m0[i] = profile<KIND, true>(s0[i]);
          m1[i] = profile<KIND, true>(s1[i]);
        }
        if (a.square) {
          const int64_t arow = (ablk0 + ab) * 16;
          if (arow == ch * 32) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if ((lane & 15) == 4 * g + i) m0[i] = 0.f;
          } else if (arow == ch * 32 + 16) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if ((lane & 15) == 4 * g + i) m1[i] = 0.f;
          }
        }
#pragma unroll
        for (int cb = 0; cb < NT; ++cb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            acc[ab][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(m0[i], V0[cb][i], acc[ab][cb], 0, 0, 0);
            acc[ab][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(m1[i], V1[cb][i], acc[ab][cb], 0, 0, 0);
          }
      }
    }
#pragma unroll
    for (int ab = 0; ab < NA; ++ab)
#pragma unroll
      for (int cb = 0; cb < NT; ++cb)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc64[ab][cb][i] += (double)acc[ab][cb][i];
  }
#pragma unroll
  for (int ab = 0; ab < NA; ++ab)
#pragma unroll
    for (int cb = 0; cb < NT; ++cb) {
      const int64_t col = (int64_t)(cb0 + cb) * 16 + (lane & 15);
      const int64_t row = (ablk0 + ab) * 16 + 4 * g;
      double* dst = a.part + ((int64_t)blockIdx.y * a.tpad + col) * a.mpad + row;
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[i] = acc64[ab][cb][i];
    }
}

// out[c*ldo + r] = s_f * inv[c] * sum_split part + (square ? (s_f + sigma^2) V[c*ldv + r] : 0)
// (inv: the mixed form's column factors, a power of two; null for the FP32 form)
__global__ void kmm_epilogue_kernel(const double* __restrict__ part, int64_t nsplit, int tpad,
                                    int64_t mpad, int64_t m, int t, double sf, double diag,
                                    const double* __restrict__ inv, const double* __restrict__ V, int64_t ldv,
                                    double* __restrict__ out, int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * t) return;
  const int64_t c = idx / m, r = idx - c * m;
  double s = 0.0;
  for (int64_t sp = 0; sp < nsplit; ++sp) s += part[(sp * tpad + c) * mpad + r];
  if (inv) s *= inv[c];
  double o = sf * s;
  if (V) o += diag * V[c * ldv + r];
  out[c * ldo + r] = o;
}

// The split sum of the wide sweep: a workgroup takes one column and 64 rows,
// wave k adds the splits k, k + 4, ... in split order, and the four sums are
// then added in wave order, so the order depends on n alone.
template <typename T>
__global__ __launch_bounds__(256) void wide_epilogue_kernel(const T* __restrict__ part, int64_t nsplit, int tpad,
                                                            int64_t mpad, int64_t m, double sf,
                                                            const double* __restrict__ inv,
                                                            double* __restrict__ out, int64_t ldo) {
  __shared__ double red[4][64];
  const int r = threadIdx.x & 63;
  const int k = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * 64 + r;
  const int64_t c = blockIdx.y;
  double s = 0.0;
  if (q < m) {
    // splits k, k + 4, ... added in that order; eight loads in flight per batch
    const int64_t step = 4 * (int64_t)tpad * mpad;
    const T* src = part + ((int64_t)k * tpad + c) * mpad + q;
    int64_t sp = k;
    for (; sp + 28 < nsplit; sp += 32, src += 8 * step) {
      T v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = src[j * step];
#pragma unroll
      for (int j = 0; j < 8; ++j) s += (double)v[j];
    }
    for (; sp < nsplit; sp += 4, src += step) s += (double)src[0];
  }
  red[k][r] = s;
  __syncthreads();
  if (k == 0 && q < m) out[c * ldo + q] = sf * ((((red[0][r] + red[1][r]) + red[2][r]) + red[3][r]) * inv[c]);
}

// ------------------------------------------------------------------ host side

// Optional timing of the tile sweeps: HIP events recorded on the sweep's own
// stream around each launch, with the launch's nominal flops 2 m n (d + t).
namespace {
struct SweepTiming {
  std::mutex mu;
  bool on = false;
  struct Rec {
    hipEvent_t a, b;
    double flops;
    int64_t n, m;
    int t;
  };
  std::vector<Rec> recs;
};
SweepTiming& timing() {
  static SweepTiming t;
  return t;
}
}  // namespace

void profile_enable(bool on) {
  std::lock_guard<std::mutex> g(timing().mu);
  timing().on = on;
}

int profile_records(int64_t cap, int64_t* n, int64_t* m, int* t, double* ms, int64_t* count) {
  std::lock_guard<std::mutex> g(timing().mu);
  int64_t k = 0;
  for (auto& r : timing().recs) {
    if (k >= cap) break;
    if (hipEventSynchronize(r.b) != hipSuccess) return -1;
    float e = 0.f;
    if (hipEventElapsedTime(&e, r.a, r.b) != hipSuccess) return -1;
    n[k] = r.n;
    m[k] = r.m;
    t[k] = r.t;
    ms[k] = e;
    ++k;
  }
  *count = k;
  return 0;
}

int profile_read(int64_t* launches, double* total_ms, double* flops, bool reset) {
  std::lock_guard<std::mutex> g(timing().mu);
  int64_t n = 0;
  double ms = 0.0, fl = 0.0;
  for (auto& r : timing().recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return -1;
    float e = 0.f;
    if (hipEventElapsedTime(&e, r.a, r.b) != hipSuccess) return -1;
    ms += e;
    fl += r.flops;
    ++n;
  }
  if (reset) {
    for (auto& r : timing().recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    timing().recs.clear();
  }
  *launches = n;
  *total_ms = ms;
  *flops = fl;
  return 0;
}

static int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int kmm_ksteps(int precision, int d) {
  if (precision == GP_PREC_FP64) return d <= kF64MaxD ? 1 : -1;
  if (precision == GP_PREC_BF16X3) {
    const int need = (3 * d + 6 + 31) / 32;
    static const int kAvail[] = {2, 4, 5, 7, 13};  // the instantiated sweeps
    for (int k : kAvail)
      if (k >= need) return k;
    return -1;
  }
  const int need = (d + 15) / 16;
  static const int kAvail32[] = {1, 2, 3, 4, 8};  // the instantiated sweeps
  for (int k : kAvail32)
    if (k >= need) return k;
  return -1;
}

// Column blocks handled per launch (grid.z groups the rest).
static int nt_launch(int ntb) { return ntb >= 4 ? 4 : ntb; }
static int na_of(int ks, int nt, bool mixed) {  // NAOf<KS, NT> of the launched kernel
  if (!mixed) return nt == 1 ? 4 : (nt == 2 ? 2 : 1);
  return nt == 1 ? 4 : (nt == 2 || ks <= 5 ? 2 : 1);
}

struct SplitChoice {
  int nt, groups, tpad;
  int64_t cps, nsplit;
};

static SplitChoice choose_split(int64_t npad, int64_t mpad, int ntb, bool row_independent, int ks, bool mixed) {
  SplitChoice s;
  s.nt = nt_launch(ntb);
  s.groups = (ntb + s.nt - 1) / s.nt;
  s.tpad = s.groups * s.nt * 16;
  const int64_t nchunks = npad / 32;
  if (row_independent) {
    // depends on n only: each output row sees the same chunk boundaries whatever m is
    s.cps = std::max<int64_t>(8, (nchunks + 255) / 256);
  } else {
    const int64_t row_wgs = mpad / (64 * na_of(ks, s.nt, mixed)) * s.groups;
    const int64_t want = std::max<int64_t>(1, (2048 + row_wgs - 1) / row_wgs);
    s.cps = std::max<int64_t>(2, (nchunks + want - 1) / want);
  }
  s.nsplit = (nchunks + s.cps - 1) / s.cps;
  return s;
}

static size_t part_bytes_max(int64_t npad, int64_t mpad, int ntb, bool row_independent, int ks, bool mixed) {
  size_t best = 0;
  for (int nb = 1; nb <= ntb; ++nb) {
    const SplitChoice s = choose_split(npad, mpad, nb, row_independent, ks, mixed);
    best = std::max(best, (size_t)s.nsplit * s.tpad * mpad * sizeof(double));
  }
  return best;
}

// V region: [fragments | scale (tpad) | inv (tpad) | column-max partials (kVParts tpad)].
static size_t vfrag_core_bytes(int64_t n, int ntb_alloc) {
  return align256((size_t)round_up(n, 32) * ntb_alloc * 64 + 64);
}

size_t kmm_vfrag_bytes(int64_t n, int t) {
  const int ntb0 = (t + 15) / 16;
  const int ntb = (ntb0 + nt_launch(ntb0) - 1) / nt_launch(ntb0) * nt_launch(ntb0);
  return vfrag_core_bytes(n, ntb) + 2 * align256((size_t)ntb * 16 * 8) + align256((size_t)kVParts * ntb * 16 * 8);
}

static void carve_vfrag(KmmPlan& p, char* c) {
  const int ntb_alloc = (p.ntb + nt_launch(p.ntb) - 1) / nt_launch(p.ntb) * nt_launch(p.ntb);
  const int tpad = ntb_alloc * 16;
  p.vf = c;
  c += vfrag_core_bytes(p.n, ntb_alloc);
  p.vscale = (double*)c;  c += align256((size_t)tpad * 8);
  p.vinv = (double*)c;    c += align256((size_t)tpad * 8);
  p.vpart = (double*)c;
}

size_t kmm_plan_bytes(int precision, int d, int64_t n, int64_t m, bool square, int tmax) {
  const int ks = kmm_ksteps(precision, d);
  if (ks < 0) return 0;
  if (precision == GP_PREC_FP64)
    return align256((size_t)d * 8) + align256((size_t)n * 8) + (square ? 0 : align256((size_t)m * 8)) + 256;
  const int64_t npad = round_up(n, 32);
  const int64_t mrows = square ? n : m;
  const int64_t mpad = round_up(mrows, 256);
  const int64_t bpad = std::max(npad, mpad);  // the square case prepares mpad rows of X
  const int ntb0 = (tmax + 15) / 16;
  size_t b = 0;
  b += align256((size_t)bpad * ks * 64);           // xr
  b += align256((size_t)mpad * ks * 64);           // xc
  b += align256((size_t)bpad * 4);                 // nrm_b
  b += align256((size_t)mpad * 4);                 // nrm_a
  b += align256((size_t)bpad * 8);                 // nrm64
  b += align256((size_t)d * 8);                    // ctr
  b += align256(colmean_scratch_doubles(n, d) * 8);  // column-mean partials
  b += kmm_vfrag_bytes(n, tmax);                   // vf, column scales
  b += align256(part_bytes_max(npad, mpad, ntb0, !square, ks, precision == GP_PREC_BF16X3));  // partials
  return b;
}

bool kmm_plan_init(KmmPlan& p, const gp_kernel* kern, int precision, int64_t n, int64_t m,
                   bool square, int tmax, void* ws, size_t ws_bytes) {
  const size_t need = kmm_plan_bytes(precision, kern->d, n, m, square, tmax);
  if (need == 0 || ws == nullptr || ws_bytes < need) return false;
  p.precision = precision;
  p.kind = kern->kind;
  p.d = kern->d;
  p.square = square;
  p.n = n;
  p.m = square ? n : m;
  p.npad = round_up(n, 32);
  p.mpad = round_up(p.m, 256);
  p.nchunks = p.npad / 32;
  p.ks = kmm_ksteps(precision, kern->d);
  p.tmax = tmax;
  p.ntb = (tmax + 15) / 16;
  p.sf = kern->outputscale;
  p.noise = kern->noise;
  if (precision == GP_PREC_FP64) {
    char* c = (char*)ws;
    p.sc64 = (double*)c;  c += align256((size_t)p.d * 8);
    p.nb64 = (double*)c;  c += align256((size_t)n * 8);
    p.na64 = square ? p.nb64 : (double*)c;
    return true;
  }
  const int64_t bpad = std::max(p.npad, p.mpad);
  char* c = (char*)ws;
  p.xr = c;  c += align256((size_t)bpad * p.ks * 64);
  p.xc = c;  c += align256((size_t)p.mpad * p.ks * 64);
  p.nrm_b = (float*)c;  c += align256((size_t)bpad * 4);
  p.nrm_a = (float*)c;  c += align256((size_t)p.mpad * 4);
  p.nrm64 = (double*)c; c += align256((size_t)bpad * 8);
  p.ctr = (double*)c;   c += align256((size_t)p.d * 8);
  p.cpart = (double*)c; c += align256(colmean_scratch_doubles(n, p.d) * 8);
  carve_vfrag(p, c);
  c += kmm_vfrag_bytes(n, tmax);
  p.part = (double*)c;
  return true;
}

// Model buffer: [b-stream fragments | b norms (FP32) | V fragments | centre (d) | column-mean and FP64 norm
// scratch of the prepare step].
size_t kmm_model_bytes(int precision, int d, int64_t n, int tmax) {
  if (precision == GP_PREC_FP64) return 0;  // prediction models use the matrix-core forms
  const int ks = kmm_ksteps(precision, d);
  if (ks < 0) return 0;
  const int64_t npad = round_up(n, 32);
  return align256((size_t)npad * ks * 64) + align256((size_t)npad * 4) + kmm_vfrag_bytes(n, tmax) +
         align256((size_t)d * 8) + align256(colmean_scratch_doubles(n, d) * 8) + align256((size_t)npad * 8);
}

// Query workspace: [row fragments | row norms (FP32) | FP64 norm scratch | partials].
size_t kmm_query_bytes(int precision, int d, int64_t n, int64_t m, int tmax) {
  if (precision == GP_PREC_FP64) return 0;
  const int ks = kmm_ksteps(precision, d);
  if (ks < 0) return 0;
  const int64_t npad = round_up(n, 32);
  const int64_t mpad = round_up(m, 256);
  const int ntb = (tmax + 15) / 16;
  return align256((size_t)mpad * ks * 64) + align256((size_t)mpad * 4) + align256((size_t)mpad * 8) +
         align256(part_bytes_max(npad, mpad, ntb, true, ks, precision == GP_PREC_BF16X3));
}

bool kmm_plan_model(KmmPlan& p, const gp_kernel* kern, int precision, int64_t n, int64_t m, int tmax, void* model,
                    size_t model_bytes, void* ws, size_t ws_bytes) {
  if (!model || model_bytes < kmm_model_bytes(precision, kern->d, n, tmax)) return false;
  if (m > 0 && (!ws || ws_bytes < kmm_query_bytes(precision, kern->d, n, m, tmax))) return false;
  p.precision = precision;
  p.kind = kern->kind;
  p.d = kern->d;
  p.square = false;
  p.n = n;
  p.m = m;
  p.npad = round_up(n, 32);
  p.mpad = round_up(m > 0 ? m : 1, 256);
  p.nchunks = p.npad / 32;
  p.ks = kmm_ksteps(precision, kern->d);
  p.tmax = tmax;
  p.ntb = (tmax + 15) / 16;
  p.sf = kern->outputscale;
  p.noise = kern->noise;
  char* c = (char*)model;
  p.xr = c;  c += align256((size_t)p.npad * p.ks * 64);
  p.nrm_b = (float*)c;  c += align256((size_t)p.npad * 4);
  carve_vfrag(p, c);
  c += kmm_vfrag_bytes(n, tmax);
  p.ctr = (double*)c;  c += align256((size_t)p.d * 8);
  p.cpart = (double*)c;  c += align256(colmean_scratch_doubles(n, p.d) * 8);
  if (m > 0) {
    char* w = (char*)ws;
    p.xc = w;  w += align256((size_t)p.mpad * p.ks * 64);
    p.nrm_a = (float*)w;  w += align256((size_t)p.mpad * 4);
    p.nrm64 = (double*)w;  w += align256((size_t)p.mpad * 8);
    p.part = (double*)w;
  } else {
    // preparing the model only: the FP64 norm scratch lives at the end of the model buffer
    p.xc = nullptr;
    p.nrm_a = nullptr;
    p.nrm64 = (double*)c;
    p.part = nullptr;
  }
  return true;
}

// ------------------------------------------------------------------ FP64 form
//
// The low-noise regime (sigma^2 down to 1e-8, Sec. 3.2 and Sec. 4) needs K_hat V
// to FP64 accuracy.  Both contractions run on the FP64 matrix cores
// (v_mfma_f64_16x16x4: lane l supplies A(l % 16, k = l / 16) and B(k = l / 16,
// l % 16), and holds D(l / 16 + 4 i, l % 16)).  A workgroup owns 64 output rows
// and up to 64 columns; wave w owns rows 16 w .. 16 w + 15, their scaled
// features held in registers as the B operand.  Per 32-point chunk of the b
// stream (scaled points, norms and V values staged in LDS), for each 16-point
// half: the MFMA gives x_b . x_a with the point along D's rows, so after the
// profile (r^2 = n_a + n_b - 2 x_a.x_b, then m(r) in FP64) register i of every
// lane holds the entries of points 4 i .. 4 i + 3 of that half, exactly the A
// operand of the M V step that contracts over them.  Each entry is evaluated
// once and never leaves registers; the output tile goes through LDS so that
// the stores are coalesced.  The diagonal entry is exactly s_f (m(0) = 1) and
// sigma^2 V is added exactly.  Every row's sums run in the same order whatever
// the other rows are.
typedef double f64x4 __attribute__((ext_vector_type(4)));

// sc64[f] = feature scale (thread f < d); nrm[p] = |x_p (.) sc|^2 for p < rows.
__global__ void prep_fp64_kernel(const double* __restrict__ X, int64_t rows, int d, Scale sc,
                                 double* __restrict__ sc64, double* __restrict__ nrm) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sc64 && p < d) sc64[p] = sc.s[p];
  if (p >= rows) return;
  double s = 0.0;
  for (int f = 0; f < d; ++f) {
    const double v = X[p * d + f] * sc.s[f];
    s = fma(v, v, s);
  }
  nrm[p] = s;
}

template <int DP, int KIND>
__global__ __launch_bounds__(256) void sweep_fp64_kernel(const double* __restrict__ Xb, const double* __restrict__ nb,
                                                         int64_t n, const double* __restrict__ Xa,
                                                         const double* __restrict__ na, int64_t m, int d,
                                                         const double* __restrict__ sc64, const double* __restrict__ V,
                                                         int64_t ldv, int t, double sf, double noise, int square,
                                                         double* __restrict__ out, int64_t ldo) {
  constexpr int kBLd = DP + 2;           // point rows: the MFMA's 16-lane reads hit distinct banks
  constexpr int kVLd = kF64Chunk + 2;    // V columns, likewise
  constexpr int kOLd = kF64Rows + 1;     // output tile columns
  constexpr int kKs = DP / 4;            // K steps of the distance MFMA
  constexpr int kStage = kF64Chunk * kBLd + kF64Cols * kVLd;
  constexpr int kBuf = kStage > kF64Cols * kOLd ? kStage : kF64Cols * kOLd;
  __shared__ double buf[kBuf];  // the chunk's points [j][f] and V [c][j]; at the end the output tile [c][row]
  __shared__ double Ns[kF64Chunk];
  double* const Bs = buf;
  double* const Vs = buf + kF64Chunk * kBLd;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t a0 = (int64_t)blockIdx.x * kF64Rows;
  const int c0 = blockIdx.y * kF64Cols;
  const int tc = t - c0 < kF64Cols ? t - c0 : kF64Cols;  // columns of this pass
  const int ncb = (tc + 15) / 16;                        // 16-column blocks
  const int64_t arow = a0 + 16 * wave + lr;              // this lane's row in the products
  double xa[kKs];
#pragma unroll
  for (int s = 0; s < kKs; ++s) {
    const int f = 4 * s + lk;
    xa[s] = (arow < m && f < d) ? Xa[arow * d + f] * sc64[f] : 0.0;
  }
  const double naa = arow < m ? na[arow] : 0.0;
  // the staging threads' feature scales (the same features in every chunk)
  static_assert(kF64Chunk * DP % 256 == 0 && kF64Chunk * kF64Cols % 256 == 0, "256 threads");
  double bs[kF64Chunk * DP / 256];
#pragma unroll
  for (int it = 0; it < kF64Chunk * DP / 256; ++it) {
    const int f = (tid + 256 * it) % DP;
    bs[it] = f < d ? sc64[f] : 0.0;
  }
  f64x4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = f64x4{0.0, 0.0, 0.0, 0.0};
  // staging: the next chunk's points, V and norms are loaded into registers
  // while the current chunk is computed from LDS
  constexpr int kBPer = kF64Chunk * DP / 256, kVPer = kF64Chunk * kF64Cols / 256;
  double bv[kBPer], vv[kVPer], nv;
  auto load = [&](int64_t c0b) {
#pragma unroll
    for (int it = 0; it < kBPer; ++it) {
      const int e = tid + 256 * it, j = e / DP, f = e - j * DP;
      const int64_t b = c0b + j;
      bv[it] = (b < n && f < d) ? Xb[b * d + f] : 0.0;
    }
#pragma unroll
    for (int it = 0; it < kVPer; ++it) {
      const int e = tid + 256 * it, c = e / kF64Chunk, j = e - c * kF64Chunk;
      const int64_t b = c0b + j;
      vv[it] = (b < n && c < tc) ? V[(int64_t)(c0 + c) * ldv + b] : 0.0;
    }
    nv = (tid < kF64Chunk && c0b + tid < n) ? nb[c0b + tid] : 0.0;
  };
  load(0);
  for (int64_t b0 = 0; b0 < n; b0 += kF64Chunk) {
    __syncthreads();  // the previous chunk's readers are done
#pragma unroll
    for (int it = 0; it < kBPer; ++it) {
      const int e = tid + 256 * it, j = e / DP, f = e - j * DP;
      Bs[j * kBLd + f] = bv[it] * bs[it];
    }
#pragma unroll
    for (int it = 0; it < kVPer; ++it) {
      const int e = tid + 256 * it, c = e / kF64Chunk;
      Vs[c * kVLd + e - c * kF64Chunk] = vv[it];
    }
    if (tid < kF64Chunk) Ns[tid] = nv;
    __syncthreads();
    if (b0 + kF64Chunk < n) load(b0 + kF64Chunk);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int pb = 0; pb < 2; ++pb) {
      // x_b . x_a: D(point 16 pb + lk + 4 i, row arow)
      f64x4 dt = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < kKs; ++s)
        dt = __builtin_amdgcn_mfma_f64_16x16x4f64(Bs[(16 * pb + lr) * kBLd + 4 * s + lk], xa[s], dt, 0, 0, 0);
      double mt[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = 16 * pb + lk + 4 * i;
        const int64_t b = b0 + j;
        const double S = fmax(naa + Ns[j] - 2.0 * dt[i], 0.0);
        double mv;
        if (b >= n) {
          mv = 0.0;
        } else if (square && b == arow) {
          mv = 1.0;
        } else if constexpr (KIND == GP_MATERN52) {
          const double u = sqrt(S);
          mv = fma(u, fma(u, 1.0 / 3.0, 1.0), 1.0) * exp(-u);
        } else {
          mv = exp(-0.5 * S);
        }
        mt[i] = mv;
      }
      // acc(row, column) += sum over the half's points of M(row, point) V(point, column)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        if (cb < ncb) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                mt[i], Vs[(16 * cb + lr) * kVLd + 16 * pb + 4 * i + lk], acc[cb], 0, 0, 0);
        }
      }
    }
  }
  // acc[cb][i]: row 16 wave + lk + 4 i, column 16 cb + lr -> LDS tile [column][row]
  __syncthreads();
  double* const Os = buf;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    if (cb < ncb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) Os[(16 * cb + lr) * kOLd + 16 * wave + lk + 4 * i] = acc[cb][i];
    }
  }
  __syncthreads();
  const int64_t a = a0 + lane;
  if (a >= m) return;
  for (int c = wave; c < tc; c += 4) {
    double y = sf * Os[c * kOLd + lane];
    if (square) y = fma(noise, V[(int64_t)(c0 + c) * ldv + a], y);
    out[(int64_t)(c0 + c) * ldo + a] = y;
  }
}

// Feature scales of the FP64 form: Matern sqrt5 / l (so that r^2 -> u^2, u = sqrt5 r), RBF 1 / l.
static Scale make_scale64(const gp_kernel* kern) {
  Scale s{};
  const double c = kern->kind == GP_MATERN52 ? std::sqrt(5.0) : 1.0;
  for (int j = 0; j < kern->d; ++j) s.s[j] = c / kern->lengthscale[j];
  return s;
}

template <int DP>
static void launch_fp64(int kind, dim3 grid, const KmmPlan& p, const double* V, int64_t ldv, int t, double* out,
                        int64_t ldo, hipStream_t st) {
  if (kind == GP_MATERN52)
    sweep_fp64_kernel<DP, GP_MATERN52><<<grid, 256, 0, st>>>(p.x64, p.nb64, p.n, p.z64, p.na64, p.m, p.d, p.sc64, V,
                                                             ldv, t, p.sf, p.noise, p.square ? 1 : 0, out, ldo);
  else
    sweep_fp64_kernel<DP, GP_RBF><<<grid, 256, 0, st>>>(p.x64, p.nb64, p.n, p.z64, p.na64, p.m, p.d, p.sc64, V, ldv,
                                                        t, p.sf, p.noise, p.square ? 1 : 0, out, ldo);
}

static hipError_t sweep_fp64(const KmmPlan& p, const double* V, int64_t ldv, int t, double* out, int64_t ldo,
                             hipStream_t st) {
  if (!p.x64 || !p.z64 || !V || !out || t < 1) return hipErrorInvalidValue;
  dim3 grid((unsigned)((p.m + kF64Rows - 1) / kF64Rows), (unsigned)((t + kF64Cols - 1) / kF64Cols));
  const int dp = (p.d + 15) / 16 * 16;
  switch (dp) {
    case 16: launch_fp64<16>(p.kind, grid, p, V, ldv, t, out, ldo, st); break;
    case 32: launch_fp64<32>(p.kind, grid, p, V, ldv, t, out, ldo, st); break;
    case 48: launch_fp64<48>(p.kind, grid, p, V, ldv, t, out, ldo, st); break;
    case 64: launch_fp64<64>(p.kind, grid, p, V, ldv, t, out, ldo, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

double profile_coordinate_scale(int kind) {
  return kind == GP_MATERN52 ? std::sqrt(5.0) * M_LOG2E : std::sqrt(0.5 * M_LOG2E);
}

static Scale make_scale(const gp_kernel* kern) {
  Scale s{};
  const double c = profile_coordinate_scale(kern->kind);
  for (int j = 0; j < kern->d; ++j) s.s[j] = c / kern->lengthscale[j];
  return s;
}

// set_centre: P is the b stream (the training points), whose column means become
// the centre of the mixed form's coordinates (p.ctr); otherwise P is query rows,
// prepared against the centre already in p.ctr.
static hipError_t prep_points(const KmmPlan& p, const Scale& sc, const double* P, int64_t rows,
                              int64_t rows_pad, void* xr, void* xc, float* nr, float* nc, bool set_centre,
                              hipStream_t st) {
  if (!p.nrm64 || !P || (!xr && !xc)) return hipErrorInvalidValue;
  const int mixed = p.precision == GP_PREC_BF16X3;
  if (mixed && (!p.ctr || (set_centre && !p.cpart))) return hipErrorInvalidValue;
  if (mixed && set_centre) {
    const hipError_t e = column_means(P, rows, p.d, p.cpart, p.ctr, st);
    if (e != hipSuccess) return e;
  }
  const int thr = 256;
  prep_norm_kernel<<<(unsigned)((rows_pad + thr - 1) / thr), thr, 0, st>>>(P, rows, rows_pad, p.d, sc, mixed,
                                                                           mixed ? p.ctr : nullptr, p.nrm64);
  const int64_t nblk = rows_pad / 16;
  const int64_t total = nblk * p.ks * 64;
  if (mixed) {
    prep_frag_f16x3_kernel<<<(unsigned)((total + thr - 1) / thr), thr, 0, st>>>(
        P, p.nrm64, p.ctr, rows, nblk, p.d, p.ks, sc, (bf16x8*)xr, (bf16x8*)xc);
  } else {
    prep_frag_fp32_kernel<<<(unsigned)((total + thr - 1) / thr), thr, 0, st>>>(
        P, p.nrm64, rows, nblk, p.d, p.ks, sc, (f32x4*)xr, (f32x4*)xc, nr, nc);
  }
  return hipGetLastError();
}

hipError_t kmm_prepare(KmmPlan& p, const gp_kernel* kern, const double* X, const double* Z,
                       hipStream_t st) {
  if (p.precision == GP_PREC_FP64) {
    if (!X || (!p.square && !Z) || !p.sc64) return hipErrorInvalidValue;
    const Scale s64 = make_scale64(kern);
    p.x64 = X;
    p.z64 = p.square ? X : Z;
    const int thr = 256;
    prep_fp64_kernel<<<(unsigned)((std::max<int64_t>(p.n, p.d) + thr - 1) / thr), thr, 0, st>>>(X, p.n, p.d, s64,
                                                                                              p.sc64, p.nb64);
    if (!p.square)
      prep_fp64_kernel<<<(unsigned)((p.m + thr - 1) / thr), thr, 0, st>>>(Z, p.m, p.d, s64, nullptr, p.na64);
    return hipGetLastError();
  }
  const Scale sc = make_scale(kern);
  if (p.square) {
    // one pass gives both sides; rows up to max(npad, mpad) so xc covers mpad
    const int64_t rows_pad = std::max(p.npad, p.mpad);
    return prep_points(p, sc, X, p.n, rows_pad, p.xr, p.xc, p.nrm_b, p.nrm_a, true, st);
  }
  hipError_t e = kmm_prepare_rows(p, kern, X, st);
  if (e != hipSuccess) return e;
  return kmm_prepare_cols(p, kern, Z, st);
}

hipError_t kmm_prepare_rows(KmmPlan& p, const gp_kernel* kern, const double* X, hipStream_t st) {
  if (p.precision == GP_PREC_FP64) return hipErrorInvalidValue;
  return prep_points(p, make_scale(kern), X, p.n, p.npad, p.xr, nullptr, p.nrm_b, nullptr, true, st);
}

hipError_t kmm_prepare_cols(KmmPlan& p, const gp_kernel* kern, const double* Z, hipStream_t st) {
  if (p.precision == GP_PREC_FP64) return hipErrorInvalidValue;
  return prep_points(p, make_scale(kern), Z, p.m, p.mpad, nullptr, p.xc, nullptr, p.nrm_a, false, st);
}

hipError_t prep_dist(const gp_kernel* kern, const double* X, int64_t n, int64_t rows_pad, int ks, const double* ctr,
                     void* xr, void* xc, double* nrm64, hipStream_t st) {
  if (!X || !ctr || !nrm64 || (!xr && !xc) || ks * 32 < 3 * kern->d + 6 || rows_pad % 64 != 0)
    return hipErrorInvalidValue;
  const Scale sc = make_scale(kern);
  const int thr = 256;
  prep_norm_kernel<<<(unsigned)((rows_pad + thr - 1) / thr), thr, 0, st>>>(X, n, rows_pad, kern->d, sc, 1, ctr,
                                                                           nrm64);
  const int64_t nblk = rows_pad / 16;
  const int64_t total = nblk * ks * 64;
  prep_frag_f16x3_kernel<<<(unsigned)((total + thr - 1) / thr), thr, 0, st>>>(X, nrm64, ctr, n, nblk, kern->d, ks,
                                                                             sc, (bf16x8*)xr, (bf16x8*)xc);
  return hipGetLastError();
}


template <int KS>
static void launch_one(bool mixed, int nt, int kind, dim3 grid, const SweepArgs& a, hipStream_t st);

// BF16X3 K steps (32 wide) and FP32 K groups (16 wide) that are instantiated.
static bool dispatch_ks(int ks, int nt, int kind, bool mixed, dim3 grid, const SweepArgs& a,
                        hipStream_t st) {
  if (mixed) {
    switch (ks) {
      case 2: launch_one<2>(true, nt, kind, grid, a, st); return true;
      case 4: launch_one<4>(true, nt, kind, grid, a, st); return true;
      case 5: launch_one<5>(true, nt, kind, grid, a, st); return true;
      case 7: launch_one<7>(true, nt, kind, grid, a, st); return true;
      case 13: launch_one<13>(true, nt, kind, grid, a, st); return true;
      default: return false;
    }
  }
  switch (ks) {
    case 1: launch_one<1>(false, nt, kind, grid, a, st); return true;
    case 2: launch_one<2>(false, nt, kind, grid, a, st); return true;
    case 3: launch_one<3>(false, nt, kind, grid, a, st); return true;
    case 4: launch_one<4>(false, nt, kind, grid, a, st); return true;
    case 8: launch_one<8>(false, nt, kind, grid, a, st); return true;
    default: return false;
  }
}

template <int KS, int NT, int KIND>
static void launch_form(bool mixed, dim3 grid, const SweepArgs& a, hipStream_t st) {
  if constexpr (KS == 2 || KS == 4 || KS == 5 || KS == 7 || KS == 13) {
    if (mixed) {
      sweep_bf16x3_kernel<KS, NT, KIND><<<grid, 256, 0, st>>>(a);
      return;
    }
  }
  if constexpr (KS == 1 || KS == 2 || KS == 3 || KS == 4 || KS == 8) {
    if (!mixed) sweep_fp32_kernel<KS, NT, KIND><<<grid, 256, 0, st>>>(a);
  }
}

template <int KS>
static void launch_one(bool mixed, int nt, int kind, dim3 grid, const SweepArgs& a, hipStream_t st) {
  const bool m52 = kind == GP_MATERN52;
  switch (nt) {
    case 1: m52 ? launch_form<KS, 1, GP_MATERN52>(mixed, grid, a, st) : launch_form<KS, 1, GP_RBF>(mixed, grid, a, st); break;
    case 2: m52 ? launch_form<KS, 2, GP_MATERN52>(mixed, grid, a, st) : launch_form<KS, 2, GP_RBF>(mixed, grid, a, st); break;
    case 3: m52 ? launch_form<KS, 3, GP_MATERN52>(mixed, grid, a, st) : launch_form<KS, 3, GP_RBF>(mixed, grid, a, st); break;
    default: m52 ? launch_form<KS, 4, GP_MATERN52>(mixed, grid, a, st) : launch_form<KS, 4, GP_RBF>(mixed, grid, a, st); break;
  }
}

hipError_t kmm_prepare_v(const KmmPlan& p, const double* V, int64_t ldv, int t, bool row_independent,
                         hipStream_t st, const double* col0) {
  if (t < 1 || t > p.tmax || !p.vf || !V) return hipErrorInvalidValue;
  const int ntb = (t + 15) / 16;
  const SplitChoice sc = choose_split(p.npad, p.mpad, ntb, row_independent, p.ks, p.precision == GP_PREC_BF16X3);
  const int ntb_alloc = sc.groups * sc.nt;  // vf holds whole launch groups (zero padded)
  const int thr = 256;
  if (p.precision == GP_PREC_BF16X3) {
    if (!p.vscale || !p.vinv || !p.vpart) return hipErrorInvalidValue;
    vmax_partial_kernel<<<dim3(kVParts, (unsigned)t), 256, 0, st>>>(V, ldv, col0, p.n, p.vpart);
    vscale_kernel<<<(unsigned)((t + 63) / 64), 64, 0, st>>>(p.vpart, t, p.vscale, p.vinv);
    const int64_t total = p.nchunks * ntb_alloc * 64;
    prep_v_f16x3_kernel<<<(unsigned)((total + thr - 1) / thr), thr, 0, st>>>(V, ldv, col0, p.vscale, p.n, t,
                                                                              p.nchunks, ntb_alloc, (bf16x8*)p.vf);
  } else {
    const int64_t total = p.nchunks * ntb_alloc * 2 * 64;
    prep_v_fp32_kernel<<<(unsigned)((total + thr - 1) / thr), thr, 0, st>>>(V, ldv, col0, p.n, t, p.nchunks,
                                                                             ntb_alloc, (f32x4*)p.vf);
  }
  return hipGetLastError();
}

template <int KS>
static void launch_wide(int kind, dim3 grid, const WideArgs& a, hipStream_t st) {
  if (kind == GP_MATERN52)
    wide_cross_bf16x3_kernel<KS, GP_MATERN52><<<grid, 256, 0, st>>>(a);
  else
    wide_cross_bf16x3_kernel<KS, GP_RBF><<<grid, 256, 0, st>>>(a);
}

// Row-independent BF16X3 cross products (prediction): the wide sweep, same splits and partials.
static hipError_t kmm_sweep_wide(const KmmPlan& p, int t, const SplitChoice& sc, double* out, int64_t ldo,
                                 hipStream_t st) {
  WideArgs a;
  a.xr = p.xr;
  a.xc = p.xc;
  a.vf = p.vf;
  a.part = p.part;
  a.mpad = p.mpad;
  a.nchunks = p.nchunks;
  a.cps = sc.cps;
  a.nsplit = sc.nsplit;
  a.ntb = (t + 15) / 16;
  a.vstride = sc.groups * sc.nt;  // the V fragments hold whole launch groups
  a.tpad = a.ntb * 16;
  a.rgroups = (int)std::max<int64_t>(1, (p.m + 63) / 64);  // live 64-row groups (mpad is a multiple of 256)
  a.f32part = sc.cps <= kFlush ? 1 : 0;
  const dim3 grid((unsigned)(a.rgroups * ((sc.nsplit + 7) / 8 * 8)));
  SweepTiming::Rec rec{};
  bool timed = false;
  {
    std::lock_guard<std::mutex> g(timing().mu);
    timed = timing().on && !p.no_timing;
  }
  if (timed) {
    hipError_t e = hipEventCreate(&rec.a);
    if (e == hipSuccess) e = hipEventCreate(&rec.b);
    if (e == hipSuccess) e = hipEventRecord(rec.a, st);
    if (e != hipSuccess) return e;
  }
  switch (p.ks) {
    case 2: launch_wide<2>(p.kind, grid, a, st); break;
    case 4: launch_wide<4>(p.kind, grid, a, st); break;
    case 5: launch_wide<5>(p.kind, grid, a, st); break;
    case 7: launch_wide<7>(p.kind, grid, a, st); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (timed) {
    e = hipEventRecord(rec.b, st);
    if (e != hipSuccess) return e;
    rec.flops = 2.0 * (double)p.m * (double)p.n * (double)(p.d + t);
    rec.n = p.n;
    rec.m = p.m;
    rec.t = t;
    std::lock_guard<std::mutex> g(timing().mu);
    timing().recs.push_back(rec);
  }
  const dim3 egrid((unsigned)((p.m + 63) / 64), (unsigned)t);
  if (a.f32part)
    wide_epilogue_kernel<float><<<egrid, 256, 0, st>>>((const float*)p.part, sc.nsplit, a.tpad, p.mpad, p.m, p.sf,
                                                       p.vinv, out, ldo);
  else
    wide_epilogue_kernel<double><<<egrid, 256, 0, st>>>(p.part, sc.nsplit, a.tpad, p.mpad, p.m, p.sf, p.vinv, out,
                                                        ldo);
  return hipGetLastError();
}

hipError_t kmm_sweep(const KmmPlan& p, int t, const double* Vdiag, int64_t ldv, double* out, int64_t ldo,
                     hipStream_t st, bool row_independent) {
  if (t < 1 || t > p.tmax) return hipErrorInvalidValue;
  if (!p.xr || !p.xc || !p.nrm_b || !p.nrm_a || !p.vf || !p.part || !out) return hipErrorInvalidValue;
  const bool mixed = p.precision == GP_PREC_BF16X3;
  const int ntb = (t + 15) / 16;
  const SplitChoice sc = choose_split(p.npad, p.mpad, ntb, row_independent, p.ks, p.precision == GP_PREC_BF16X3);
  if (row_independent && mixed && !p.square && ntb <= 4 * kWideNB && p.ks <= 7)
    return kmm_sweep_wide(p, t, sc, out, ldo, st);
  SweepArgs a;
  a.xr = p.xr;
  a.xc = p.xc;
  a.nrm_b = p.nrm_b;
  a.nrm_a = p.nrm_a;
  a.vf = p.vf;
  a.part = p.part;
  a.mpad = p.mpad;
  a.nchunks = p.nchunks;
  a.cps = sc.cps;
  a.ntb = sc.groups * sc.nt;
  a.tpad = sc.tpad;
  a.square = p.square ? 1 : 0;
  const int na = na_of(p.ks, sc.nt, mixed);
  dim3 grid((unsigned)(p.mpad / (64 * na)), (unsigned)sc.nsplit, (unsigned)sc.groups);
  SweepTiming::Rec rec{};
  bool timed = false;
  {
    std::lock_guard<std::mutex> g(timing().mu);
    timed = timing().on && !p.no_timing;
  }
  if (timed) {
    hipError_t e = hipEventCreate(&rec.a);
    if (e == hipSuccess) e = hipEventCreate(&rec.b);
    if (e == hipSuccess) e = hipEventRecord(rec.a, st);
    if (e != hipSuccess) return e;
  }
  if (!dispatch_ks(p.ks, sc.nt, p.kind, mixed, grid, a, st)) return hipErrorInvalidValue;
  if (timed) {
    hipError_t e = hipEventRecord(rec.b, st);
    if (e != hipSuccess) return e;
    rec.flops = 2.0 * (double)p.m * (double)p.n * (double)(p.d + t);
    rec.n = p.n;
    rec.m = p.m;
    rec.t = t;
    std::lock_guard<std::mutex> g(timing().mu);
    timing().recs.push_back(rec);
  }
  const int thr = 256;
  const int64_t total = p.m * t;
  kmm_epilogue_kernel<<<(unsigned)((total + thr - 1) / thr), thr, 0, st>>>(
      p.part, sc.nsplit, sc.tpad, p.mpad, p.m, t, p.sf, p.square ? p.sf + p.noise : 0.0, mixed ? p.vinv : nullptr,
      p.square ? Vdiag : nullptr, ldv, out, ldo);
  return hipGetLastError();
}

hipError_t kmm_apply(const KmmPlan& p, const double* V, int64_t ldv, int t, double* out, int64_t ldo,
                     hipStream_t st, bool row_independent) {
  if (p.precision == GP_PREC_FP64) return sweep_fp64(p, V, ldv, t, out, ldo, st);
  hipError_t e = kmm_prepare_v(p, V, ldv, t, row_independent, st);
  if (e != hipSuccess) return e;
  return kmm_sweep(p, t, V, ldv, out, ldo, st, row_independent);
}

}  // namespace gpk

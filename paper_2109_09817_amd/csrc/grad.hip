// Hyperparameter-derivative bilinear forms (the gradient of the log marginal
// likelihood, Eq. 2, as estimated by mBCG in Sec. 3.2):
//
//   g_j = sum_c w_c U_c^T (dK_hat/dlog theta_j) W_c,   theta = (l_1..l_d, s_f, sigma^2)
//
// With C_ab = sum_c w_c U_ac W_bc and M = psi(r) (.) C,
//   g_{l_j} = sum_ab M_ab (x~_aj - x~_bj)^2
//           = sum_a [ x~_aj^2 sum_b M_ab + sum_b M_ab x~_bj^2 - 2 x~_aj sum_b M_ab x~_bj ]
//   g_{s_f} = sum_ab K_ab C_ab ,   g_{sigma^2} = sigma^2 sum_c w_c U_c.W_c
// (x~ = (x - mu) / l; the shift mu cancels in every difference and only
// reduces rounding).  Tiles are recomputed, never stored.  The diagonal a = b
// contributes only to g_{s_f} (s_f C_aa) and is added exactly in FP64.
//
// FP32 form: every (16 rows a) x (32 points b) tile of the full matrix on the
// FP32 matrix cores: the distance tile (as in the K_hat V sweep), the tile of
// C, and M times the 2d+1 columns [x~ | 1 | x~^2] of the b points.
// BF16X3 form: the pairs a < b only, with the symmetric part of C (grad_tri.h).
#include <algorithm>
#include <vector>

#include "api_common.h"
#include "grad_tri.h"
#include "mfma_bf16.h"
#include "solver.h"

namespace gpk {

constexpr int kGradFlush = 32;

// float4 fragments of t columns of a column-major block, optionally weighted:
// (blk, q, lane) -> w_c M[c*ld + p] for c = 16 q + 4 s + lane/16, p = 16 blk + lane%16.
__global__ void prep_colfrag_kernel(const double* __restrict__ M, int64_t ld, int64_t n, int t,
                                    const double* __restrict__ w, int64_t nblk, int KQ, f32x4* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nblk * KQ * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;
  const int q = (int)(rest % KQ);
  const int64_t blk = rest / KQ;
  const int64_t p = blk * 16 + (lane & 15);
  const int g = lane >> 4;
  f32x4 o;
  for (int s = 0; s < 4; ++s) {
    const int c = 16 * q + 4 * s + g;
    o[s] = (p < n && c < t) ? (float)((w ? w[c] : 1.0) * M[(int64_t)c * ld + p]) : 0.f;
  }
  out[idx] = o;
}

// Fragments of the 2d+1 columns [x~ | 1 | x~^2] in the layout of the FP32
// product's B operand: (chunk, cb, tile, lane) -> float4 over i of column
// 16 cb + lane%16 at point 32 chunk + 16 tile + 4 (lane/16) + i.
__global__ void prep_gv_kernel(const double* __restrict__ X, int64_t n, int d, Scale inv_ell,
                               const double* __restrict__ mu, int64_t nchunks, int ncb, f32x4* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nchunks * ncb * 2 * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;
  const int tile = (int)(rest & 1);
  const int64_t cbch = rest >> 1;
  const int cb = (int)(cbch % ncb);
  const int64_t ch = cbch / ncb;
  const int col = 16 * cb + (lane & 15);
  const int g = lane >> 4;
  f32x4 o;
  for (int i = 0; i < 4; ++i) {
    const int64_t b = ch * 32 + 16 * tile + 4 * g + i;
    float v = 0.f;
    if (b < n) {
      if (col < d) {
        v = (float)((X[b * d + col] - mu[col]) * inv_ell.s[col]);
      } else if (col == d) {
        v = 1.f;
      } else if (col <= 2 * d) {
        const int j = col - d - 1;
        const double x = (X[b * d + j] - mu[j]) * inv_ell.s[j];
        v = (float)(x * x);
      }
    }
    o[i] = v;
  }
  out[idx] = o;
}

struct GradArgs {
  const f32x4* xr;   // b-stream distance fragments (-2 x^)
  const f32x4* xc;   // a-row distance fragments (x^)
  const float* nrm_b;
  const float* nrm_a;
  const f32x4* wf;   // b-stream fragments of W
  const f32x4* uf;   // a-row fragments of w (.) U
  const f32x4* gv;   // b-stream fragments of [x~ | 1 | x~^2]
  const double* X;
  const double* mu;
  Scale inv_ell;
  int d;
  int64_t n;
  int64_t mpad;
  int64_t nchunks;
  int64_t cps;
  double* part;      // per (block, split): d + 1 partial sums
};

template <int KQ, int KQC, int NG, int KIND>
__global__ __launch_bounds__(256, 2) void grad_sweep_kernel(GradArgs a) {
  __shared__ double sh_rows[4][16][NG * 16 + 1];
  __shared__ double sh_red[4][GP_MAX_D + 1];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int g = lane >> 4;
  const int64_t ablk = (int64_t)blockIdx.x * 4 + wave;  // one 16-row block per wave
  const bool live = ablk * 16 < a.mpad;

  f32x4 A[KQ], UA[KQC];
  float na = 0.f;
  if (live) {
#pragma unroll
    for (int q = 0; q < KQ; ++q) A[q] = a.xc[(ablk * KQ + q) * 64 + lane];
#pragma unroll
    for (int q = 0; q < KQC; ++q) UA[q] = a.uf[(ablk * KQC + q) * 64 + lane];
    na = a.nrm_a[ablk * 16 + (lane & 15)];
  }
  double acc64[NG][4];
#pragma unroll
  for (int nb = 0; nb < NG; ++nb)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc64[nb][i] = 0.0;
  double sfsum = 0.0;

  const int64_t c_begin = (int64_t)blockIdx.y * a.cps;
  const int64_t c_end = c_begin + a.cps < a.nchunks ? c_begin + a.cps : a.nchunks;
  if (live) {
    for (int64_t c0 = c_begin; c0 < c_end; c0 += kGradFlush) {
      const int64_t c1 = c0 + kGradFlush < c_end ? c0 + kGradFlush : c_end;
      f32x4 acc[NG];
#pragma unroll
      for (int nb = 0; nb < NG; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
      float sfacc = 0.f;
      for (int64_t ch = c0; ch < c1; ++ch) {
        f32x4 s[2], cm[2];
#pragma unroll
        for (int tl = 0; tl < 2; ++tl) {
          const int64_t bblk = 2 * ch + tl;
          s[tl] = *(const f32x4*)(a.nrm_b + bblk * 16 + 4 * g) + na;
          cm[tl] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int q = 0; q < KQ; ++q) {
            const f32x4 B = a.xr[(bblk * KQ + q) * 64 + lane];
#pragma unroll
            for (int e = 0; e < 4; ++e) s[tl] = __builtin_amdgcn_mfma_f32_16x16x4f32(B[e], A[q][e], s[tl], 0, 0, 0);
          }
#pragma unroll
          for (int q = 0; q < KQC; ++q) {
            const f32x4 Wb = a.wf[(bblk * KQC + q) * 64 + lane];
#pragma unroll
            for (int e = 0; e < 4; ++e) cm[tl] = __builtin_amdgcn_mfma_f32_16x16x4f32(Wb[e], UA[q][e], cm[tl], 0, 0, 0);
          }
        }
        f32x4 Mv[2];
#pragma unroll
        for (int tl = 0; tl < 2; ++tl)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float m, psi;
            if constexpr (KIND == GP_MATERN52) {
              const float sv = __builtin_fmaxf(__builtin_fabsf(s[tl][i]), 1e-30f);
              const float y = __builtin_amdgcn_rsqf(sv);
              const float u0 = sv * y;
              const float u = __builtin_fmaf(__builtin_fmaf(-u0, u0, sv), 0.5f * y, u0);
              const float e = __builtin_amdgcn_exp2f(-u);
              m = __builtin_fmaf(__builtin_fmaf(u, kMaternC2, kMaternC1), u, 1.0f) * e;
              psi = __builtin_fmaf(u, kMaternC1, 1.0f) * e;
            } else {
              m = __builtin_amdgcn_exp2f(-__builtin_fabsf(s[tl][i]));
              psi = m;
            }
            const int64_t arow = ablk * 16 + (lane & 15);
            const int64_t brow = ch * 32 + 16 * tl + 4 * g + i;
            if (arow == brow) {
              m = 0.f;
              psi = 0.f;
            }
            sfacc = __builtin_fmaf(m, cm[tl][i], sfacc);
            Mv[tl][i] = psi * cm[tl][i];
          }
        const int64_t vbase = (ch * NG) * 2 * 64 + lane;
#pragma unroll
        for (int nb = 0; nb < NG; ++nb) {
          const f32x4 G0 = a.gv[vbase + (nb * 2 + 0) * 64];
          const f32x4 G1 = a.gv[vbase + (nb * 2 + 1) * 64];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(Mv[0][i], G0[i], acc[nb], 0, 0, 0);
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(Mv[1][i], G1[i], acc[nb], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int nb = 0; nb < NG; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc64[nb][i] += (double)acc[nb][i];
      sfsum += (double)sfacc;
    }
  }
  // rows of this wave: [MX (d) | rowsum | MX2 (d)] through LDS
#pragma unroll
  for (int nb = 0; nb < NG; ++nb)
#pragma unroll
    for (int i = 0; i < 4; ++i) sh_rows[wave][4 * g + i][16 * nb + (lane & 15)] = acc64[nb][i];
  __syncthreads();
  const int d = a.d;
  double gj = 0.0;
  if (live && lane < d) {
    const int j = lane;
    for (int r = 0; r < 16; ++r) {
      const int64_t arow = ablk * 16 + r;
      if (arow >= a.n) break;
      const double x = (a.X[arow * d + j] - a.mu[j]) * a.inv_ell.s[j];
      const double mx = sh_rows[wave][r][j];
      const double rs = sh_rows[wave][r][d];
      const double mx2 = sh_rows[wave][r][d + 1 + j];
      gj += x * x * rs + mx2 - 2.0 * x * mx;
    }
  }
  // lengthscale partials (lanes < d) and the s_f partial (all lanes) per wave
  double sfw = sfsum;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sfw += __shfl_down(sfw, off, 64);
  if (lane < d) sh_red[wave][lane] = gj;
  if (lane == 0) sh_red[wave][GP_MAX_D] = live ? sfw : 0.0;
  __syncthreads();
  const int64_t slot = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * (d + 1);
  if (threadIdx.x < d) {
    double s = 0.0;
    for (int w = 0; w < 4; ++w) s += sh_red[w][threadIdx.x];
    a.part[slot + threadIdx.x] = s;
  } else if (threadIdx.x == 64) {
    double s = 0.0;
    for (int w = 0; w < 4; ++w) s += sh_red[w][GP_MAX_D];
    a.part[slot + d] = s;
  }
}

__global__ void grad_final_kernel(const double* __restrict__ part, int64_t nparts, int dd, double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= dd) return;
  double s = 0.0;
  for (int64_t p = 0; p < nparts; ++p) s += part[p * dd + j];
  out[j] = s;
}

// ------------------------------------------------------------------ host side

// ------------------------------------------------------------ BF16X3 form
//
// The BF16X3 form runs the upper-triangle sweep of grad_tri.h: every unordered
// pair once, with the symmetric part of C.

__device__ __forceinline__ float bf16r(double x) { return (float)(__bf16)(float)x; }

// BF16X3 fragments of the 2t columns [M1 | M2] (weighted by w and, for point p,
// scaled by pscale[p] when given), K
// index 6t long.  A-operand role: [hi | hi | lo]; B-operand role: [hi | lo | hi],
// so that sum_K A B = hi.hi + hi.lo + lo.hi over the 2t columns.  Fragment
// (blk, q, lane) holds K = 32 q + 8 (lane/16) + j of point 16 blk + lane%16.
__global__ void prep_pairfrag_bf16x3_kernel(const double* __restrict__ M1, const double* __restrict__ M2,
                                            int64_t ld, int64_t n, int t, const double* __restrict__ w,
                                            const double* __restrict__ pscale, int64_t nblk, int KSC, int b_role,
                                            bf16x8* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nblk * KSC * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;
  const int q = (int)(rest % KSC);
  const int64_t blk = rest / KSC;
  const int64_t p = blk * 16 + (lane & 15);
  const int g = lane >> 4;
  const double ps = pscale && p < n ? pscale[p] : 1.0;
  bf16x8 o;
  for (int j = 0; j < 8; ++j) {
    const int k = 32 * q + 8 * g + j;
    float v = 0.f;
    if (p < n && k < 6 * t) {
      const int seg = k / (2 * t), cc = k - seg * 2 * t;
      const int c = cc < t ? cc : cc - t;
      const double* M = cc < t ? M1 : M2;
      const double x = ps * (w ? w[c] : 1.0) * M[(int64_t)c * ld + p];
      const float h = bf16r(x);
      const float l = bf16r(x - (double)h);
      v = b_role ? (seg == 1 ? l : h) : (seg == 2 ? l : h);
    }
    o[j] = (__bf16)v;
  }
  out[idx] = o;
}

// FP16 fragments of the 2 NJ column blocks [x~ | x~^2] (each d columns padded to
// 16 NJ), every column scaled by its power of two (scal[j], scal[d + j]), in
// the B-operand layout of the forms product: (chunk, cb, hl, lane) -> 8 FP16 (hi =
// RNE16(v), lo = RNE16(v - hi)) of column 16 cb + lane%16 at the points
// 32 chunk + vperm(lane/16, j).
__device__ __forceinline__ double f16r(double x) { return (double)(_Float16)(float)x; }

__global__ void prep_formfrag_f16x3_kernel(const double* __restrict__ X, int64_t n, int d, int nj,
                                           const double* __restrict__ inv_ell, const double* __restrict__ mu,
                                           const double* __restrict__ scal, int64_t nchunks,
                                           bf16x8* __restrict__ out) {
  const int ng = 2 * nj;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nchunks * ng * 64) return;
  const int lane = (int)(idx & 63);
  const int64_t rest = idx >> 6;  // ch * ng + cb
  const int cb = (int)(rest % ng);
  const int64_t ch = rest / ng;
  const bool square = cb >= nj;
  const int jj = 16 * (square ? cb - nj : cb) + (lane & 15);
  const int g = lane >> 4;
  const double sc = jj < d ? scal[(square ? d : 0) + jj] : 0.0;
  f16x8 hi, lo;
  for (int j = 0; j < 8; ++j) {
    const int64_t b = ch * 32 + vperm(g, j);
    double v = 0.0;
    if (b < n && jj < d) {
      const double x = (X[b * d + jj] - mu[jj]) * inv_ell[jj];
      v = (square ? x * x : x) * sc;
    }
    const double h = f16r(v);
    hi[j] = (_Float16)(float)h;
    lo[j] = (_Float16)(float)(v - h);
  }
  out[(rest * 2 + 0) * 64 + lane] = __builtin_bit_cast(bf16x8, hi);
  out[(rest * 2 + 1) * 64 + lane] = __builtin_bit_cast(bf16x8, lo);
}

// 2^e with e = 15 - E for x = f 2^E (f in [1/2, 1)): puts x in [2^14, 2^15); 1 for zero or non-finite x.
__device__ __forceinline__ int pow2_exponent(double x) {
  if (!(x > 0.0) || !(x <= 1.7976931348623157e308)) return 0;
  int E = 0;
  (void)frexp(x, &E);
  const int e = 15 - E;
  return e < -1022 ? -1022 : (e > 1023 ? 1023 : e);
}

// Column scalings of the forms product (layout in grad_tri.h), one block, thread j < d.
// nmax[0] is the largest squared norm of the prescaled, centred coordinates
// c (x - mean) / l of the distance operands, so that sqrt(nmax) / c bounds every
// |x~_j| = |x_j - mean_j| / l_j: one bound for all columns (a column's values then lie
// in FP16's normal range down to 2^-29 of it).
__global__ void grad_scales_kernel(const double* __restrict__ nmax, double c, int d, double* __restrict__ scal) {
  const int j = threadIdx.x;
  if (j >= d) return;
  const double bx = sqrt(nmax[0]) / c;
  const int ex = pow2_exponent(bx), esq = pow2_exponent(bx * bx);
  scal[j] = ldexp(1.0, ex);
  scal[d + j] = ldexp(1.0, esq);
  scal[2 * d + j] = ldexp(1.0, -ex);
  scal[3 * d + j] = ldexp(1.0, -esq);
}

// Group scalings of C^s: for each group of `grp` rows (one wave's rows: 16 or 32), s = 2^e
// for the largest row bound sum_c |w_c| (|U_ac| max|W_c| + |W_ac| max|U_c|) of its rows
// a < n (a group with none: 1); rs holds s for every row (the scale prep_pairfrag
// applies), binv 1 / s per group.  One thread per row (mpad rows, a multiple of grp, in
// blocks of 64 so that a group never straddles a wave); U, W column-major with leading
// dimension n.
__global__ __launch_bounds__(64) void grad_group_scale_kernel(const double* __restrict__ U,
                                                              const double* __restrict__ W, int64_t n, int64_t mpad,
                                                              int grp, int t, const double* __restrict__ w,
                                                              const double* __restrict__ umax,
                                                              const double* __restrict__ wmax,
                                                              double* __restrict__ rs, double* __restrict__ binv) {
  const int64_t a = (int64_t)blockIdx.x * 64 + threadIdx.x;
  double bound = 0.0;
  if (a < n)
    for (int c = 0; c < t; ++c)
      bound += fabs(w[c]) * (fabs(U[(int64_t)c * n + a]) * wmax[c] + fabs(W[(int64_t)c * n + a]) * umax[c]);
  for (int off = 1; off < grp; off <<= 1) bound = fmax(bound, __shfl_xor(bound, off, 64));
  const int e = pow2_exponent(bound);
  if (a < mpad) {
    rs[a] = ldexp(1.0, e);
    if (a % grp == 0) binv[a / grp] = ldexp(1.0, -e);
  }
}

// First level of the unit reduction: block b sums units [b kRedUnits, ...) per entry.
constexpr int kRedUnits = 512;
__global__ void grad_reduce_units_kernel(const double* __restrict__ part, int64_t nunits, int dd,
                                         double* __restrict__ out) {
  const int j = threadIdx.x;
  if (j >= dd) return;
  const int64_t u0 = (int64_t)blockIdx.x * kRedUnits;
  const int64_t u1 = u0 + kRedUnits < nunits ? u0 + kRedUnits : nunits;
  double s = 0.0;
  for (int64_t u = u0; u < u1; ++u) s += part[u * dd + j];
  out[(int64_t)blockIdx.x * dd + j] = s;
}

// Work units of the triangle sweep: for each row group R (`rows` rows), the
// chunks [R rows/32, nchunks) cut at multiples of cps, ordered by chunk segment
// then row group so that concurrently running workgroups stream the same chunks.
static int64_t tri_units(int64_t n, int64_t rows, int64_t nchunks, int64_t cps, std::vector<int2>* out) {
  const int64_t groups = (n + rows - 1) / rows;
  const int64_t segs = (nchunks + cps - 1) / cps;
  int64_t count = 0;
  for (int64_t k = 0; k < segs; ++k) {
    const int64_t seg_end = std::min((k + 1) * cps, nchunks);
    for (int64_t R = 0; R < groups; ++R) {
      const int64_t f = R * (rows / 32);
      if (f >= seg_end) break;
      if (out) out->push_back(int2{(int)R, (int)std::max(f, k * cps)});
      ++count;
    }
  }
  return count;
}

// Unit length in chunks: enough units to fill the GPU, and short enough that
// one chunk segment's staged data (chunk_bytes each) stays within an XCD's
// 4 MB L2 while the workgroups streaming it drift apart.
static int64_t tri_cps(int64_t n, int64_t rows, int64_t nchunks, int64_t chunk_bytes) {
  const int64_t groups = (n + rows - 1) / rows;
  const int64_t f_last = (groups - 1) * (rows / 32);
  const int64_t work = groups * nchunks - (f_last + rows / 32) * groups / 2;  // chunk visits, approximately
  const int64_t fit_l2 = (int64_t)(3 << 20) / chunk_bytes;
  return std::min<int64_t>(1024, std::max<int64_t>(32, std::min(work / 4096, fit_l2)));
}

// Column blocks of [x~ | 1 | x~^2] of the FP32 form, sized for the instantiated
// K groups so that the fragment buffer and the kernel's template agree for every d.
static int ncb_fp32(int kq) { return 2 * kq + 1; }  // d <= 16 kq

struct GradGeom {
  bool mixed;
  int ks, ksc, ncb;  // distance K steps, C K steps, form column blocks
  int nj;            // BF16X3: 16-column blocks of x~
  int64_t rows;      // BF16X3: rows per row group
  int64_t npad, mpad, nchunks;
  int64_t cps;       // chunks per split (FP32) / unit alignment (BF16X3)
  int64_t nsplit, nblk_x;  // FP32 form: full-matrix splits x row blocks
  int64_t nunits;          // BF16X3 form: triangle work units
  int64_t nparts() const { return mixed ? nunits : nsplit * nblk_x; }
};

static GradGeom grad_geom(int precision, int d, int64_t n, int t) {
  GradGeom g{};
  g.mixed = precision == GP_PREC_BF16X3;
  g.ks = g.mixed ? tri_ks_of(d) : kmm_ksteps(precision, d);
  g.npad = (n + 31) / 32 * 32;
  g.nchunks = g.npad / 32;
  if (g.mixed) {
    g.ksc = grad_tri_ksc(t);
    g.nj = (d + 15) / 16;
    g.ncb = 2 * g.nj;
    g.rows = g.ksc > 0 ? tri_rows(g.ks, g.ksc, g.nj) : 16 * kTriWaves;
    g.mpad = (n + g.rows - 1) / g.rows * g.rows;
    g.cps = tri_cps(n, g.rows, g.nchunks, (int64_t)(2 * g.ks + 2 * g.ksc + 2 * g.ncb) * 64 * 16);
    g.nunits = tri_units(n, g.rows, g.nchunks, g.cps, nullptr);
  } else {
    g.ksc = (t + 15) / 16;
    g.ncb = ncb_fp32(g.ks);
    g.mpad = (n + 255) / 256 * 256;
    g.nblk_x = g.mpad / 64;
    const int64_t want = std::max<int64_t>(1, (2048 + g.nblk_x - 1) / g.nblk_x);
    g.cps = std::max<int64_t>(2, (g.nchunks + want - 1) / want);
    g.nsplit = (g.nchunks + g.cps - 1) / g.cps;
  }
  return g;
}

// BF16X3 form: its own FP16 distance operands for the mpad rows (>= npad), at
// the sweep's K step count: b-side and a-side fragments and the FP64 norm scratch.
static size_t dist_bytes(const GradGeom& g) {
  return 2 * align256((size_t)g.mpad * g.ks * 64) + align256((size_t)g.mpad * 8);
}

size_t grad_ws_bytes(int precision, int d, int64_t n, int t) {
  const GradGeom g = grad_geom(precision, d, n, t);
  if (g.ks < 0 || g.ksc < 0) return 0;
  const int64_t nparts = g.nparts();
  size_t b = g.mixed ? dist_bytes(g) : kmm_plan_bytes(precision, d, n, n, true, 1);
  b += align256((size_t)std::max(g.npad, g.mpad) * g.ksc * 64);  // b-side C fragments
  b += align256((size_t)g.mpad * g.ksc * 64);                    // a-side C fragments
  b += align256((size_t)g.npad * g.ncb * 64);                    // form fragments (hi+lo or float4 pairs)
  b += align256((size_t)nparts * (d + 1) * 8);                   // partials
  b += align256((size_t)((nparts + kRedUnits - 1) / kRedUnits) * (d + 1) * 8);  // first-level sums
  b += align256((size_t)(d + 1) * 8);                            // reduced
  b += align256((size_t)t * 8) + 2 * align256((size_t)d * 8);    // weights, mean, 1/l
  b += align256((size_t)std::max<int64_t>(g.nunits, 1) * sizeof(int2));  // unit table
  b += align256(std::max((size_t)row_split(n, kDotBlocks).nblk * std::max(d, t), colmean_scratch_doubles(n, d)) *
                8);  // reductions, column means
  b += align256((size_t)t * 8);                                  // U_c . W_c
  if (g.mixed) {
    b += align256(column_absmax_scratch_doubles(t) * 8) + 2 * align256((size_t)t * 8);  // max |U_c|, max |W_c|
    b += align256(column_absmax_scratch_doubles(1) * 8) + align256(8) + align256((size_t)grad_scale_doubles(d) * 8);
    b += 2 * align256((size_t)g.mpad * 8);                                                      // row-group scales
  }
  return b + 4096;
}

template <int KQ, int KQC, int NG>
static void launch_grad3(int kind, dim3 grid, const GradArgs& a, hipStream_t st) {
  if (kind == GP_MATERN52)
    grad_sweep_kernel<KQ, KQC, NG, GP_MATERN52><<<grid, 256, 0, st>>>(a);
  else
    grad_sweep_kernel<KQ, KQC, NG, GP_RBF><<<grid, 256, 0, st>>>(a);
}

template <int KQ, int KQC>
static bool launch_grad2(int ng, int kind, dim3 grid, const GradArgs& a, hipStream_t st) {
  constexpr int NG = 2 * KQ + 1;
  if (ng != NG) return false;
  launch_grad3<KQ, KQC, NG>(kind, grid, a, st);
  return true;
}

template <int KQ>
static bool launch_grad1(int kqc, int ng, int kind, dim3 grid, const GradArgs& a, hipStream_t st) {
  switch (kqc) {
    case 1: return launch_grad2<KQ, 1>(ng, kind, grid, a, st);
    case 2: return launch_grad2<KQ, 2>(ng, kind, grid, a, st);
    case 3: return launch_grad2<KQ, 3>(ng, kind, grid, a, st);
    case 4: return launch_grad2<KQ, 4>(ng, kind, grid, a, st);
    default: return false;
  }
}

int run_kmm_grad(const gp_kernel* kern, int precision, const double* X, int64_t n, const double* U, int64_t ldu,
                 const double* W, int64_t ldw, int t, const double* colw, double* grad, void* ws, size_t ws_bytes,
                 hipStream_t st) {
  const int d = kern->d;
  const GradGeom g = grad_geom(precision, d, n, t);
  if (g.ks < 0 || g.ksc < 0) return fail(GP_EINVAL, "gp_kmm_grad: unsupported d=%d or t=%d", d, t);
  const size_t kb = g.mixed ? dist_bytes(g) : kmm_plan_bytes(precision, d, n, n, true, 1);
  KmmPlan plan;
  if (!g.mixed && !kmm_plan_init(plan, kern, precision, n, n, true, 1, ws, kb))
    return fail(GP_EWORKSPACE, "gp_kmm_grad: workspace too small");
  if (ws_bytes < align256(kb)) return fail(GP_EWORKSPACE, "gp_kmm_grad: workspace too small");
  const int64_t nparts = g.nparts();
  const int64_t nred = (nparts + kRedUnits - 1) / kRedUnits;
  Carve cv((char*)ws + align256(kb), ws_bytes - align256(kb));
  char* wf = cv.take<char>((size_t)std::max(g.npad, g.mpad) * g.ksc * 64);
  char* uf = cv.take<char>((size_t)g.mpad * g.ksc * 64);
  char* gv = cv.take<char>((size_t)g.npad * g.ncb * 64);
  double* part = cv.take<double>((size_t)nparts * (d + 1));
  double* part2 = cv.take<double>((size_t)nred * (d + 1));
  double* red = cv.take<double>(d + 1);
  double* wdev = cv.take<double>(t);
  double* mu = cv.take<double>(d);
  double* inv_dev = cv.take<double>(d);
  int2* unit_dev = cv.take<int2>((size_t)std::max<int64_t>(g.nunits, 1));
  double* rpart = cv.take<double>(std::max((size_t)row_split(n, kDotBlocks).nblk * std::max(d, t),
                                           colmean_scratch_doubles(n, d)));
  double* uw = cv.take<double>(t);
  if (!uw) return fail(GP_EWORKSPACE, "gp_kmm_grad: workspace layout failed");
  double *cmpart = nullptr, *umax = nullptr, *wmax = nullptr, *fpart = nullptr, *scal = nullptr;
  double *rs = nullptr, *rinv = nullptr;
  if (g.mixed) {
    cmpart = cv.take<double>(column_absmax_scratch_doubles(t));
    umax = cv.take<double>(t);
    wmax = cv.take<double>(t);
    fpart = cv.take<double>(column_absmax_scratch_doubles(1) + 32);  // norm-max scratch, then the max at the end
    scal = cv.take<double>((size_t)grad_scale_doubles(d));
    rs = cv.take<double>((size_t)g.mpad);
    rinv = cv.take<double>((size_t)g.mpad);
    if (!rinv) return fail(GP_EWORKSPACE, "gp_kmm_grad: workspace layout failed");
  }
  std::vector<double> invh(d);
  for (int j = 0; j < d; ++j) invh[j] = 1.0 / kern->lengthscale[j];
  std::vector<int2> units;
  GPK_HIP(hipMemcpyAsync(wdev, colw, sizeof(double) * t, hipMemcpyHostToDevice, st));
  GPK_HIP(hipMemcpyAsync(inv_dev, invh.data(), sizeof(double) * d, hipMemcpyHostToDevice, st));
  GPK_HIP(column_means(X, n, d, rpart, mu, st));
  const unsigned thr = 256;
  char* dxr = (char*)ws;  // BF16X3 form: [b-side | a-side | norms] at the front of ws
  char* dxc = dxr + align256((size_t)g.mpad * g.ks * 64);
  double* dxn = (double*)(dxc + align256((size_t)g.mpad * g.ks * 64));
  if (g.mixed)
    GPK_HIP(prep_dist(kern, X, n, g.mpad, g.ks, mu, dxr, dxc, dxn, st));
  else
    GPK_HIP(kmm_prepare(plan, kern, X, nullptr, st));
  bool ok = false;
  if (g.mixed) {
    units.reserve((size_t)g.nunits);
    tri_units(n, g.rows, g.nchunks, g.cps, &units);
    GPK_HIP(hipMemcpyAsync(unit_dev, units.data(), sizeof(int2) * units.size(), hipMemcpyHostToDevice, st));
    const int64_t nbr = g.npad / 16, nba = g.mpad / 16;
    const int64_t tot = nbr * g.ksc * 64;
    // scalings of the FP16 forms product: column maxima of U, W and of the form coordinates
    GPK_HIP(column_absmax(U, n, n, t, cmpart, umax, st));
    GPK_HIP(column_absmax(W, n, n, t, cmpart, wmax, st));
    double* nmax = fpart + column_absmax_scratch_doubles(1);
    GPK_HIP(column_absmax(dxn, g.mpad, g.mpad, 1, fpart, nmax, st));
    grad_scales_kernel<<<1, 64, 0, st>>>(nmax, profile_coordinate_scale(kern->kind), d, scal);
    const int grp = (int)(g.rows / kTriWaves);  // rows per wave
    grad_group_scale_kernel<<<(unsigned)((g.mpad + 63) / 64), 64, 0, st>>>(U, W, n, g.mpad, grp, t, wdev, umax,
                                                                           wmax, rs, rinv);
    prep_pairfrag_bf16x3_kernel<<<(unsigned)((tot + thr - 1) / thr), thr, 0, st>>>(W, U, n, n, t, nullptr, nullptr,
                                                                                  nbr, g.ksc, 0, (bf16x8*)wf);
    const int64_t tot2 = nba * g.ksc * 64;
    prep_pairfrag_bf16x3_kernel<<<(unsigned)((tot2 + thr - 1) / thr), thr, 0, st>>>(U, W, n, n, t, wdev, rs, nba,
                                                                                   g.ksc, 1, (bf16x8*)uf);
    const int64_t tot3 = g.nchunks * g.ncb * 64;
    prep_formfrag_f16x3_kernel<<<(unsigned)((tot3 + thr - 1) / thr), thr, 0, st>>>(X, n, d, g.nj, inv_dev, mu, scal,
                                                                                  g.nchunks, (bf16x8*)gv);
    GPK_HIP(hipGetLastError());
    GradTriArgs a;
    a.xr = (const bf16x8*)dxr;
    a.xc = (const bf16x8*)dxc;
    a.cb = (const bf16x8*)wf;
    a.ca = (const bf16x8*)uf;
    a.gv = (const bf16x8*)gv;
    a.units = unit_dev;
    a.X = X;
    a.mu = mu;
    a.inv_ell = inv_dev;
    a.scal = scal;
    a.grpinv = rinv;
    a.d = d;
    a.n = n;
    a.nchunks = g.nchunks;
    a.cps = (int)g.cps;
    a.part = part;
    ok = kern->kind == GP_MATERN52 ? launch_grad_tri_matern(g.ks, g.nj, g.ksc, (unsigned)g.nunits, a, st)
                                   : launch_grad_tri_rbf(g.ks, g.nj, g.ksc, (unsigned)g.nunits, a, st);
  } else {
    Scale inv{};
    for (int j = 0; j < d; ++j) inv.s[j] = invh[j];
    const int64_t nbr = std::max(g.npad, g.mpad) / 16;
    const int64_t nba = g.mpad / 16;
    dim3 grid((unsigned)g.nblk_x, (unsigned)g.nsplit);
    const int64_t tot = nbr * g.ksc * 64;
    prep_colfrag_kernel<<<(unsigned)((tot + thr - 1) / thr), thr, 0, st>>>(W, ldw, n, t, nullptr, nbr, g.ksc,
                                                                          (f32x4*)wf);
    const int64_t tot2 = nba * g.ksc * 64;
    prep_colfrag_kernel<<<(unsigned)((tot2 + thr - 1) / thr), thr, 0, st>>>(U, ldu, n, t, wdev, nba, g.ksc,
                                                                           (f32x4*)uf);
    const int64_t tot3 = g.nchunks * g.ncb * 2 * 64;
    prep_gv_kernel<<<(unsigned)((tot3 + thr - 1) / thr), thr, 0, st>>>(X, n, d, inv, mu, g.nchunks, g.ncb,
                                                                       (f32x4*)gv);
    GPK_HIP(hipGetLastError());
    GradArgs a;
    a.xr = (const f32x4*)plan.xr;
    a.xc = (const f32x4*)plan.xc;
    a.nrm_b = plan.nrm_b;
    a.nrm_a = plan.nrm_a;
    a.wf = (const f32x4*)wf;
    a.uf = (const f32x4*)uf;
    a.gv = (const f32x4*)gv;
    a.X = X;
    a.mu = mu;
    a.inv_ell = inv;
    a.d = d;
    a.n = n;
    a.mpad = g.mpad;
    a.nchunks = g.nchunks;
    a.cps = g.cps;
    a.part = part;
    switch (g.ks) {
      case 1: ok = launch_grad1<1>(g.ksc, g.ncb, kern->kind, grid, a, st); break;
      case 2: ok = launch_grad1<2>(g.ksc, g.ncb, kern->kind, grid, a, st); break;
      case 3: ok = launch_grad1<3>(g.ksc, g.ncb, kern->kind, grid, a, st); break;
      case 4: ok = launch_grad1<4>(g.ksc, g.ncb, kern->kind, grid, a, st); break;
      default: ok = false;
    }
  }
  if (!ok) return fail(GP_EINVAL, "gp_kmm_grad: unsupported d=%d or t=%d (d <= 64, t <= 64)", d, t);
  GPK_HIP(hipGetLastError());
  grad_reduce_units_kernel<<<(unsigned)nred, 128, 0, st>>>(part, nparts, d + 1, part2);
  grad_final_kernel<<<1, 256, 0, st>>>(part2, nred, d + 1, red);
  GPK_HIP(coldot(U, W, n, t, uw, rpart, st));  // requires ldu == ldw == n
  std::vector<double> r(d + 1), uwh(t);
  GPK_HIP(hipMemcpyAsync(r.data(), red, sizeof(double) * (d + 1), hipMemcpyDeviceToHost, st));
  GPK_HIP(hipMemcpyAsync(uwh.data(), uw, sizeof(double) * t, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipStreamSynchronize(st));
  double diag = 0.0;
  for (int c = 0; c < t; ++c) diag += colw[c] * uwh[c];
  const double sf = kern->outputscale;
  const double psi_scale = kern->kind == GP_MATERN52 ? (5.0 / 3.0) * sf : sf;
  for (int j = 0; j < d; ++j) grad[j] = psi_scale * r[j];
  grad[d] = sf * (r[d] + diag);
  grad[d + 1] = kern->noise * diag;
  for (int j = 0; j < d + 2; ++j)
    if (!std::isfinite(grad[j])) return fail(GP_ENONFINITE, "gp_kmm_grad: non-finite gradient entry %d", j);
  return GP_OK;
}

}  // namespace gpk

using namespace gpk;

extern "C" int gp_kmm_grad(const gp_kernel* kern, int32_t precision, const double* X, int64_t n, const double* U,
                           int64_t ldu, const double* W, int64_t ldw, int32_t t, const double* colw, double* grad,
                           void* ws, size_t ws_bytes, void* stream) {
  GPK_TRY(check_kernel(kern));
  GPK_TRY(check_precision(precision));
  if (!X || !U || !W || !colw || !grad) return fail(GP_EINVAL, "gp_kmm_grad: NULL argument");
  if (n < 1) return fail(GP_EINVAL, "gp_kmm_grad: n must be >= 1");
  if (t < 1 || t > 64) return fail(GP_EINVAL, "gp_kmm_grad: t=%d outside [1, 64]", t);
  if (kern->d > 64) return fail(GP_EINVAL, "gp_kmm_grad: d=%d > 64 not supported", kern->d);
  if (ldu != n || ldw != n) return fail(GP_EINVAL, "gp_kmm_grad: ldu and ldw must equal n");
  for (int c = 0; c < t; ++c)
    if (!std::isfinite(colw[c])) return fail(GP_EINVAL, "gp_kmm_grad: colw[%d] not finite", c);
  GPK_TRY(check_ws(ws, ws_bytes, grad_ws_bytes(precision, kern->d, n, t), "gp_kmm_grad"));
  return run_kmm_grad(kern, precision, X, n, U, ldu, W, ldw, t, colw, grad, ws, ws_bytes, (hipStream_t)stream);
}

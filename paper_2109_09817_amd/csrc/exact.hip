// Exact GP on a subset (the AltBBMM hyperparameter protocol, Sec. 3.2 and
// Sec. 4: the hyperparameters come from a full GP on a random subset of the
// training molecules).  Dense FP64 throughout:
//
//   K_hat = L L^T (blocked right-looking Cholesky, 64-wide panels)
//   K_hat^{-1} = L^{-T} L^{-1}   (two blocked triangular solves against I,
//                                 each restricted to the lower triangle)
//   omega = K_hat^{-1} y
//   L(theta) = -1/2 y^T omega - sum_a log L_aa - n/2 log 2 pi       (Eq. 2)
//   dL/dlog theta = 1/2 sum_ab (omega omega^T - K_hat^{-1})_ab dK_hat_ab/dlog theta
//
// with dK/dlog l_j = psi(r) (dx_j / l_j)^2, psi(r) = (5/3) s_f (1 + sqrt5 r)
// e^{-sqrt5 r} (Matern-5/2; RBF: k), dK/dlog s_f = K and dK_hat/dlog sigma^2
// = sigma^2 I.  Every O(n^3) step is a sequence of 64 x 64 FP64 tile
// products C -= P Q (or C = P Q) over k <= 256 on the FP64 matrix cores, the
// panels staged in LDS; triangular solves against a 64 x 64 diagonal block
// multiply by its inverse (formed in LDS by one workgroup), so that they are
// tile products too.
#include <algorithm>
#include <cmath>
#include <vector>

#include "api_common.h"
#include "solver.h"

namespace gpk {

constexpr int kEb = 64;         // panel width and tile edge
constexpr int kExactMaxD = 64;  // features (the derivative sweep keeps a row of d in LDS)
constexpr int64_t kExactMaxN = 65536;

// ---------------------------------------------------------------- K_hat

// A[a n + b] = s_f m(r_ab) + sigma^2 [a == b] by direct differences.  sc[f]:
// Matern sqrt5 / l_f (so u = sqrt5 r), RBF 1 / l_f.
template <int KIND>
__global__ __launch_bounds__(256) void form_khat_kernel(const double* __restrict__ X, int64_t n, int d,
                                                        const double* __restrict__ sc, double sf, double noise,
                                                        double* __restrict__ A) {
  __shared__ double xa[kEb][33];
  __shared__ double xbT[32][kEb];
  const int64_t a0 = (int64_t)blockIdx.y * kEb, b0 = (int64_t)blockIdx.x * kEb;
  const int c = threadIdx.x % kEb, rb = threadIdx.x / kEb;
  double acc[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.0;
  for (int f0 = 0; f0 < d; f0 += 32) {
    __syncthreads();
    for (int e = threadIdx.x; e < kEb * 32; e += 256) {
      const int row = e / 32, f = e % 32;
      const bool fin = f0 + f < d;
      xa[row][f] = (a0 + row < n && fin) ? X[(a0 + row) * d + f0 + f] * sc[f0 + f] : 0.0;
      xbT[f][row] = (b0 + row < n && fin) ? X[(b0 + row) * d + f0 + f] * sc[f0 + f] : 0.0;
    }
    __syncthreads();
    for (int f = 0; f < 32; ++f) {
      const double xb = xbT[f][c];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double t = xa[rb + 4 * j][f] - xb;
        acc[j] = fma(t, t, acc[j]);
      }
    }
  }
  const int64_t b = b0 + c;
  if (b >= n) return;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int64_t a = a0 + rb + 4 * j;
    if (a >= n) continue;
    double m;
    if constexpr (KIND == GP_MATERN52) {
      const double u = sqrt(acc[j]);
      m = (1.0 + u + u * u / 3.0) * exp(-u);
    } else {
      m = exp(-0.5 * acc[j]);
    }
    A[a * n + b] = sf * m + (a == b ? noise : 0.0);
  }
}

// ---------------------------------------------------------------- Cholesky

// Load the factored diagonal block L[i0.., i0..] (ib rows) into LDS, identity-padded.
__device__ __forceinline__ void load_diag_block(const double* __restrict__ L, int64_t n, int64_t i0, int ib,
                                                double (*Ls)[kEb + 1]) {
  constexpr int kPer = kEb * kEb / 256;  // 256 threads
  double v[kPer];  // every load in flight before the first LDS write
#pragma unroll
  for (int it = 0; it < kPer; ++it) {
    const int e = (int)threadIdx.x + 256 * it, r = e / kEb, c = e % kEb;
    v[it] = (r < ib && c < ib) ? (c <= r ? L[(i0 + r) * n + i0 + c] : 0.0) : (r == c ? 1.0 : 0.0);
  }
#pragma unroll
  for (int it = 0; it < kPer; ++it) {
    const int e = (int)threadIdx.x + 256 * it;
    Ls[e / kEb][e % kEb] = v[it];
  }
}

// Xs = Ls^{-1} for a lower-triangular 64 x 64 Ls in LDS (zero above the
// diagonal), 256 threads: lanes 4j..4j+3 form column j by forward
// substitution against e_j, lane s keeping in registers the entries
// X[4q + s][j] of its residue class and summing their terms.  Entries not yet
// formed (and those above the diagonal) are zero, so every row takes the same
// 16 terms per lane and no index test; the four partial sums meet by shuffles.
// Ends with a barrier; Xs is complete (zero above the diagonal).
__device__ __forceinline__ void diag_inverse(const double (*Ls)[kEb + 1], double (*Xs)[kEb + 1]) {
  const int j = threadIdx.x >> 2, sub = threadIdx.x & 3;
  double x[kEb / 4];
#pragma unroll
  for (int q = 0; q < kEb / 4; ++q) x[q] = 0.0;
#pragma unroll
  for (int r = 0; r < kEb; ++r) {
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < kEb / 4; ++q) part = fma(Ls[r][4 * q + sub], x[q], part);
    part += __shfl_xor(part, 1);
    part += __shfl_xor(part, 2);
    const double xr = ((r == j ? 1.0 : 0.0) - part) / Ls[r][r];
    if ((r & 3) == sub) x[r >> 2] = xr;
  }
#pragma unroll
  for (int q = 0; q < kEb / 4; ++q) Xs[4 * q + sub][j] = x[q];
  __syncthreads();
}

// Unblocked Cholesky of the diagonal block A[j0.., j0..] (jb <= 64 rows) in
// LDS, the block outside jb padded with the identity; writes L (lower, zero
// above the diagonal) and, when Dinv is given, L^{-1} (64 x 64 row-major).  A
// pivot that is not positive records its global index + 1 in *info (the first
// one only) and continues with 1, so that every later step stays finite and
// bounded.
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ A, int64_t n, int64_t j0, int jb,
                                                         int* __restrict__ info, double* __restrict__ Dinv) {
  __shared__ double Ls[kEb][kEb + 1];
  __shared__ double Xs[kEb][kEb + 1];
  {
    constexpr int kPer = kEb * kEb / 256;
    double v[kPer];  // every load in flight before the first LDS write
#pragma unroll
    for (int it = 0; it < kPer; ++it) {
      const int e = (int)threadIdx.x + 256 * it, r = e / kEb, c = e % kEb;
      v[it] = (r < jb && c < jb) ? A[(j0 + r) * n + j0 + c] : (r == c ? 1.0 : 0.0);
    }
#pragma unroll
    for (int it = 0; it < kPer; ++it) {
      const int e = (int)threadIdx.x + 256 * it;
      Ls[e / kEb][e % kEb] = v[it];
    }
  }
  int bad = 0;  // thread 0 only
  for (int k = 0; k < kEb; ++k) {
    __syncthreads();
    double p = Ls[k][k];
    if (!(p > 0.0) || !isfinite(p)) {
      if (threadIdx.x == 0 && bad == 0) bad = (int)(j0 + k + 1);
      p = 1.0;
    }
    const double piv = sqrt(p);
    if ((int)threadIdx.x > k && (int)threadIdx.x < kEb) Ls[threadIdx.x][k] /= piv;
    __syncthreads();
    if (threadIdx.x == 0) Ls[k][k] = piv;
    // thread (wave w, lane c) updates entry c of the rows w + 4 it; every read
    // is issued unconditionally so that they overlap, the write is guarded
    const int c = threadIdx.x & (kEb - 1), w = threadIdx.x >> 6;
    const double lck = Ls[c][k];
#pragma unroll
    for (int it = 0; it < kEb / 4; ++it) {
      const int r = w + 4 * it;
      const double v = Ls[r][c] - Ls[r][k] * lck;
      if (c > k && c <= r) Ls[r][c] = v;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kEb * kEb; e += 256) {
    const int r = e / kEb, c = e % kEb;
    if (c > r) Ls[r][c] = 0.0;
    if (r < jb && c < jb) A[(j0 + r) * n + j0 + c] = c <= r ? Ls[r][c] : 0.0;
  }
  if (threadIdx.x == 0 && bad != 0 && *info == 0) *info = bad;
  if (!Dinv) return;
  __syncthreads();
  diag_inverse(Ls, Xs);
  for (int e = threadIdx.x; e < kEb * kEb; e += 256) Dinv[e] = Xs[e / kEb][e % kEb];
}

// Dinv + 64 * 64 * bi = L_ii^{-1} for every diagonal block bi (one workgroup each).
__global__ __launch_bounds__(256) void trtri_blocks_kernel(const double* __restrict__ L, int64_t n,
                                                           double* __restrict__ Dinv) {
  __shared__ double Ls[kEb][kEb + 1];
  __shared__ double Xs[kEb][kEb + 1];
  const int64_t i0 = (int64_t)blockIdx.x * kEb;
  load_diag_block(L, n, i0, (int)(n - i0 < kEb ? n - i0 : kEb), Ls);
  __syncthreads();
  diag_inverse(Ls, Xs);
  double* D = Dinv + (int64_t)blockIdx.x * kEb * kEb;
  for (int e = threadIdx.x; e < kEb * kEb; e += 256) D[e] = Xs[e / kEb][e % kEb];
}

// ---------------------------------------------------------------- tile updates

// C[R + r][Cc + c] -= sum_{k < kb} P(r, k) Q(k, c) (ASSIGN: =) over a set of
// 64 x 64 tiles (k in chunks of 64 staged in LDS in turn), with
//   P(r, k) = PT ? Pm[(p0 + k) ldp + pr + r] : Pm[(pr + r) ldp + p0 + k]
//   Q(k, c) = QT ? Qm[(qc + c) ldq + q0 + k] : Qm[(q0 + k) ldq + qc + c]
// where pr = R (pfix < 0) or pfix, and qc = Cc (qfix < 0) or qfix.  Tile (ti,
// tj) has R = rbase + 64 ti, Cc = cbase + 64 tj; LOWER enumerates tj <= ti <
// nrt, otherwise the nrt x nct rectangle.  Output rows and columns at or beyond
// n are skipped (their operands read as 0).  Every operand is read before
// the tile is written, so C's tile may be one of the operand tiles (never
// another workgroup's).  The products run on the FP64 matrix cores
// (v_mfma_f64_16x16x4: lane l supplies P(row l % 16, k l / 16) and Q(k l / 16,
// column l % 16) and receives rows l / 16 + 4 i of column l % 16); wave w
// owns the 32 x 32 quadrant (w / 2, w % 2).  Each operand keeps in LDS the
// orientation of its source rows, so that a wave's staging writes are
// contiguous: k-major [k][x] (pitch 80 doubles) when the source runs along x,
// x-major [x][k] (pitch 66) when it runs along k.  Both pitches put the 32
// lanes of a half-wave on distinct banks for the operand reads.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kKMajorLd = kEb + 16;
constexpr int kXMajorLd = kEb + 2;

template <bool KMAJOR>
__device__ __forceinline__ int lds_at(int k, int x) {
  return KMAJOR ? k * kKMajorLd + x : x * kXMajorLd + k;
}

template <bool PT, bool QT, bool LOWER, bool ASSIGN>
__global__ __launch_bounds__(256) void tile_update_kernel(const double* Pm, int64_t ldp, int64_t pfix, int64_t p0,
                                                          const double* Qm, int64_t ldq, int64_t qfix, int64_t q0,
                                                          double* Cm, int64_t n, int kb, int64_t rbase, int64_t cbase,
                                                          int nrt, int nct) {
  __shared__ double Ps[kEb * kKMajorLd];  // P(r, k) at lds_at<PT>(k, r)
  __shared__ double Qs[kEb * kKMajorLd];  // Q(k, c) at lds_at<!QT>(k, c)
  int64_t ti, tj;
  // Workgroup h runs on XCD h % 8; each XCD takes a contiguous run of tiles
  // (consecutive tiles of a tile row share their P panel in that XCD's L2).
  const int64_t T = LOWER ? (int64_t)nrt * (nrt + 1) / 2 : (int64_t)nrt * nct;
  const int64_t h = blockIdx.x, xcd = h & 7, q8 = T >> 3, rem8 = T & 7;
  const int64_t b = xcd * q8 + (xcd < rem8 ? xcd : rem8) + (h >> 3);
  if (LOWER) {
    ti = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
    while (ti * (ti + 1) / 2 > b) --ti;
    tj = b - ti * (ti + 1) / 2;
  } else {
    ti = b / nct;
    tj = b - ti * nct;
  }
  const int64_t R = rbase + kEb * ti, Cc = cbase + kEb * tj;
  const int64_t pr = pfix < 0 ? R : pfix, qc = qfix < 0 ? Cc : qfix;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = 32 * (wave >> 1), c0 = 32 * (wave & 1);
  const int lr = lane & 15, lk = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  // Each thread stages 16 elements of each operand per 64-wide k chunk; the
  // loads of chunk c + 1 are in flight while chunk c is multiplied.
  constexpr int kPer = kEb * kEb / 256;
  double pv[kPer], qv[kPer];
  auto load = [&](int kc) {
#pragma unroll
    for (int it = 0; it < kPer; ++it) {
      const int e = (int)threadIdx.x + 256 * it;
      const int x = e / kEb, y = e % kEb;  // consecutive threads: consecutive y
      {
        const int r = PT ? y : x, k = PT ? x : y;
        const bool ok = kc + k < kb && R + r < n;
        const int64_t kk = p0 + kc + k;
        pv[it] = ok ? (PT ? Pm[kk * ldp + pr + r] : Pm[(pr + r) * ldp + kk]) : 0.0;
      }
      {
        const int c = QT ? x : y, k = QT ? y : x;
        const bool ok = kc + k < kb && Cc + c < n;
        const int64_t kk = q0 + kc + k;
        qv[it] = ok ? (QT ? Qm[(qc + c) * ldq + kk] : Qm[kk * ldq + qc + c]) : 0.0;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int it = 0; it < kPer; ++it) {
      const int e = (int)threadIdx.x + 256 * it;
      const int x = e / kEb, y = e % kEb;
      Ps[PT ? lds_at<true>(x, y) : lds_at<false>(y, x)] = pv[it];
      Qs[QT ? lds_at<false>(y, x) : lds_at<true>(x, y)] = qv[it];
    }
  };
  load(0);
  for (int kc = 0; kc < kb; kc += kEb) {
    if (kc > 0) __syncthreads();  // every wave is done with the previous chunk
    store();
    __syncthreads();
    if (kc + kEb < kb) load(kc + kEb);
#pragma unroll 4
    for (int k = 0; k < kEb; k += 4) {
      const double a0 = Ps[lds_at<PT>(k + lk, r0 + lr)], a1 = Ps[lds_at<PT>(k + lk, r0 + 16 + lr)];
      const double q0v = Qs[lds_at<!QT>(k + lk, c0 + lr)], q1v = Qs[lds_at<!QT>(k + lk, c0 + 16 + lr)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, q0v, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, q1v, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, q0v, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, q1v, acc[1][1], 0, 0, 0);
    }
  }
  // the subtracting form reads all 16 of its C entries before writing any
  double old[2][2][4];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = R + r0 + 16 * rb + lk + 4 * i, col = Cc + c0 + 16 * cb + lr;
        old[rb][cb][i] = (!ASSIGN && row < n && col < n) ? Cm[row * n + col] : 0.0;
      }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = R + r0 + 16 * rb + lk + 4 * i, col = Cc + c0 + 16 * cb + lr;
        if (row < n && col < n) Cm[row * n + col] = ASSIGN ? acc[rb][cb][i] : old[rb][cb][i] - acc[rb][cb][i];
      }
}

template <bool PT, bool QT, bool LOWER, bool ASSIGN>
static hipError_t tile_update(const double* Pm, int64_t ldp, int64_t pfix, int64_t p0, const double* Qm, int64_t ldq,
                              int64_t qfix, int64_t q0, double* Cm, int64_t n, int kb, int64_t rbase, int64_t cbase,
                              int nrt, int nct, hipStream_t st) {
  const int64_t tiles = LOWER ? (int64_t)nrt * (nrt + 1) / 2 : (int64_t)nrt * nct;
  if (tiles <= 0) return hipSuccess;
  tile_update_kernel<PT, QT, LOWER, ASSIGN><<<(unsigned)tiles, 256, 0, st>>>(Pm, ldp, pfix, p0, Qm, ldq, qfix, q0, Cm,
                                                                             n, kb, rbase, cbase, nrt, nct);
  return hipGetLastError();
}

// General FP64 product C = A B (m x nn, row-major with ldc) on the matrix
// cores, 64 x 64 output tiles, k in chunks of 64 staged in LDS as in the tile
// kernel above:  A(i, k) = TA ? A[k lda + i] : A[i lda + k],
//                B(k, j) = TB ? B[j ldb + k] : B[k ldb + j].
// LOWER computes only the tiles with tj <= ti (m = nn).  Rows, columns and k
// beyond the matrices read as zero; nothing outside C's m x nn block is written.
template <bool TA, bool TB, bool LOWER>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const double* A, int64_t lda, const double* B, int64_t ldb,
                                                       double* C, int64_t ldc, int64_t m, int64_t nn, int64_t kk,
                                                       int nrt, int nct) {
  __shared__ double As[kEb * kKMajorLd];  // A(r, k) at lds_at<TA>(k, r)
  __shared__ double Bs[kEb * kKMajorLd];  // B(k, c) at lds_at<!TB>(k, c)
  const int64_t T = LOWER ? (int64_t)nrt * (nrt + 1) / 2 : (int64_t)nrt * nct;
  const int64_t h = blockIdx.x, xcd = h & 7, q8 = T >> 3, rem8 = T & 7;
  const int64_t b = xcd * q8 + (xcd < rem8 ? xcd : rem8) + (h >> 3);
  int64_t ti, tj;
  if (LOWER) {
    ti = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
    while (ti * (ti + 1) / 2 > b) --ti;
    tj = b - ti * (ti + 1) / 2;
  } else {
    ti = b / nct;
    tj = b - ti * nct;
  }
  const int64_t R = kEb * ti, Cc = kEb * tj;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r0 = 32 * (wave >> 1), c0 = 32 * (wave & 1);
  const int lr = lane & 15, lk = lane >> 4;
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  constexpr int kPer = kEb * kEb / 256;
  double av[kPer], bv[kPer];
  auto load = [&](int64_t kc) {
#pragma unroll
    for (int it = 0; it < kPer; ++it) {
      const int e = (int)threadIdx.x + 256 * it;
      const int x = e / kEb, y = e % kEb;  // consecutive threads: consecutive y
      {
        const int r = TA ? y : x, k = TA ? x : y;
        const bool ok = kc + k < kk && R + r < m;
        av[it] = ok ? (TA ? A[(kc + k) * lda + R + r] : A[(R + r) * lda + kc + k]) : 0.0;
      }
      {
        const int c = TB ? x : y, k = TB ? y : x;
        const bool ok = kc + k < kk && Cc + c < nn;
        bv[it] = ok ? (TB ? B[(Cc + c) * ldb + kc + k] : B[(kc + k) * ldb + Cc + c]) : 0.0;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int it = 0; it < kPer; ++it) {
      const int e = (int)threadIdx.x + 256 * it;
      const int x = e / kEb, y = e % kEb;
      As[TA ? lds_at<true>(x, y) : lds_at<false>(y, x)] = av[it];
      Bs[TB ? lds_at<false>(y, x) : lds_at<true>(x, y)] = bv[it];
    }
  };
  load(0);
  for (int64_t kc = 0; kc < kk; kc += kEb) {
    if (kc > 0) __syncthreads();  // every wave is done with the previous chunk
    store();
    __syncthreads();
    if (kc + kEb < kk) load(kc + kEb);
#pragma unroll 4
    for (int k = 0; k < kEb; k += 4) {
      const double a0 = As[lds_at<TA>(k + lk, r0 + lr)], a1 = As[lds_at<TA>(k + lk, r0 + 16 + lr)];
      const double b0 = Bs[lds_at<!TB>(k + lk, c0 + lr)], b1 = Bs[lds_at<!TB>(k + lk, c0 + 16 + lr)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = R + r0 + 16 * rb + lk + 4 * i, col = Cc + c0 + 16 * cb + lr;
        if (row < m && col < nn) C[row * ldc + col] = acc[rb][cb][i];
      }
}

static int ntiles(int64_t len) { return (int)((len + kEb - 1) / kEb); }

// A = L L^T in place (lower triangle; the diagonal blocks' upper parts are
// zeroed, the rest of the upper triangle is left as it was).  Two levels of
// blocking: 64-wide panels inside 256-wide super-panels.  A panel updates only
// the columns of its own super-panel; the trailing matrix beyond it takes the
// whole super-panel at once (k = 256), so that it is read and written once per
// 256 columns instead of once per 64.
constexpr int kSp = 4 * kEb;

static hipError_t cholesky(double* A, int64_t n, int* info, double* Dinv, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int64_t J0 = 0; J0 < n; J0 += kSp) {
    const int64_t Jend = std::min<int64_t>(n, J0 + kSp);
    for (int64_t j0 = J0; j0 < Jend; j0 += kEb) {
      const int jb = (int)std::min<int64_t>(kEb, n - j0);
      const int64_t rest = n - j0 - jb;
      potrf_diag_kernel<<<1, 256, 0, st>>>(A, n, j0, jb, info, rest > 0 ? Dinv : nullptr);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if (rest <= 0) return hipSuccess;
      // L21 = A21 L11^{-T} = A21 Dinv^T for every row below (jb = 64 here)
      e = tile_update<false, true, false, true>(A, n, -1, j0, Dinv, kEb, 0, 0, A, n, jb, j0 + jb, j0, ntiles(rest),
                                                1, st);
      if (e != hipSuccess) return e;
      // the rest of this super-panel's columns, [j0 + 64, Jend): the lower
      // triangle of its diagonal part, then the rows below the super-panel
      const int64_t wcols = Jend - j0 - jb;
      if (wcols > 0) {
        e = tile_update<false, true, true, false>(A, n, -1, j0, A, n, -1, j0, A, n, jb, j0 + jb, j0 + jb,
                                                  ntiles(wcols), 0, st);
        if (e != hipSuccess) return e;
        if (n > Jend) {
          e = tile_update<false, true, false, false>(A, n, -1, j0, A, n, -1, j0, A, n, jb, Jend, j0 + jb,
                                                     ntiles(n - Jend), ntiles(wcols), st);
          if (e != hipSuccess) return e;
        }
      }
    }
    // A22 -= L21 L21^T over the lower tiles beyond the super-panel, k = Jend - J0
    if (n > Jend) {
      e = tile_update<false, true, true, false>(A, n, -1, J0, A, n, -1, J0, A, n, (int)(Jend - J0), Jend, Jend,
                                                ntiles(n - Jend), 0, st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// ---------------------------------------------------------------- K_hat^{-1}

__global__ void identity_kernel(double* __restrict__ B, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  B[e] = (e / n == e % n) ? 1.0 : 0.0;
}

// B <- K_hat^{-1} from the Cholesky factor in L: first L^{-1} (lower
// triangular, so block row i needs columns [0, i0 + 64) only), then
// L^{-T} L^{-1} on the lower triangle, then mirrored.  Both passes are blocked
// like the factorisation: 64-row blocks update the rest of their 256-row
// super-block, and the rows beyond it take the whole super-block at once.
// B <- L^{-1} B for B = I on entry (the diagonal blocks' inverses in Dinv):
// block row i needs columns [0, i0 + 64) only.
static hipError_t lower_inverse_forward(const double* L, double* B, double* Dinv, int64_t n, hipStream_t st) {
  hipError_t e = hipSuccess;
  // forward: X_i = L_ii^{-1} B_i on columns [0, i0 + ib); then B_r -= L_ri X_i
  // on the same columns for the rows r of the super-block below block i; after
  // the super-block, the rows below it at once (k = its height, columns
  // [0, Iend), where X is zero beyond each block's own columns)
  for (int64_t I0 = 0; I0 < n; I0 += kSp) {
    const int64_t Iend = std::min<int64_t>(n, I0 + kSp);
    for (int64_t i0 = I0; i0 < Iend; i0 += kEb) {
      const int64_t bi = i0 / kEb;
      const int ib = (int)std::min<int64_t>(kEb, n - i0);
      const int64_t ncols = i0 + ib;
      e = tile_update<false, false, false, true>(Dinv + bi * kEb * kEb, kEb, 0, 0, B, n, -1, i0, B, n, ib, i0, 0, 1,
                                                 ntiles(ncols), st);
      if (e != hipSuccess) return e;
      const int64_t below = Iend - i0 - ib;
      if (below > 0) {
        e = tile_update<false, false, false, false>(L, n, -1, i0, B, n, -1, i0, B, n, ib, i0 + ib, 0, ntiles(below),
                                                    ntiles(ncols), st);
        if (e != hipSuccess) return e;
      }
    }
    if (n > Iend) {
      e = tile_update<false, false, false, false>(L, n, -1, I0, B, n, -1, I0, B, n, (int)(Iend - I0), Iend, 0,
                                                  ntiles(n - Iend), ntiles(Iend), st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

static hipError_t inverse_from_cholesky(const double* L, double* B, double* Dinv, int64_t n, hipStream_t st) {
  identity_kernel<<<(unsigned)((n * n + 255) / 256), 256, 0, st>>>(B, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // The diagonal blocks' inverses, kept for both passes: block bi at Dinv + 64 * 64 * bi.
  const int64_t nb = (n + kEb - 1) / kEb;
  trtri_blocks_kernel<<<(unsigned)nb, 256, 0, st>>>(L, n, Dinv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = lower_inverse_forward(L, B, Dinv, n, st)) != hipSuccess) return e;
  // backward, from the last block: Z_i = L_ii^{-T} C_i on columns
  // [0, i0 + ib); then C[R][Cc] -= L[i-block][R]^T Z[i-block][Cc] on the lower
  // tiles of the super-block's rows above block i (their triangle, then the
  // columns left of the super-block); after the super-block, the lower tiles
  // of every row above it at once
  const int64_t nsb = (n + kSp - 1) / kSp;
  for (int64_t sb = nsb - 1; sb >= 0; --sb) {
    const int64_t I0 = sb * kSp;
    const int64_t Iend = std::min<int64_t>(n, I0 + kSp);
    for (int64_t bi = (Iend - 1) / kEb; bi >= I0 / kEb; --bi) {
      const int64_t i0 = bi * kEb;
      const int ib = (int)std::min<int64_t>(kEb, n - i0);
      const int64_t ncols = i0 + ib;
      e = tile_update<true, false, false, true>(Dinv + bi * kEb * kEb, kEb, 0, 0, B, n, -1, i0, B, n, ib, i0, 0, 1,
                                                ntiles(ncols), st);
      if (e != hipSuccess) return e;
      if (i0 > I0) {
        e = tile_update<true, false, true, false>(L, n, -1, i0, B, n, -1, i0, B, n, ib, I0, I0, ntiles(i0 - I0), 0,
                                                  st);
        if (e != hipSuccess) return e;
        if (I0 > 0) {
          e = tile_update<true, false, false, false>(L, n, -1, i0, B, n, -1, i0, B, n, ib, I0, 0, ntiles(i0 - I0),
                                                     ntiles(I0), st);
          if (e != hipSuccess) return e;
        }
      }
    }
    if (I0 > 0) {
      e = tile_update<true, false, true, false>(L, n, -1, I0, B, n, -1, I0, B, n, (int)(Iend - I0), 0, 0,
                                                ntiles(I0), 0, st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// B[r][c] = B[c][r] for c > r (the upper triangle from the lower one).
__global__ void mirror_kernel(double* __restrict__ B, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int64_t r = e / n, c = e - r * n;
  if (c > r) B[e] = B[c * n + r];
}

// out[a] = sum_b B[a][b] v[b], one wave per row (fixed summation order).
__global__ __launch_bounds__(256) void gemv_rows_kernel(const double* __restrict__ B, const double* __restrict__ v,
                                                        int64_t n, double* __restrict__ out) {
  const int64_t a = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (a >= n) return;
  double s = 0.0;
  for (int64_t b = lane; b < n; b += 64) s = fma(B[a * n + b], v[b], s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) out[a] = s;
}

__global__ void diag_kernel(const double* __restrict__ A, const double* __restrict__ B, int64_t n,
                            double* __restrict__ dA, double* __restrict__ dB) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dA[i] = A[i * n + i];
  dB[i] = B[i * n + i];
}

// ---------------------------------------------------------------- gradient

// Per lower tile (a >= b): partial sums over its pairs of
//   w M_ab psi_ab (x~_aj - x~_bj)^2   (j < d)   and   w M_ab k_ab   (entry d),
// M = omega omega^T - K_hat^{-1}, w = 2 below the diagonal and 1 on it,
// x~ = x / l.  One partial row of DP + 1 per tile.
template <int KIND, int DP>
__global__ __launch_bounds__(256) void exact_grad_kernel(const double* __restrict__ X, int64_t n, int d,
                                                         const double* __restrict__ il, double sf,
                                                         const double* __restrict__ Kinv,
                                                         const double* __restrict__ om,
                                                         double* __restrict__ partial) {
  __shared__ double xa[kEb][DP];   // rows of a tile are wave-uniform: broadcast reads
  __shared__ double xbT[DP][kEb];
  double(*red)[DP + 1] = reinterpret_cast<double(*)[DP + 1]>(&xa[0][0]);  // after the pair loop only
  const int64_t b = blockIdx.x;
  int64_t ti = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
  while (ti * (ti + 1) / 2 > b) --ti;
  const int64_t tj = b - ti * (ti + 1) / 2;
  const int64_t a0 = ti * kEb, b0 = tj * kEb;
  for (int e = threadIdx.x; e < kEb * DP; e += 256) {
    const int row = e / DP, f = e % DP;
    const bool fin = f < d;
    xa[row][f] = (a0 + row < n && fin) ? X[(a0 + row) * d + f] * il[f] : 0.0;
    xbT[f][row] = (b0 + row < n && fin) ? X[(b0 + row) * d + f] * il[f] : 0.0;
  }
  __syncthreads();
  const int c = threadIdx.x % kEb, rb = threadIdx.x / kEb;
  double acc[DP + 1];
#pragma unroll
  for (int f = 0; f <= DP; ++f) acc[f] = 0.0;
  const int64_t bb = b0 + c;
  if (bb < n) {
    const double ob = om[bb];
    for (int j = 0; j < 16; ++j) {
      const int r = rb + 4 * j;
      const int64_t aa = a0 + r;
      if (aa >= n || aa < bb) continue;
      double r2 = 0.0;
#pragma unroll
      for (int f = 0; f < DP; ++f) {
        const double t = xa[r][f] - xbT[f][c];
        r2 = fma(t, t, r2);
      }
      double k, psi;
      if constexpr (KIND == GP_MATERN52) {
        const double u = sqrt(5.0 * r2);
        const double e = exp(-u);
        k = sf * (1.0 + u + u * u / 3.0) * e;
        psi = (5.0 / 3.0) * sf * (1.0 + u) * e;
      } else {
        k = sf * exp(-0.5 * r2);
        psi = k;
      }
      const double w = (aa == bb ? 1.0 : 2.0) * (om[aa] * ob - Kinv[aa * n + bb]);
      const double wp = w * psi;
#pragma unroll
      for (int f = 0; f < DP; ++f) {
        const double t = xa[r][f] - xbT[f][c];
        acc[f] = fma(wp * t, t, acc[f]);
      }
      acc[DP] = fma(w, k, acc[DP]);
    }
  }
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
  for (int f = 0; f <= DP; ++f)
    for (int o = 32; o > 0; o >>= 1) acc[f] += __shfl_xor(acc[f], o);
  __syncthreads();  // every wave is done with xa before it becomes the reduction rows
  if (lane == 0) {
#pragma unroll
    for (int f = 0; f <= DP; ++f) red[wave][f] = acc[f];
  }
  __syncthreads();
  for (int f = threadIdx.x; f <= DP; f += 256)
    partial[b * (DP + 1) + f] = ((red[0][f] + red[1][f]) + red[2][f]) + red[3][f];
}

// out[f] = sum over units of partial[u][f], f <= dp, in unit order.
__global__ void sum_units_kernel(const double* __restrict__ partial, int64_t units, int dp1,
                                 double* __restrict__ out) {
  const int f = blockIdx.x;
  __shared__ double s[256];
  double v = 0.0;
  for (int64_t u = threadIdx.x; u < units; u += 256) v += partial[u * dp1 + f];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[f] = s[0];
}

static int exact_dp(int d) { return d <= 16 ? 16 : d <= 32 ? 32 : d <= 48 ? 48 : 64; }

template <int KIND>
static hipError_t launch_exact_grad(int dp, unsigned tiles, const double* X, int64_t n, int d, const double* il,
                                    double sf, const double* Kinv, const double* om, double* partial,
                                    hipStream_t st) {
  switch (dp) {
    case 16: exact_grad_kernel<KIND, 16><<<tiles, 256, 0, st>>>(X, n, d, il, sf, Kinv, om, partial); break;
    case 32: exact_grad_kernel<KIND, 32><<<tiles, 256, 0, st>>>(X, n, d, il, sf, Kinv, om, partial); break;
    case 48: exact_grad_kernel<KIND, 48><<<tiles, 256, 0, st>>>(X, n, d, il, sf, Kinv, om, partial); break;
    default: exact_grad_kernel<KIND, 64><<<tiles, 256, 0, st>>>(X, n, d, il, sf, Kinv, om, partial); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- driver

static int64_t lower_tiles(int64_t n) {
  const int64_t t = (n + kEb - 1) / kEb;
  return t * (t + 1) / 2;
}

size_t exact_ws_bytes(int d, int64_t n) {
  if (n < 1 || n > kExactMaxN || d < 1 || d > kExactMaxD) return 0;
  size_t b = 2 * align256((size_t)n * n * 8);                            // K_hat -> L; I -> K_hat^{-1}
  b += 3 * align256((size_t)n * 8);                                      // omega, diag L, diag K_hat^{-1}
  b += 2 * align256((size_t)GP_MAX_D * 8);                               // feature scales
  b += align256((size_t)lower_tiles(n) * (exact_dp(d) + 1) * 8);         // gradient partials
  b += align256((size_t)(kExactMaxD + 1) * 8) + align256(sizeof(int));   // sums, info
  b += align256((size_t)((n + kEb - 1) / kEb) * kEb * kEb * 8);          // diagonal-block inverses
  return b + 4096;
}

int run_exact(const gp_kernel* kern, const double* X, const double* y, int64_t n, double* mll, double* grad,
              double* omega_out, void* ws, size_t ws_bytes, hipStream_t st) {
  const int d = kern->d;
  const int dp = exact_dp(d);
  Carve cv(ws, ws_bytes);
  double* A = cv.take<double>((size_t)n * n);
  double* B = cv.take<double>((size_t)n * n);
  double* om = cv.take<double>(n);
  double* dA = cv.take<double>(n);
  double* dB = cv.take<double>(n);
  double* sc = cv.take<double>(GP_MAX_D);
  double* il = cv.take<double>(GP_MAX_D);
  const int64_t tiles = lower_tiles(n);
  double* part = cv.take<double>((size_t)tiles * (dp + 1));
  double* sums = cv.take<double>(kExactMaxD + 1);
  int* info = cv.take<int>(1);
  double* Dinv = cv.take<double>((size_t)((n + kEb - 1) / kEb) * kEb * kEb);
  if (!Dinv) return fail(GP_EWORKSPACE, "gp_exact_mll_and_grad: workspace layout failed");
  std::vector<double> h_sc(d), h_il(d);
  for (int f = 0; f < d; ++f) {
    h_il[f] = 1.0 / kern->lengthscale[f];
    h_sc[f] = (kern->kind == GP_MATERN52 ? std::sqrt(5.0) : 1.0) * h_il[f];
  }
  const int zero = 0;
  GPK_HIP(hipMemcpyAsync(sc, h_sc.data(), sizeof(double) * d, hipMemcpyHostToDevice, st));
  GPK_HIP(hipMemcpyAsync(il, h_il.data(), sizeof(double) * d, hipMemcpyHostToDevice, st));
  GPK_HIP(hipMemcpyAsync(info, &zero, sizeof(int), hipMemcpyHostToDevice, st));
  const dim3 g2((unsigned)ntiles(n), (unsigned)ntiles(n));
  if (kern->kind == GP_MATERN52)
    form_khat_kernel<GP_MATERN52><<<g2, 256, 0, st>>>(X, n, d, sc, kern->outputscale, kern->noise, A);
  else
    form_khat_kernel<GP_RBF><<<g2, 256, 0, st>>>(X, n, d, sc, kern->outputscale, kern->noise, A);
  GPK_HIP(hipGetLastError());
  GPK_HIP(cholesky(A, n, info, Dinv, st));
  GPK_HIP(inverse_from_cholesky(A, B, Dinv, n, st));
  mirror_kernel<<<(unsigned)((n * n + 255) / 256), 256, 0, st>>>(B, n);
  GPK_HIP(hipGetLastError());
  gemv_rows_kernel<<<(unsigned)((n + 3) / 4), 256, 0, st>>>(B, y, n, om);
  GPK_HIP(hipGetLastError());
  diag_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(A, B, n, dA, dB);
  GPK_HIP(hipGetLastError());
  if (grad) {
    if (kern->kind == GP_MATERN52)
      GPK_HIP(launch_exact_grad<GP_MATERN52>(dp, (unsigned)tiles, X, n, d, il, kern->outputscale, B, om, part, st));
    else
      GPK_HIP(launch_exact_grad<GP_RBF>(dp, (unsigned)tiles, X, n, d, il, kern->outputscale, B, om, part, st));
    sum_units_kernel<<<(unsigned)(dp + 1), 256, 0, st>>>(part, tiles, dp + 1, sums);
    GPK_HIP(hipGetLastError());
  }
  std::vector<double> h_om(n), h_dA(n), h_dB(n), h_y(n), h_sums(dp + 1);
  int h_info = 0;
  GPK_HIP(hipMemcpyAsync(h_om.data(), om, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipMemcpyAsync(h_dA.data(), dA, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipMemcpyAsync(h_dB.data(), dB, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipMemcpyAsync(h_y.data(), y, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  if (grad) GPK_HIP(hipMemcpyAsync(h_sums.data(), sums, sizeof(double) * (dp + 1), hipMemcpyDeviceToHost, st));
  GPK_HIP(hipMemcpyAsync(&h_info, info, sizeof(int), hipMemcpyDeviceToHost, st));
  if (omega_out) GPK_HIP(hipMemcpyAsync(omega_out, om, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  GPK_HIP(hipStreamSynchronize(st));
  if (h_info != 0)
    return fail(GP_ENOTPD, "gp_exact_mll_and_grad: K_hat is not numerically positive definite (pivot %d)", h_info - 1);
  double quad = 0.0, logdet = 0.0, wtw = 0.0, tr = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    quad += h_y[i] * h_om[i];
    logdet += 2.0 * std::log(h_dA[i]);
    wtw += h_om[i] * h_om[i];
    tr += h_dB[i];
  }
  const double v = -0.5 * quad - 0.5 * logdet - 0.5 * (double)n * std::log(2.0 * M_PI);
  if (!std::isfinite(v)) return fail(GP_ENONFINITE, "gp_exact_mll_and_grad: non-finite log marginal likelihood");
  *mll = v;
  if (grad) {
    for (int j = 0; j < d; ++j) grad[j] = 0.5 * h_sums[j];
    grad[d] = 0.5 * h_sums[dp];
    grad[d + 1] = 0.5 * kern->noise * (wtw - tr);
    for (int j = 0; j < d + 2; ++j)
      if (!std::isfinite(grad[j])) return fail(GP_ENONFINITE, "gp_exact_mll_and_grad: non-finite gradient");
  }
  return GP_OK;
}

// ---------------------------------------------------------------- exported dense pieces

hipError_t dense_gemm(bool ta, bool tb, bool lower, int64_t m, int64_t nn, int64_t kk, const double* A, int64_t lda,
                      const double* B, int64_t ldb, double* C, int64_t ldc, hipStream_t st) {
  if (m <= 0 || nn <= 0) return hipSuccess;
  if (lower && m != nn) return hipErrorInvalidValue;
  const int nrt = ntiles(m), nct = ntiles(nn);
  const int64_t tiles = lower ? (int64_t)nrt * (nrt + 1) / 2 : (int64_t)nrt * nct;
  if (tiles > 0x7fffffff) return hipErrorInvalidValue;
  const unsigned g = (unsigned)tiles;
#define GPK_GEMM(TA, TB, LO) gemm_f64_kernel<TA, TB, LO><<<g, 256, 0, st>>>(A, lda, B, ldb, C, ldc, m, nn, kk, nrt, nct)
  if (lower) {
    if (ta && tb) GPK_GEMM(true, true, true); else if (ta) GPK_GEMM(true, false, true);
    else if (tb) GPK_GEMM(false, true, true); else GPK_GEMM(false, false, true);
  } else {
    if (ta && tb) GPK_GEMM(true, true, false); else if (ta) GPK_GEMM(true, false, false);
    else if (tb) GPK_GEMM(false, true, false); else GPK_GEMM(false, false, false);
  }
#undef GPK_GEMM
  return hipGetLastError();
}

size_t dense_dinv_doubles(int64_t n) { return (size_t)((n + kEb - 1) / kEb) * kEb * kEb; }

hipError_t dense_cholesky(double* A, int64_t n, int* info, double* Dinv, hipStream_t st) {
  return cholesky(A, n, info, Dinv, st);
}

// B = L^{-1} (lower triangular, zero above the diagonal) for the lower factor L
// (row-major n x n, ld n): the forward pass of inverse_from_cholesky.
hipError_t dense_lower_inverse(const double* L, double* B, double* Dinv, int64_t n, hipStream_t st) {
  identity_kernel<<<(unsigned)((n * n + 255) / 256), 256, 0, st>>>(B, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nb = (n + kEb - 1) / kEb;
  trtri_blocks_kernel<<<(unsigned)nb, 256, 0, st>>>(L, n, Dinv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return lower_inverse_forward(L, B, Dinv, n, st);
}

}  // namespace gpk

using namespace gpk;

extern "C" int gp_exact_mll_and_grad(const gp_kernel* kern, const double* X, const double* y, int64_t n, double* mll,
                                     double* grad, double* omega, void* ws, size_t ws_bytes, void* stream) {
  GPK_TRY(check_kernel(kern));
  if (!X || !y || !mll) return fail(GP_EINVAL, "gp_exact_mll_and_grad: NULL argument");
  if (n < 1 || n > kExactMaxN) return fail(GP_EINVAL, "gp_exact_mll_and_grad: n=%lld outside [1, %lld]", (long long)n,
                                           (long long)kExactMaxN);
  if (kern->d > kExactMaxD) return fail(GP_EINVAL, "gp_exact_mll_and_grad: d=%d above %d", kern->d, kExactMaxD);
  GPK_TRY(check_ws(ws, ws_bytes, exact_ws_bytes(kern->d, n), "gp_exact_mll_and_grad"));
  return run_exact(kern, X, y, n, mll, grad, omega, ws, ws_bytes, (hipStream_t)stream);
}

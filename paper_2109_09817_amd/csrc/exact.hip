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
// = sigma^2 I.  Every O(n^3) step is a sequence of 64 x 64 x 64 FP64 tile
// products C -= P Q (or C = P Q), the panels staged in LDS; triangular solves
// against a 64 x 64 diagonal block multiply by its inverse (formed in LDS by
// one workgroup), so that they are tile products too.
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
  for (int e = threadIdx.x; e < kEb * kEb; e += blockDim.x) {
    const int r = e / kEb, c = e % kEb;
    Ls[r][c] = (r < ib && c < ib) ? (c <= r ? L[(i0 + r) * n + i0 + c] : 0.0) : (r == c ? 1.0 : 0.0);
  }
}

// Xs = Ls^{-1} for a lower-triangular 64 x 64 Ls in LDS, 256 threads: lanes
// 4j..4j+3 form column j by forward substitution against e_j, lane s summing
// the terms m = s (mod 4) and keeping in Xs only the entries of its own class,
// so that each lane reads back what it wrote; the four partial sums meet by
// shuffles.  Ends with a barrier; Xs is complete (zero above the diagonal).
__device__ __forceinline__ void diag_inverse(const double (*Ls)[kEb + 1], double (*Xs)[kEb + 1]) {
  const int j = threadIdx.x >> 2, sub = threadIdx.x & 3;
  for (int r = 0; r < kEb; ++r) {
    if (r < j) {
      if ((r & 3) == sub) Xs[r][j] = 0.0;
      continue;  // uniform over the four lanes of column j
    }
    double part = 0.0;
    for (int m = j + ((sub - j) & 3); m < r; m += 4) part = fma(Ls[r][m], Xs[m][j], part);
    part += __shfl_xor(part, 1);
    part += __shfl_xor(part, 2);
    const double x = ((r == j ? 1.0 : 0.0) - part) / Ls[r][r];
    if ((r & 3) == sub) Xs[r][j] = x;
  }
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
  for (int e = threadIdx.x; e < kEb * kEb; e += 256) {
    const int r = e / kEb, c = e % kEb;
    Ls[r][c] = (r < jb && c < jb) ? A[(j0 + r) * n + j0 + c] : (r == c ? 1.0 : 0.0);
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
#pragma unroll
    for (int it = 0; it < kEb * kEb / 256; ++it) {
      const int e = threadIdx.x + 256 * it;
      const int r = e / kEb, c = e % kEb;
      if (c > k && c <= r) Ls[r][c] -= Ls[r][k] * Ls[c][k];
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
// 64 x 64 tiles, with
//   P(r, k) = PT ? Pm[(p0 + k) ldp + pr + r] : Pm[(pr + r) ldp + p0 + k]
//   Q(k, c) = QT ? Qm[(qc + c) ldq + q0 + k] : Qm[(q0 + k) ldq + qc + c]
// where pr = R (pfix < 0) or pfix, and qc = Cc (qfix < 0) or qfix.  Tile (ti,
// tj) has R = rbase + 64 ti, Cc = cbase + 64 tj; LOWER enumerates tj <= ti <
// nrt, otherwise the nrt x nct rectangle.  Output rows and columns at or beyond
// n are skipped (their operands read as 0).  Every operand is staged in LDS
// before the tile is written, so C's tile may be one of the operand tiles
// (never another workgroup's).  Each thread owns a 4 x 4 block (rows 4 tr + i,
// columns 4 tc + j), so that its operands are two 16-byte LDS reads per side.
template <bool PT, bool QT, bool LOWER, bool ASSIGN>
__global__ __launch_bounds__(256) void tile_update_kernel(const double* Pm, int64_t ldp, int64_t pfix, int64_t p0,
                                                          const double* Qm, int64_t ldq, int64_t qfix, int64_t q0,
                                                          double* Cm, int64_t n, int kb, int64_t rbase, int64_t cbase,
                                                          int nrt, int nct) {
  __shared__ double Ps[kEb][kEb];  // [k][r]
  __shared__ double Qs[kEb][kEb];  // [k][c]
  int64_t ti, tj;
  const int64_t b = blockIdx.x;
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
  for (int e = threadIdx.x; e < kEb * kEb; e += 256) {
    int r, k;
    if (PT) {
      k = e / kEb;
      r = e % kEb;  // consecutive threads: consecutive columns of row p0 + k
    } else {
      r = e / kEb;
      k = e % kEb;  // consecutive threads: consecutive columns of row pr + r
    }
    const bool ok = k < kb && R + r < n;
    Ps[k][r] = ok ? (PT ? Pm[(p0 + k) * ldp + pr + r] : Pm[(pr + r) * ldp + p0 + k]) : 0.0;
  }
  for (int e = threadIdx.x; e < kEb * kEb; e += 256) {
    int c, k;
    if (QT) {
      c = e / kEb;
      k = e % kEb;
    } else {
      k = e / kEb;
      c = e % kEb;
    }
    const bool ok = k < kb && Cc + c < n;
    Qs[k][c] = ok ? (QT ? Qm[(qc + c) * ldq + q0 + k] : Qm[(q0 + k) * ldq + qc + c]) : 0.0;
  }
  __syncthreads();
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k = 0; k < kEb; ++k) {
    double a[4], q[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = Ps[k][4 * tr + i];
#pragma unroll
    for (int j = 0; j < 4; ++j) q[j] = Qs[k][4 * tc + j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], q[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = R + 4 * tr + i;
    if (row >= n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = Cc + 4 * tc + j;
      if (col >= n) continue;
      if (ASSIGN)
        Cm[row * n + col] = acc[i][j];
      else
        Cm[row * n + col] -= acc[i][j];
    }
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

static int ntiles(int64_t len) { return (int)((len + kEb - 1) / kEb); }

// A = L L^T in place (lower triangle; the diagonal blocks' upper parts are
// zeroed, the rest of the upper triangle is left as it was).
static hipError_t cholesky(double* A, int64_t n, int* info, double* Dinv, hipStream_t st) {
  for (int64_t j0 = 0; j0 < n; j0 += kEb) {
    const int jb = (int)std::min<int64_t>(kEb, n - j0);
    const int64_t rest = n - j0 - jb;
    potrf_diag_kernel<<<1, 256, 0, st>>>(A, n, j0, jb, info, rest > 0 ? Dinv : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (rest <= 0) break;
    // L21 = A21 L11^{-T} = A21 Dinv^T (jb = 64 here: only the last block is narrower)
    e = tile_update<false, true, false, true>(A, n, -1, j0, Dinv, kEb, 0, 0, A, n, jb, j0 + jb, j0, ntiles(rest), 1,
                                              st);
    if (e != hipSuccess) return e;
    // A22 -= L21 L21^T over the lower tiles of the trailing matrix
    e = tile_update<false, true, true, false>(A, n, -1, j0, A, n, -1, j0, A, n, jb, j0 + jb, j0 + jb, ntiles(rest),
                                              0, st);
    if (e != hipSuccess) return e;
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
// L^{-T} L^{-1} on the lower triangle, then mirrored.
static hipError_t inverse_from_cholesky(const double* L, double* B, double* Dinv, int64_t n, hipStream_t st) {
  identity_kernel<<<(unsigned)((n * n + 255) / 256), 256, 0, st>>>(B, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // The diagonal blocks' inverses, kept for both passes: block bi at Dinv + 64 * 64 * bi.
  const int64_t nb = (n + kEb - 1) / kEb;
  trtri_blocks_kernel<<<(unsigned)nb, 256, 0, st>>>(L, n, Dinv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // forward, right-looking: X_i = L_ii^{-1} B_i on columns [0, i0 + ib); then
  // B_below -= L_below,i X_i on the same columns
  for (int64_t bi = 0; bi < nb; ++bi) {
    const int64_t i0 = bi * kEb;
    const int ib = (int)std::min<int64_t>(kEb, n - i0);
    const int64_t ncols = i0 + ib;
    e = tile_update<false, false, false, true>(Dinv + bi * kEb * kEb, kEb, 0, 0, B, n, -1, i0, B, n, ib, i0, 0, 1,
                                               ntiles(ncols), st);
    if (e != hipSuccess) return e;
    const int64_t below = n - i0 - ib;
    if (below > 0) {
      e = tile_update<false, false, false, false>(L, n, -1, i0, B, n, -1, i0, B, n, ib, i0 + ib, 0, ntiles(below),
                                                  ntiles(ncols), st);
      if (e != hipSuccess) return e;
    }
  }
  // backward, right-looking from the last block: Z_i = L_ii^{-T} C_i on
  // columns [0, i0 + ib); then, on the lower tiles above,
  // C[R][Cc] -= L[i-block][R]^T Z[i-block][Cc]
  for (int64_t bi = nb - 1; bi >= 0; --bi) {
    const int64_t i0 = bi * kEb;
    const int ib = (int)std::min<int64_t>(kEb, n - i0);
    const int64_t ncols = i0 + ib;
    e = tile_update<true, false, false, true>(Dinv + bi * kEb * kEb, kEb, 0, 0, B, n, -1, i0, B, n, ib, i0, 0, 1,
                                              ntiles(ncols), st);
    if (e != hipSuccess) return e;
    if (i0 > 0) {
      e = tile_update<true, false, true, false>(L, n, -1, i0, B, n, -1, i0, B, n, ib, 0, 0, ntiles(i0), 0, st);
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

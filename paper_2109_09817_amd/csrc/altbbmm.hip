// AltBBMM (Sec. 3.2): block conjugate gradients (Sec. 3.1) in FP64 on the
// symmetrically preconditioned system P^{-1/2} K_hat P^{-1/2} U = P^{-1/2} B,
// W = P^{-1/2} U, with the Nystrom preconditioner over r landmark rows M
//
//   P = K_XM K_MM^{-1} K_MX + sigma^2 I.
//
// Spectral square root.  K_MM^{-1} is taken rank-revealing: K_MM = U diag(lam) U^T
// and C = U_k diag(lam_k)^{-1/2} over the eigenvalues above 1e-7 lam_max (nearly
// repeated landmarks make K_MM numerically singular; the dropped directions are
// left to CG).  F = K_XM C (n x k, formed on the GPU) carries the approximation
// F F^T; with the eigendecomposition F^T F = V diag(S) V^T the thin SVD is
// F = U_F S^{1/2} V^T, and P = U_F diag(S + sigma^2) U_F^T + sigma^2 (I - U_F U_F^T):
//
//   P^{-1/2} = sigma^{-1} I + Z^T diag(g) Z,   Z^T = F V = U_F S^{1/2},
//   g = ((S + sigma^2)^{-1/2} - sigma^{-1}) / S
//     = -1 / (sigma sqrt(S + sigma^2) (sigma + sqrt(S + sigma^2))).
//
// The factor form matters at low noise: F^T F is taken from F itself, never as
// C^T (K_MX K_XM) C, whose rounding (eps |K|^2 |C|^2 ~ eps |K|^2 / lam_min(K_MM))
// can exceed sigma^2; and P^{-1/2} is applied through Z (rows of norm S^{1/2}),
// never through K_XM and an r x r middle factor with entries ~ |C|^2 |g|.
// One application costs two tall-skinny products with Z.  The block CG
// recurrences (O'Leary):
//   Q = A D;  alpha = (D^T Q)^{-1} (R^T R);  U += D alpha;  R -= Q alpha;
//   beta = (R_old^T R_old)^{-1} (R^T R);  D = R + D beta,
// with the s x s Gram matrices reduced on the GPU and solved on the host.
#include <algorithm>
#include <cmath>
#include <vector>

#include "api_common.h"
#include "solver.h"

namespace gpk {

constexpr int kNysTile = 32;   // landmarks per workgroup of the column kernel
constexpr int kTallK = 32;     // K rows of C staged per step of the tall product
constexpr int kTallMaxS = 64;  // columns of the tall product
constexpr int kNysMaxR = 1024;
constexpr double kNysRcond = 1e-7;  // K_MM eigenvalues kept: lam > kNysRcond * lam_max

// KXM[j n + p] = s_f m(r(x_p, x_{M_j})) in FP64.  sc[f]: feature scale (Matern
// sqrt5 / l_f, so that u = sqrt5 r; RBF 1 / l_f).
template <int KIND>
__global__ __launch_bounds__(256) void kernel_cols_kernel(const double* __restrict__ X, int64_t n, int d,
                                                          const double* __restrict__ sc,
                                                          const int64_t* __restrict__ M, int r, double sf,
                                                          double* __restrict__ out) {
  __shared__ double Z[kNysTile][GP_MAX_D];
  __shared__ double S[GP_MAX_D];
  const int j0 = blockIdx.y * kNysTile;
  for (int e = threadIdx.x; e < d; e += blockDim.x) S[e] = sc[e];
  __syncthreads();
  for (int e = threadIdx.x; e < kNysTile * d; e += blockDim.x) {
    const int j = e / d, f = e - j * d;
    Z[j][f] = j0 + j < r ? X[M[j0 + j] * d + f] * S[f] : 0.0;
  }
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double acc[kNysTile];
#pragma unroll
  for (int j = 0; j < kNysTile; ++j) acc[j] = 0.0;
  for (int f = 0; f < d; ++f) {
    const double x = X[p * d + f] * S[f];
#pragma unroll
    for (int j = 0; j < kNysTile; ++j) {
      const double t = x - Z[j][f];
      acc[j] = fma(t, t, acc[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < kNysTile; ++j) {
    if (j0 + j >= r) continue;
    double m;
    if constexpr (KIND == GP_MATERN52) {
      const double u = sqrt(acc[j]);
      m = (1.0 + u + u * u / 3.0) * exp(-u);
    } else {
      m = exp(-0.5 * acc[j]);
    }
    out[(int64_t)(j0 + j) * n + p] = sf * m;
  }
}

// KMM[j r + i] = KXM[j n + M_i].
__global__ void gather_landmark_rows_kernel(const double* __restrict__ KXM, int64_t n, const int64_t* __restrict__ M,
                                            int r, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)r * r) return;
  const int64_t j = e / r, i = e - j * r;
  out[e] = KXM[j * n + M[i]];
}

// Y = alpha V + A C for A (nrows x kk, column-major, lda), C (kk x s, row-major
// with row stride ldc), V and Y (nrows x s): column-major with ldv / ldy, or
// (ROWMAJOR) row-major with s per row.  One thread per row; each thread reads all of its row of A before
// writing its row of Y, so Y may alias A or V.
template <bool ROWMAJOR>
__global__ __launch_bounds__(256) void tall_product_kernel(const double* __restrict__ A, int64_t lda,
                                                           int64_t nrows, int kk, const double* __restrict__ C,
                                                           int64_t ldc, int s, double alpha, const double* V, int64_t ldv,
                                                           double* Y, int64_t ldy) {
  __shared__ double Cs[kTallK][kTallMaxS];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[kTallMaxS];
#pragma unroll
  for (int c = 0; c < kTallMaxS; ++c) acc[c] = 0.0;
  for (int k0 = 0; k0 < kk; k0 += kTallK) {
    __syncthreads();
    for (int e = threadIdx.x; e < kTallK * kTallMaxS; e += blockDim.x) {
      const int k = e / kTallMaxS, c = e - k * kTallMaxS;
      Cs[k][c] = (k0 + k < kk && c < s) ? C[(int64_t)(k0 + k) * ldc + c] : 0.0;
    }
    __syncthreads();
    if (p < nrows) {
      const int kn = kk - k0 < kTallK ? kk - k0 : kTallK;
      for (int k = 0; k < kn; ++k) {
        const double a = A[(int64_t)(k0 + k) * lda + p];
#pragma unroll
        for (int c = 0; c < kTallMaxS; ++c) acc[c] = fma(a, Cs[k][c], acc[c]);
      }
    }
  }
  if (p >= nrows) return;
#pragma unroll
  for (int c = 0; c < kTallMaxS; ++c) {
    if (c < s) {
      double y = acc[c];
      if (V) y += alpha * (ROWMAJOR ? V[p * s + c] : V[(int64_t)c * ldv + p]);
      if (ROWMAJOR)
        Y[p * s + c] = y;
      else
        Y[(int64_t)c * ldy + p] = y;
    }
  }
}

static hipError_t tall_product(const double* A, int64_t lda, int64_t nrows, int kk, const double* C, int64_t ldc,
                               int s, double alpha, const double* V, int64_t ldv, double* Y, int64_t ldy,
                               bool rowmajor, hipStream_t st) {
  const unsigned grid = (unsigned)((nrows + 255) / 256);
  if (rowmajor)
    tall_product_kernel<true><<<grid, 256, 0, st>>>(A, lda, nrows, kk, C, ldc, s, alpha, V, ldv, Y, ldy);
  else
    tall_product_kernel<false><<<grid, 256, 0, st>>>(A, lda, nrows, kk, C, ldc, s, alpha, V, ldv, Y, ldy);
  return hipGetLastError();
}

// Y = A C for C (kk x m row-major) with any m: column blocks of kTallMaxS.
// A (nrows x kk) and Y (nrows x m) column-major with ld nrows.
static hipError_t tall_product_wide(const double* A, int64_t nrows, int kk, const double* C, int m, double* Y,
                                    hipStream_t st) {
  for (int c0 = 0; c0 < m; c0 += kTallMaxS) {
    const int sc = std::min(kTallMaxS, m - c0);
    hipError_t e = tall_product(A, nrows, nrows, kk, C + c0, m, sc, 0.0, nullptr, 0, Y + (int64_t)c0 * nrows,
                                nrows, false, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// out[e] = a in[e] for e < count.
__global__ void tall_scale_kernel(const double* __restrict__ in, int64_t count, double a, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) out[e] = a * in[e];
}

// out[e] = g[e / s] in[e] for e < r s (rows of an r x s row-major block).
__global__ void scale_rows_kernel(const double* __restrict__ in, const double* __restrict__ g, int r, int s,
                                  double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < r * s) out[e] = g[e / s] * in[e];
}

// A^T B with the row split sized to the output: ~2048 workgroups whatever pa, qb.
static int64_t gram_blocks(int64_t n, int pa, int qb) {
  const int64_t tiles = (int64_t)((pa + 63) / 64) * ((qb + 63) / 64);
  return std::max<int64_t>(1, std::min<int64_t>((n + 63) / 64, 2048 / tiles));
}
static size_t gram_partial_doubles(int64_t n, int pa, int qb) {
  return (size_t)gram_blocks(n, pa, qb) * pa * qb;
}
// Largest partial buffer of a k x k Gram over k <= r (the row split grows as k shrinks).
static size_t gram_partial_doubles_upto(int64_t n, int r) {
  size_t m = 0;
  for (int k = 1; k <= r; ++k) m = std::max(m, gram_partial_doubles(n, k, k));
  return m;
}
static hipError_t gram(const double* A, int pa, const double* B, int qb, int64_t n, double* out, double* partial,
                       hipStream_t st) {
  return atb_n(A, pa, B, qb, n, out, partial, gram_blocks(n, pa, qb), st);
}

// ---------------------------------------------------------------- Nystrom build

size_t nystrom_ws_bytes(int d, int64_t n, int r) {
  size_t b = 0;
  b += align256((size_t)r * 8);                                // landmark indices
  b += align256((size_t)d * 8);                                // feature scales
  b += 2 * align256((size_t)r * r * 8);                        // K_MM then F^T F; C then V
  b += align256((size_t)n * r * 8);                            // F = K_XM C
  b += align256(gram_partial_doubles_upto(n, r) * 8);          // Gram partials (F^T F, k <= r)
  return b + 4096;
}

// Symmetrise a row-major m x m matrix evaluated in two halves.
static void symmetrise(std::vector<double>& A, int m) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < i; ++j) A[(size_t)i * m + j] = A[(size_t)j * m + i] = 0.5 * (A[(size_t)i * m + j] + A[(size_t)j * m + i]);
}

int run_nystrom(const gp_kernel* kern, const double* X, int64_t n, const int64_t* landmarks, int r, double* Zt,
                double* g, void* ws, size_t ws_bytes, hipStream_t st) {
  const int d = kern->d;
  Carve cv(ws, ws_bytes);
  int64_t* Mdev = cv.take<int64_t>(r);
  double* scd = cv.take<double>(d);
  double* Sq = cv.take<double>((size_t)r * r);   // K_MM, later F^T F
  double* Cd = cv.take<double>((size_t)r * r);   // C, later V
  double* F = cv.take<double>((size_t)n * r);
  double* part = cv.take<double>(gram_partial_doubles_upto(n, r));
  if (!part) return fail(GP_EWORKSPACE, "gp_nystrom_precond: workspace layout failed");
  std::vector<double> sc(d);
  for (int f = 0; f < d; ++f)
    sc[f] = (kern->kind == GP_MATERN52 ? std::sqrt(5.0) : 1.0) / kern->lengthscale[f];
  GPK_HIP(hipMemcpyAsync(Mdev, landmarks, sizeof(int64_t) * r, hipMemcpyHostToDevice, st));
  GPK_HIP(hipMemcpyAsync(scd, sc.data(), sizeof(double) * d, hipMemcpyHostToDevice, st));
  // K_XM (column j = K(X, x_{M_j})) into the output buffer; it is replaced by the factor below
  double* KXM = Zt;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)((r + kNysTile - 1) / kNysTile));
  if (kern->kind == GP_MATERN52)
    kernel_cols_kernel<GP_MATERN52><<<grid, 256, 0, st>>>(X, n, d, scd, Mdev, r, kern->outputscale, KXM);
  else
    kernel_cols_kernel<GP_RBF><<<grid, 256, 0, st>>>(X, n, d, scd, Mdev, r, kern->outputscale, KXM);
  GPK_HIP(hipGetLastError());
  gather_landmark_rows_kernel<<<(unsigned)(((int64_t)r * r + 255) / 256), 256, 0, st>>>(KXM, n, Mdev, r, Sq);
  GPK_HIP(hipGetLastError());
  std::vector<double> L((size_t)r * r);
  GPK_HIP(hipMemcpyAsync(L.data(), Sq, sizeof(double) * r * r, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipStreamSynchronize(st));
  for (double v : L)
    if (!std::isfinite(v)) return fail(GP_ENONFINITE, "gp_nystrom_precond: non-finite kernel");
  // K_MM is stored column by column; it is symmetric up to the order of its evaluation
  symmetrise(L, r);
  // Rank-revealing inverse of K_MM: K_MM = U diag(lam) U^T, directions with lam <= kNysRcond lam_max
  // (nearly repeated landmarks) dropped; C = U_keep diag(lam_keep)^{-1/2} (r x k).
  std::vector<double> lam, U;
  if (!sym_eig(r, L, lam, U)) return fail(GP_ENOTPD, "gp_nystrom_precond: eigen-decomposition of K_MM did not converge");
  double lmax = 0.0;
  for (double v : lam) lmax = std::max(lmax, v);
  std::vector<int> keep;
  for (int i = 0; i < r; ++i)
    if (lam[i] > kNysRcond * lmax) keep.push_back(i);
  const int k = (int)keep.size();
  if (k == 0) return fail(GP_ENOTPD, "gp_nystrom_precond: K_MM is numerically zero");
  std::vector<double> Cm((size_t)r * k);
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < k; ++j) Cm[(size_t)i * k + j] = U[(size_t)i * r + keep[j]] / std::sqrt(lam[keep[j]]);
  // F = K_XM C (n x k, column-major) and F^T F (k x k)
  GPK_HIP(hipMemcpyAsync(Cd, Cm.data(), sizeof(double) * r * k, hipMemcpyHostToDevice, st));
  GPK_HIP(tall_product_wide(KXM, n, r, Cd, k, F, st));
  GPK_HIP(gram(F, k, F, k, n, Sq, part, st));
  std::vector<double> T((size_t)k * k);
  GPK_HIP(hipMemcpyAsync(T.data(), Sq, sizeof(double) * k * k, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipStreamSynchronize(st));  // also completes C's upload before Cm is released
  for (double v : T)
    if (!std::isfinite(v)) return fail(GP_ENONFINITE, "gp_nystrom_precond: non-finite F^T F");
  symmetrise(T, k);
  std::vector<double> S, V;
  if (!sym_eig(k, T, S, V)) return fail(GP_ENOTPD, "gp_nystrom_precond: eigen-decomposition of F^T F did not converge");
  // Z^T = F V into the first k rows of the output (K_XM is no longer needed), zero rows beyond k
  std::vector<double> gv(r, 0.0);
  const double sig = std::sqrt(kern->noise);
  for (int m = 0; m < k; ++m) {
    const double q = std::sqrt(std::max(S[m], 0.0) + kern->noise);
    gv[m] = -1.0 / (sig * q * (sig + q));
  }
  GPK_HIP(hipMemcpyAsync(Cd, V.data(), sizeof(double) * k * k, hipMemcpyHostToDevice, st));
  GPK_HIP(tall_product_wide(F, n, k, Cd, k, Zt, st));
  if (k < r) GPK_HIP(launch_fill(Zt + (int64_t)k * n, 0.0, (int64_t)(r - k) * n, st));
  GPK_HIP(hipMemcpyAsync(g, gv.data(), sizeof(double) * r, hipMemcpyHostToDevice, st));
  GPK_HIP(hipStreamSynchronize(st));
  return GP_OK;
}

// ---------------------------------------------------------------- apply P^{-1/2}

size_t nystrom_apply_ws_bytes(int64_t n, int r, int s) {
  return 2 * align256((size_t)r * s * 8) + align256(gram_partial_doubles(n, std::max(r, 1), s) * 8) + 1024;
}

// Y = sigma^{-1} V + Z^T (diag(g) (Z V)); Y may alias V.
static hipError_t nystrom_apply(const double* Zt, const double* g, int64_t n, int r, double noise, const double* V,
                                int64_t ldv, int s, double* Y, int64_t ldy, double* C1, double* C2, double* part,
                                hipStream_t st) {
  hipError_t e;
  if (ldv != n) return hipErrorInvalidValue;  // gram() takes ld = n
  if ((e = gram(Zt, r, V, s, n, C1, part, st)) != hipSuccess) return e;
  scale_rows_kernel<<<(unsigned)((r * s + 255) / 256), 256, 0, st>>>(C1, g, r, s, C2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return tall_product(Zt, n, n, r, C2, s, s, 1.0 / std::sqrt(noise), V, ldv, Y, ldy, false, st);
}

// ---------------------------------------------------------------- block CG

size_t bcg_ws_bytes(int precision, int d, int64_t n, int r, int s) {
  size_t b = kmm_plan_bytes(precision, d, n, n, true, s);
  b += 6 * align256((size_t)n * s * 8);                              // Z, R, D, Q, T1, T2
  b += nystrom_apply_ws_bytes(n, std::max(r, 1), s);                 // C1, C2, partials
  b += align256(gram_partial_doubles(n, s, s) * 8);                  // s x s Gram partials
  b += 3 * align256((size_t)s * s * 8);                              // Gram out, alpha/beta
  return b + 4096;
}

// s x s: X = A^{-1} B by LU with partial pivoting (row-major).  The block Gram
// matrices are symmetric positive definite in exact arithmetic, but once the
// search block is nearly rank-deficient rounding can make them indefinite, so
// they are not factorised by Cholesky.  False when a pivot vanishes (breakdown).
static bool host_lu_solve(std::vector<double> A, int s, const std::vector<double>& B, std::vector<double>& X) {
  X = B;
  std::vector<int> perm(s);
  for (int i = 0; i < s; ++i) perm[i] = i;
  for (int k = 0; k < s; ++k) {
    int piv = k;
    for (int i = k + 1; i < s; ++i)
      if (std::fabs(A[(size_t)i * s + k]) > std::fabs(A[(size_t)piv * s + k])) piv = i;
    const double pv = A[(size_t)piv * s + k];
    if (!(pv != 0.0) || !std::isfinite(pv)) return false;
    if (piv != k) {
      for (int j = 0; j < s; ++j) std::swap(A[(size_t)k * s + j], A[(size_t)piv * s + j]);
      for (int j = 0; j < s; ++j) std::swap(X[(size_t)k * s + j], X[(size_t)piv * s + j]);
    }
    for (int i = k + 1; i < s; ++i) {
      const double f = A[(size_t)i * s + k] / pv;
      if (f == 0.0) continue;
      for (int j = k; j < s; ++j) A[(size_t)i * s + j] -= f * A[(size_t)k * s + j];
      for (int j = 0; j < s; ++j) X[(size_t)i * s + j] -= f * X[(size_t)k * s + j];
    }
  }
  for (int k = s - 1; k >= 0; --k) {
    for (int j = 0; j < s; ++j) {
      double v = X[(size_t)k * s + j];
      for (int i = k + 1; i < s; ++i) v -= A[(size_t)k * s + i] * X[(size_t)i * s + j];
      X[(size_t)k * s + j] = v / A[(size_t)k * s + k];
    }
  }
  for (double v : X)
    if (!std::isfinite(v)) return false;
  return true;
}

int run_bcg(const gp_kernel* kern, int precision, const double* X, int64_t n, const double* Zt, const double* g,
            int r, const double* B, int64_t ldb, int s, int max_iter, double tol, double* W, int64_t ldw,
            int32_t* iters_out, double* relres, void* ws, size_t ws_bytes, hipStream_t st) {
  const int d = kern->d;
  const size_t kb = kmm_plan_bytes(precision, d, n, n, true, s);
  KmmPlan plan;
  if (!kmm_plan_init(plan, kern, precision, n, n, true, s, ws, kb)) return fail(GP_EWORKSPACE, "gp_bcg: workspace too small");
  Carve cv((char*)ws + align256(kb), ws_bytes - align256(kb));
  const size_t ns = (size_t)n * s;
  double* Z = cv.take<double>(ns);
  double* R = cv.take<double>(ns);
  double* D = cv.take<double>(ns);
  double* Q = cv.take<double>(ns);
  double* T1 = cv.take<double>(ns);
  double* T2 = cv.take<double>(ns);
  double* C1 = cv.take<double>((size_t)std::max(r, 1) * s);
  double* C2 = cv.take<double>((size_t)std::max(r, 1) * s);
  double* part = cv.take<double>(std::max(gram_partial_doubles(n, std::max(r, 1), s), gram_partial_doubles(n, s, s)));
  double* Gd = cv.take<double>((size_t)s * s);
  double* Ad = cv.take<double>((size_t)s * s);
  double* Bd = cv.take<double>((size_t)s * s);
  if (!Bd) return fail(GP_EWORKSPACE, "gp_bcg: workspace layout failed");
  const bool pre = r > 0;
  auto precond = [&](const double* in, double* out) -> hipError_t {
    if (pre) return nystrom_apply(Zt, g, n, r, kern->noise, in, n, s, out, n, C1, C2, part, st);
    return hipMemcpyAsync(out, in, sizeof(double) * ns, hipMemcpyDeviceToDevice, st);
  };
  auto gram_host = [&](const double* A, const double* Bm, std::vector<double>& out) -> hipError_t {
    hipError_t e = gram(A, s, Bm, s, n, Gd, part, st);
    if (e != hipSuccess) return e;
    out.resize((size_t)s * s);
    e = hipMemcpyAsync(out.data(), Gd, sizeof(double) * s * s, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
  };
  // B_hat = P^{-1/2} B into R (and D); Z = 0
  for (int c = 0; c < s; ++c)
    GPK_HIP(hipMemcpyAsync(T1 + (size_t)c * n, B + (size_t)c * ldb, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  GPK_HIP(precond(T1, R));
  GPK_HIP(hipMemcpyAsync(D, R, sizeof(double) * ns, hipMemcpyDeviceToDevice, st));
  GPK_HIP(launch_fill(Z, 0.0, (int64_t)ns, st));
  GPK_HIP(kmm_prepare(plan, kern, X, nullptr, st));
  // host s x s blocks; each stays untouched until the stream synchronisation that
  // follows its upload
  std::vector<double> RtR, RtRn, DtQ, alpha, nalpha, beta;
  GPK_HIP(gram_host(R, R, RtR));
  std::vector<double> bnorm(s);
  for (int c = 0; c < s; ++c) {
    bnorm[c] = std::sqrt(std::max(RtR[(size_t)c * s + c], 0.0));
    if (!std::isfinite(bnorm[c])) return fail(GP_ENONFINITE, "gp_bcg: non-finite right-hand side");
    if (!(bnorm[c] > 0.0)) return fail(GP_EINVAL, "gp_bcg: right-hand side column %d is zero", c);
    relres[c] = 1.0;
  }
  int it = 0;
  bool converged = false;
  while (it < max_iter) {
    GPK_HIP(precond(D, T1));
    GPK_HIP(kmm_apply(plan, T1, n, s, T2, n, st, false));
    GPK_HIP(precond(T2, Q));
    GPK_HIP(gram_host(D, Q, DtQ));
    if (!host_lu_solve(DtQ, s, RtR, alpha))
      return fail(GP_ENOTPD, "gp_bcg: D^T A D singular at iteration %d (block breakdown)", it);
    nalpha = alpha;
    for (auto& v : nalpha) v = -v;
    GPK_HIP(hipMemcpyAsync(Ad, alpha.data(), sizeof(double) * s * s, hipMemcpyHostToDevice, st));
    GPK_HIP(hipMemcpyAsync(Bd, nalpha.data(), sizeof(double) * s * s, hipMemcpyHostToDevice, st));
    GPK_HIP(tall_product(D, n, n, s, Ad, s, s, 1.0, Z, n, Z, n, false, st));   // Z += D alpha
    GPK_HIP(tall_product(Q, n, n, s, Bd, s, s, 1.0, R, n, R, n, false, st));   // R -= Q alpha
    GPK_HIP(gram_host(R, R, RtRn));  // also orders the uploads above before alpha is rewritten
    ++it;
    bool all = true;
    for (int c = 0; c < s; ++c) {
      relres[c] = std::sqrt(std::max(RtRn[(size_t)c * s + c], 0.0)) / bnorm[c];
      if (!std::isfinite(relres[c])) return fail(GP_ENONFINITE, "gp_bcg: non-finite residual at iteration %d", it);
      all = all && relres[c] <= tol;
    }
    if (all) {
      converged = true;
      break;
    }
    if (it == max_iter) break;
    if (!host_lu_solve(RtR, s, RtRn, beta))
      return fail(GP_ENOTPD, "gp_bcg: R^T R singular at iteration %d (block breakdown)", it);
    GPK_HIP(hipMemcpyAsync(Bd, beta.data(), sizeof(double) * s * s, hipMemcpyHostToDevice, st));
    GPK_HIP(tall_product(D, n, n, s, Bd, s, s, 1.0, R, n, D, n, false, st));   // D = R + D beta
    RtR.swap(RtRn);
    GPK_HIP(hipStreamSynchronize(st));  // beta's upload completes before the host vector is reused
  }
  // W = P^{-1/2} Z
  GPK_HIP(precond(Z, T1));
  for (int c = 0; c < s; ++c)
    GPK_HIP(hipMemcpyAsync(W + (size_t)c * ldw, T1 + (size_t)c * n, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  GPK_HIP(hipStreamSynchronize(st));
  *iters_out = it;
  return converged ? GP_OK : GP_WNOCONV;
}

// ---------------------------------------------------------------- large rank: Cholesky factor form
//
// At the paper's rank (r = 10^4, Sec. 4) the two r x r eigendecompositions of
// the spectral form are out of reach on the host.  The same Nystrom
// approximation is then carried by Cholesky factors only:
//
//   K_MM + delta I = L_M L_M^T          (delta = kNysCholJitter r s_f)
//   F = K_XM L_M^{-T}                   (n x r; F F^T = K_XM (K_MM + delta I)^{-1} K_MX)
//   F^T F + sigma^2 I = L_G L_G^T
//   E = F L_G^{-T}                      (n x r)
//   P = F F^T + sigma^2 I,   P^{-1} = sigma^{-2} (I - E E^T).
//
// E E^T = F (F^T F + sigma^2 I)^{-1} F^T has eigenvalues s / (s + sigma^2) < 1
// (s the eigenvalues of F^T F), so the P^{-1} applied is positive definite
// however the factors round: the Gram matrix is formed from F itself, never as
// L_M^{-1} K_MX K_XM L_M^{-T}.  The jitter bounds cond(K_MM + delta I) by
// about 1 / kNysCholJitter (nearly repeated landmark rows make K_MM singular)
// and keeps P an under-approximation of K_hat.  The O(n r^2) products (F, the
// Gram matrix, E) run on the FP64 matrix cores (dense_gemm), the two
// factorisations and triangular inverses on blocked FP64 tile kernels.
//
// The solver with this preconditioner is block preconditioned CG (O'Leary) on
// K_hat W = B with P^{-1}: its iterates are those of block CG on the
// symmetrically preconditioned P^{-1/2} K_hat P^{-1/2} (the form of gp_bcg), and
// its residual norm sqrt(r^T P^{-1} r) is that system's residual norm.

constexpr int kNysCholMaxR = 16384;
constexpr double kNysCholJitter = 1e-10;

__global__ void add_diag_kernel(double* __restrict__ A, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) A[i * n + i] += v;
}

// M[i] = i (the landmark rows gathered into their own matrix)
__global__ void iota_kernel(int64_t* __restrict__ M, int r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < r) M[i] = i;
}

__global__ void gather_rows_kernel(const double* __restrict__ X, int d, const int64_t* __restrict__ M, int r,
                                   double* __restrict__ XM) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)r * d) return;
  const int64_t i = e / d, f = e - i * d;
  XM[e] = X[M[i] * d + f];
}

size_t nystrom_chol_ws_bytes(int d, int64_t n, int r) {
  size_t b = 0;
  b += 2 * align256((size_t)r * 8);                 // landmark indices, iota
  b += align256((size_t)d * 8);                     // feature scales
  b += align256((size_t)r * d * 8);                 // landmark rows
  b += 2 * align256((size_t)r * r * 8);             // K_MM -> L_M -> G -> L_G; L^{-1}
  b += align256(dense_dinv_doubles(r) * 8);         // diagonal-block inverses
  b += align256((size_t)n * r * 8);                 // K_XM, later E^T
  b += align256(sizeof(int) * 2);                   // Cholesky status
  return b + 4096;
}

int run_nystrom_chol(const gp_kernel* kern, const double* X, int64_t n, const int64_t* landmarks, int r, double* E,
                     void* ws, size_t ws_bytes, hipStream_t st) {
  const int d = kern->d;
  Carve cv(ws, ws_bytes);
  int64_t* Mdev = cv.take<int64_t>(r);
  int64_t* iota = cv.take<int64_t>(r);
  double* scd = cv.take<double>(d);
  double* XM = cv.take<double>((size_t)r * d);
  double* A = cv.take<double>((size_t)r * r);
  double* Linv = cv.take<double>((size_t)r * r);
  double* Dinv = cv.take<double>(dense_dinv_doubles(r));
  double* T = cv.take<double>((size_t)n * r);
  int* info = cv.take<int>(2);
  if (!info) return fail(GP_EWORKSPACE, "gp_nystrom_chol_precond: workspace layout failed");
  std::vector<double> sc(d);
  for (int f = 0; f < d; ++f) sc[f] = (kern->kind == GP_MATERN52 ? std::sqrt(5.0) : 1.0) / kern->lengthscale[f];
  const int zero[2] = {0, 0};
  GPK_HIP(hipMemcpyAsync(Mdev, landmarks, sizeof(int64_t) * r, hipMemcpyHostToDevice, st));
  GPK_HIP(hipMemcpyAsync(scd, sc.data(), sizeof(double) * d, hipMemcpyHostToDevice, st));
  GPK_HIP(hipMemcpyAsync(info, zero, sizeof(zero), hipMemcpyHostToDevice, st));
  const unsigned thr = 256;
  iota_kernel<<<(unsigned)((r + thr - 1) / thr), thr, 0, st>>>(iota, r);
  gather_rows_kernel<<<(unsigned)(((int64_t)r * d + thr - 1) / thr), thr, 0, st>>>(X, d, Mdev, r, XM);
  GPK_HIP(hipGetLastError());
  // K_XM column by column (column j = K(X, x_{M_j})) = K_MX row-major r x n; K_MM likewise from the landmark rows
  auto kcols = [&](const double* P, int64_t np, const int64_t* idx, double* out) {
    dim3 grid((unsigned)((np + 255) / 256), (unsigned)((r + kNysTile - 1) / kNysTile));
    if (kern->kind == GP_MATERN52)
      kernel_cols_kernel<GP_MATERN52><<<grid, 256, 0, st>>>(P, np, d, scd, idx, r, kern->outputscale, out);
    else
      kernel_cols_kernel<GP_RBF><<<grid, 256, 0, st>>>(P, np, d, scd, idx, r, kern->outputscale, out);
  };
  kcols(X, n, Mdev, T);
  kcols(XM, r, iota, A);
  GPK_HIP(hipGetLastError());
  // L_M L_M^T = K_MM + delta I (lower triangle), L_M^{-1}
  add_diag_kernel<<<(unsigned)((r + thr - 1) / thr), thr, 0, st>>>(A, r, kNysCholJitter * r * kern->outputscale);
  GPK_HIP(hipGetLastError());
  GPK_HIP(dense_cholesky(A, r, info, Dinv, st));
  GPK_HIP(dense_lower_inverse(A, Linv, Dinv, r, st));
  // F^T = L_M^{-1} K_MX (r x n row-major, i.e. F column-major), into E
  GPK_HIP(dense_gemm(false, false, false, r, n, r, Linv, r, T, n, E, n, st));
  // G = F^T F + sigma^2 I (lower tiles), L_G, L_G^{-1}
  GPK_HIP(dense_gemm(false, true, true, r, r, n, E, n, E, n, A, r, st));
  add_diag_kernel<<<(unsigned)((r + thr - 1) / thr), thr, 0, st>>>(A, r, kern->noise);
  GPK_HIP(hipGetLastError());
  GPK_HIP(dense_cholesky(A, r, info + 1, Dinv, st));
  GPK_HIP(dense_lower_inverse(A, Linv, Dinv, r, st));
  // E^T = L_G^{-1} F^T (r x n row-major = E column-major)
  GPK_HIP(dense_gemm(false, false, false, r, n, r, Linv, r, E, n, T, n, st));
  GPK_HIP(hipMemcpyAsync(E, T, sizeof(double) * n * r, hipMemcpyDeviceToDevice, st));
  int h_info[2] = {0, 0};
  GPK_HIP(hipMemcpyAsync(h_info, info, sizeof(h_info), hipMemcpyDeviceToHost, st));
  GPK_HIP(hipStreamSynchronize(st));
  if (h_info[0] != 0)
    return fail(GP_ENOTPD, "gp_nystrom_chol_precond: K_MM + jitter not positive definite (pivot %d)", h_info[0] - 1);
  if (h_info[1] != 0)
    return fail(GP_ENOTPD, "gp_nystrom_chol_precond: F^T F + sigma^2 I not positive definite (pivot %d)", h_info[1] - 1);
  return GP_OK;
}

// Y = P^{-1} V = sigma^{-2} (V - E (E^T V)) for an n x s block (ld n); Y may alias V.
static hipError_t nystrom_chol_apply(const double* E, int64_t n, int r, double noise, const double* V, int s,
                                     double* Y, double* C1, double* C2, double* part, hipStream_t st) {
  hipError_t e;
  if ((e = gram(E, r, V, s, n, C1, part, st)) != hipSuccess) return e;
  const double inv = 1.0 / noise;
  // C2 = -sigma^{-2} C1
  tall_scale_kernel<<<(unsigned)(((int64_t)r * s + 255) / 256), 256, 0, st>>>(C1, (int64_t)r * s, -inv, C2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return tall_product(E, n, n, r, C2, s, s, inv, V, n, Y, n, false, st);
}

size_t bpcg_ws_bytes(int precision, int d, int64_t n, int r, int s) {
  size_t b = kmm_plan_bytes(precision, d, n, n, true, s);
  b += 5 * align256((size_t)n * s * 8);                              // U, R, Z, D, Q
  b += 2 * align256((size_t)std::max(r, 1) * s * 8);                 // E^T V and its scaled copy
  b += align256(std::max(gram_partial_doubles(n, std::max(r, 1), s), gram_partial_doubles(n, s, s)) * 8);
  b += 3 * align256((size_t)s * s * 8);                              // Gram out, alpha, beta
  return b + 4096;
}

int run_bpcg(const gp_kernel* kern, int precision, const double* X, int64_t n, const double* E, int r,
             const double* B, int64_t ldb, int s, int max_iter, double tol, double* W, int64_t ldw, int32_t* iters_out,
             double* relres, void* ws, size_t ws_bytes, hipStream_t st) {
  const int d = kern->d;
  const size_t kb = kmm_plan_bytes(precision, d, n, n, true, s);
  KmmPlan plan;
  if (!kmm_plan_init(plan, kern, precision, n, n, true, s, ws, kb)) return fail(GP_EWORKSPACE, "gp_bpcg: workspace too small");
  Carve cv((char*)ws + align256(kb), ws_bytes - align256(kb));
  const size_t ns = (size_t)n * s;
  double* U = cv.take<double>(ns);
  double* R = cv.take<double>(ns);
  double* Zb = cv.take<double>(ns);
  double* D = cv.take<double>(ns);
  double* Q = cv.take<double>(ns);
  double* C1 = cv.take<double>((size_t)std::max(r, 1) * s);
  double* C2 = cv.take<double>((size_t)std::max(r, 1) * s);
  double* part = cv.take<double>(std::max(gram_partial_doubles(n, std::max(r, 1), s), gram_partial_doubles(n, s, s)));
  double* Gd = cv.take<double>((size_t)s * s);
  double* Ad = cv.take<double>((size_t)s * s);
  double* Bd = cv.take<double>((size_t)s * s);
  if (!Bd) return fail(GP_EWORKSPACE, "gp_bpcg: workspace layout failed");
  auto precond = [&](const double* in, double* out) -> hipError_t {
    if (r > 0) return nystrom_chol_apply(E, n, r, kern->noise, in, s, out, C1, C2, part, st);
    return hipMemcpyAsync(out, in, sizeof(double) * ns, hipMemcpyDeviceToDevice, st);
  };
  auto gram_host = [&](const double* A, const double* Bm, std::vector<double>& out) -> hipError_t {
    hipError_t e = gram(A, s, Bm, s, n, Gd, part, st);
    if (e != hipSuccess) return e;
    out.resize((size_t)s * s);
    e = hipMemcpyAsync(out.data(), Gd, sizeof(double) * s * s, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
  };
  // R = B, Z = P^{-1} R, D = Z, U = 0
  for (int c = 0; c < s; ++c)
    GPK_HIP(hipMemcpyAsync(R + (size_t)c * n, B + (size_t)c * ldb, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  GPK_HIP(precond(R, Zb));
  GPK_HIP(hipMemcpyAsync(D, Zb, sizeof(double) * ns, hipMemcpyDeviceToDevice, st));
  GPK_HIP(launch_fill(U, 0.0, (int64_t)ns, st));
  GPK_HIP(kmm_prepare(plan, kern, X, nullptr, st));
  std::vector<double> RtZ, RtZn, DtQ, alpha, nalpha, beta;
  GPK_HIP(gram_host(R, Zb, RtZ));
  std::vector<double> bnorm(s);
  for (int c = 0; c < s; ++c) {
    bnorm[c] = std::sqrt(std::max(RtZ[(size_t)c * s + c], 0.0));
    if (!std::isfinite(bnorm[c])) return fail(GP_ENONFINITE, "gp_bpcg: non-finite right-hand side");
    if (!(bnorm[c] > 0.0)) return fail(GP_EINVAL, "gp_bpcg: right-hand side column %d is zero", c);
    relres[c] = 1.0;
  }
  int it = 0;
  bool converged = false;
  while (it < max_iter) {
    GPK_HIP(kmm_apply(plan, D, n, s, Q, n, st, false));
    GPK_HIP(gram_host(D, Q, DtQ));
    if (!host_lu_solve(DtQ, s, RtZ, alpha))
      return fail(GP_ENOTPD, "gp_bpcg: D^T K_hat D singular at iteration %d (block breakdown)", it);
    nalpha = alpha;
    for (auto& v : nalpha) v = -v;
    GPK_HIP(hipMemcpyAsync(Ad, alpha.data(), sizeof(double) * s * s, hipMemcpyHostToDevice, st));
    GPK_HIP(hipMemcpyAsync(Bd, nalpha.data(), sizeof(double) * s * s, hipMemcpyHostToDevice, st));
    GPK_HIP(tall_product(D, n, n, s, Ad, s, s, 1.0, U, n, U, n, false, st));   // U += D alpha
    GPK_HIP(tall_product(Q, n, n, s, Bd, s, s, 1.0, R, n, R, n, false, st));   // R -= Q alpha
    GPK_HIP(precond(R, Zb));
    GPK_HIP(gram_host(R, Zb, RtZn));  // also orders the uploads above before alpha is rewritten
    ++it;
    bool all = true;
    for (int c = 0; c < s; ++c) {
      relres[c] = std::sqrt(std::max(RtZn[(size_t)c * s + c], 0.0)) / bnorm[c];
      if (!std::isfinite(relres[c])) return fail(GP_ENONFINITE, "gp_bpcg: non-finite residual at iteration %d", it);
      all = all && relres[c] <= tol;
    }
    if (all) {
      converged = true;
      break;
    }
    if (it == max_iter) break;
    if (!host_lu_solve(RtZ, s, RtZn, beta))
      return fail(GP_ENOTPD, "gp_bpcg: R^T P^{-1} R singular at iteration %d (block breakdown)", it);
    GPK_HIP(hipMemcpyAsync(Bd, beta.data(), sizeof(double) * s * s, hipMemcpyHostToDevice, st));
    GPK_HIP(tall_product(D, n, n, s, Bd, s, s, 1.0, Zb, n, D, n, false, st));   // D = Z + D beta
    RtZ.swap(RtZn);
    GPK_HIP(hipStreamSynchronize(st));  // beta's upload completes before the host vector is reused
  }
  for (int c = 0; c < s; ++c)
    GPK_HIP(hipMemcpyAsync(W + (size_t)c * ldw, U + (size_t)c * n, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  GPK_HIP(hipStreamSynchronize(st));
  *iters_out = it;
  return converged ? GP_OK : GP_WNOCONV;
}

}  // namespace gpk

using namespace gpk;

static int check_landmarks(const int64_t* M, int r, int64_t n) {
  std::vector<int64_t> v(M, M + r);
  std::sort(v.begin(), v.end());
  for (int i = 0; i < r; ++i) {
    if (v[i] < 0 || v[i] >= n) return fail(GP_EINVAL, "landmark index %lld outside [0, %lld)", (long long)v[i], (long long)n);
    if (i > 0 && v[i] == v[i - 1]) return fail(GP_EINVAL, "landmark %lld repeated", (long long)v[i]);
  }
  return GP_OK;
}

extern "C" int gp_nystrom_precond(const gp_kernel* kern, const double* X, int64_t n, const int64_t* landmarks,
                                  int32_t r, double* Z, double* g, void* ws, size_t ws_bytes, void* stream) {
  GPK_TRY(check_kernel(kern));
  if (!X || !landmarks || !Z || !g) return fail(GP_EINVAL, "gp_nystrom_precond: NULL argument");
  if (n < 1) return fail(GP_EINVAL, "gp_nystrom_precond: n must be >= 1");
  if (r < 1 || r > kNysMaxR || r > n) return fail(GP_EINVAL, "gp_nystrom_precond: r=%d outside [1, min(n, %d)]", r, kNysMaxR);
  if (!(kern->noise > 0.0)) return fail(GP_EINVAL, "gp_nystrom_precond: the noise must be > 0");
  GPK_TRY(check_landmarks(landmarks, r, n));
  GPK_TRY(check_ws(ws, ws_bytes, nystrom_ws_bytes(kern->d, n, r), "gp_nystrom_precond"));
  return run_nystrom(kern, X, n, landmarks, r, Z, g, ws, ws_bytes, (hipStream_t)stream);
}

extern "C" int gp_nystrom_apply(const double* Z, const double* g, int64_t n, int32_t r, double noise,
                                const double* V, int32_t s, double* Y, void* ws, size_t ws_bytes, void* stream) {
  if (!Z || !g || !V || !Y) return fail(GP_EINVAL, "gp_nystrom_apply: NULL argument");
  if (n < 1 || r < 1 || r > kNysMaxR || r > n) return fail(GP_EINVAL, "gp_nystrom_apply: bad n or r");
  if (s < 1 || s > kTallMaxS) return fail(GP_EINVAL, "gp_nystrom_apply: s=%d outside [1, %d]", s, kTallMaxS);
  if (!(noise > 0.0) || !std::isfinite(noise)) return fail(GP_EINVAL, "gp_nystrom_apply: noise must be > 0");
  GPK_TRY(check_ws(ws, ws_bytes, nystrom_apply_ws_bytes(n, r, s), "gp_nystrom_apply"));
  Carve cv(ws, ws_bytes);
  double* C1 = cv.take<double>((size_t)r * s);
  double* C2 = cv.take<double>((size_t)r * s);
  double* part = cv.take<double>(gram_partial_doubles(n, r, s));
  if (!part) return fail(GP_EWORKSPACE, "gp_nystrom_apply: workspace layout failed");
  GPK_HIP(nystrom_apply(Z, g, n, r, noise, V, n, s, Y, n, C1, C2, part, (hipStream_t)stream));
  return GP_OK;
}

extern "C" int gp_bcg(const gp_kernel* kern, int32_t precision, const double* X, int64_t n, const double* Z,
                      const double* g, int32_t r, const double* B, int64_t ldb, int32_t s, int32_t max_iter, double tol,
                      double* W, int64_t ldw, int32_t* iters, double* relres, void* ws, size_t ws_bytes, void* stream) {
  GPK_TRY(check_kernel(kern));
  GPK_TRY(check_product_precision(precision));
  if (!X || !B || !W || !iters || !relres) return fail(GP_EINVAL, "gp_bcg: NULL argument");
  if (n < 1) return fail(GP_EINVAL, "gp_bcg: n must be >= 1");
  if (s < 1 || s > kTallMaxS) return fail(GP_EINVAL, "gp_bcg: s=%d outside [1, %d]", s, kTallMaxS);
  if (ldb < n || ldw < n) return fail(GP_EINVAL, "gp_bcg: ldb and ldw must be >= n");
  if (max_iter < 1) return fail(GP_EINVAL, "gp_bcg: max_iter must be >= 1");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(GP_EINVAL, "gp_bcg: tol must be finite and >= 0");
  if (r < 0 || r > kNysMaxR || r > n) return fail(GP_EINVAL, "gp_bcg: r=%d outside [0, min(n, %d)]", r, kNysMaxR);
  if (r > 0 && (!Z || !g)) return fail(GP_EINVAL, "gp_bcg: r > 0 needs Z and g");
  if (r > 0 && !(kern->noise > 0.0)) return fail(GP_EINVAL, "gp_bcg: the preconditioner needs noise > 0");
  GPK_TRY(check_ws(ws, ws_bytes, bcg_ws_bytes(precision, kern->d, n, r, s), "gp_bcg"));
  return run_bcg(kern, precision, X, n, Z, g, r, B, ldb, s, max_iter, tol, W, ldw, iters, relres, ws, ws_bytes,
                 (hipStream_t)stream);
}

extern "C" int gp_nystrom_chol_precond(const gp_kernel* kern, const double* X, int64_t n, const int64_t* landmarks,
                                       int32_t r, double* E, void* ws, size_t ws_bytes, void* stream) {
  GPK_TRY(check_kernel(kern));
  if (!X || !landmarks || !E) return fail(GP_EINVAL, "gp_nystrom_chol_precond: NULL argument");
  if (n < 1) return fail(GP_EINVAL, "gp_nystrom_chol_precond: n must be >= 1");
  if (r < 1 || r > kNysCholMaxR || r > n)
    return fail(GP_EINVAL, "gp_nystrom_chol_precond: r=%d outside [1, min(n, %d)]", r, kNysCholMaxR);
  if (!(kern->noise > 0.0)) return fail(GP_EINVAL, "gp_nystrom_chol_precond: the noise must be > 0");
  GPK_TRY(check_landmarks(landmarks, r, n));
  GPK_TRY(check_ws(ws, ws_bytes, nystrom_chol_ws_bytes(kern->d, n, r), "gp_nystrom_chol_precond"));
  return run_nystrom_chol(kern, X, n, landmarks, r, E, ws, ws_bytes, (hipStream_t)stream);
}

extern "C" int gp_bpcg(const gp_kernel* kern, int32_t precision, const double* X, int64_t n, const double* E,
                       int32_t r, const double* B, int64_t ldb, int32_t s, int32_t max_iter, double tol, double* W,
                       int64_t ldw, int32_t* iters, double* relres, void* ws, size_t ws_bytes, void* stream) {
  GPK_TRY(check_kernel(kern));
  GPK_TRY(check_product_precision(precision));
  if (!X || !B || !W || !iters || !relres) return fail(GP_EINVAL, "gp_bpcg: NULL argument");
  if (n < 1) return fail(GP_EINVAL, "gp_bpcg: n must be >= 1");
  if (s < 1 || s > kTallMaxS) return fail(GP_EINVAL, "gp_bpcg: s=%d outside [1, %d]", s, kTallMaxS);
  if (ldb < n || ldw < n) return fail(GP_EINVAL, "gp_bpcg: ldb and ldw must be >= n");
  if (max_iter < 1) return fail(GP_EINVAL, "gp_bpcg: max_iter must be >= 1");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(GP_EINVAL, "gp_bpcg: tol must be finite and >= 0");
  if (r < 0 || r > kNysCholMaxR || r > n) return fail(GP_EINVAL, "gp_bpcg: r=%d outside [0, min(n, %d)]", r, kNysCholMaxR);
  if (r > 0 && !E) return fail(GP_EINVAL, "gp_bpcg: r > 0 needs E");
  if (r > 0 && !(kern->noise > 0.0)) return fail(GP_EINVAL, "gp_bpcg: the preconditioner needs noise > 0");
  GPK_TRY(check_ws(ws, ws_bytes, bpcg_ws_bytes(precision, kern->d, n, r, s), "gp_bpcg"));
  return run_bpcg(kern, precision, X, n, E, r, B, ldb, s, max_iter, tol, W, ldw, iters, relres, ws, ws_bytes,
                  (hipStream_t)stream);
}

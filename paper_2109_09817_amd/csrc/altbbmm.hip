// AltBBMM (Sec. 3.2): block conjugate gradients (Sec. 3.1) in FP64 on the
// symmetrically preconditioned system P^{-1/2} K_hat P^{-1/2} Z = P^{-1/2} B,
// W = P^{-1/2} Z, with the Nystrom preconditioner over r landmark rows M
//
//   P = K_XM K_MM^{-1} K_MX + sigma^2 I.
//
// Spectral square root.  With K_MM = L L^T, F = K_XM L^{-T} (so K_XM K_MM^{-1}
// K_MX = F F^T) and the eigendecomposition F^T F = L^{-1} (K_MX K_XM) L^{-T} =
// V diag(S) V^T, the thin SVD F = U S^{1/2} V^T gives P = U diag(S + sigma^2) U^T
// + sigma^2 (I - U U^T), hence
//
//   P^{-1/2} = sigma^{-1} I + K_XM H K_MX,
//   H = L^{-T} V diag(g) V^T L^{-1},  g = ((S + sigma^2)^{-1/2} - sigma^{-1}) / S
//     = -1 / (sigma sqrt(S + sigma^2) (sigma + sqrt(S + sigma^2))).
//
// K_XM (n x r) is materialised once in FP64; H is formed on the host from the
// r x r matrices K_MM and K_MX K_XM.  One application costs two tall-skinny
// products with K_XM.  The block CG recurrences (O'Leary):
//   Q = A D;  alpha = (D^T Q)^{-1} (R^T R);  X += D alpha;  R -= Q alpha;
//   beta = (R_old^T R_old)^{-1} (R^T R);  D = R + D beta,
// with the s x s Gram matrices reduced on the GPU and factorised on the host.
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

// Y = alpha V + A C for A (nrows x kk, column-major, lda), C (kk x s, row-major),
// V and Y (nrows x s): column-major with ldv / ldy, or (ROWMAJOR) row-major with
// s per row.  One thread per row; each thread reads all of its row of A before
// writing its row of Y, so Y may alias A or V.
template <bool ROWMAJOR>
__global__ __launch_bounds__(256) void tall_product_kernel(const double* __restrict__ A, int64_t lda,
                                                           int64_t nrows, int kk, const double* __restrict__ C,
                                                           int s, double alpha, const double* V, int64_t ldv,
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
      Cs[k][c] = (k0 + k < kk && c < s) ? C[(int64_t)(k0 + k) * s + c] : 0.0;
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

static hipError_t tall_product(const double* A, int64_t lda, int64_t nrows, int kk, const double* C, int s,
                               double alpha, const double* V, int64_t ldv, double* Y, int64_t ldy, bool rowmajor,
                               hipStream_t st) {
  const unsigned grid = (unsigned)((nrows + 255) / 256);
  if (rowmajor)
    tall_product_kernel<true><<<grid, 256, 0, st>>>(A, lda, nrows, kk, C, s, alpha, V, ldv, Y, ldy);
  else
    tall_product_kernel<false><<<grid, 256, 0, st>>>(A, lda, nrows, kk, C, s, alpha, V, ldv, Y, ldy);
  return hipGetLastError();
}

// A^T B with the row split sized to the output: ~2048 workgroups whatever pa, qb.
static int64_t gram_blocks(int64_t n, int pa, int qb) {
  const int64_t tiles = (int64_t)((pa + 63) / 64) * ((qb + 63) / 64);
  return std::max<int64_t>(1, std::min<int64_t>((n + 63) / 64, 2048 / tiles));
}
static size_t gram_partial_doubles(int64_t n, int pa, int qb) {
  return (size_t)gram_blocks(n, pa, qb) * pa * qb;
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
  b += 2 * align256((size_t)r * r * 8);                        // K_MM, K_MX K_XM
  b += align256(gram_partial_doubles(n, r, r) * 8);            // Gram partials
  return b + 4096;
}

// host: solve L Y = B (L lower, row-major k x k; B row-major k x m, overwritten)
static void host_lower_solve(const std::vector<double>& L, int k, std::vector<double>& B, int m) {
  for (int i = 0; i < k; ++i) {
    double* bi = &B[(size_t)i * m];
    for (int j = 0; j < i; ++j) {
      const double l = L[(size_t)i * k + j];
      const double* bj = &B[(size_t)j * m];
      for (int c = 0; c < m; ++c) bi[c] -= l * bj[c];
    }
    const double inv = 1.0 / L[(size_t)i * k + i];
    for (int c = 0; c < m; ++c) bi[c] *= inv;
  }
}
// host: solve L^T Y = B
static void host_upper_solve(const std::vector<double>& L, int k, std::vector<double>& B, int m) {
  for (int i = k - 1; i >= 0; --i) {
    double* bi = &B[(size_t)i * m];
    for (int j = i + 1; j < k; ++j) {
      const double l = L[(size_t)j * k + i];
      const double* bj = &B[(size_t)j * m];
      for (int c = 0; c < m; ++c) bi[c] -= l * bj[c];
    }
    const double inv = 1.0 / L[(size_t)i * k + i];
    for (int c = 0; c < m; ++c) bi[c] *= inv;
  }
}
static void host_transpose(std::vector<double>& A, int k) {
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j) std::swap(A[(size_t)i * k + j], A[(size_t)j * k + i]);
}

int run_nystrom(const gp_kernel* kern, const double* X, int64_t n, const int64_t* landmarks, int r, double* KXM,
                double* H, void* ws, size_t ws_bytes, hipStream_t st) {
  const int d = kern->d;
  Carve cv(ws, ws_bytes);
  int64_t* Mdev = cv.take<int64_t>(r);
  double* scd = cv.take<double>(d);
  double* KMM = cv.take<double>((size_t)r * r);
  double* G = cv.take<double>((size_t)r * r);
  double* part = cv.take<double>(gram_partial_doubles(n, r, r));
  if (!part) return fail(GP_EWORKSPACE, "gp_nystrom_precond: workspace layout failed");
  std::vector<double> sc(d);
  for (int f = 0; f < d; ++f)
    sc[f] = (kern->kind == GP_MATERN52 ? std::sqrt(5.0) : 1.0) / kern->lengthscale[f];
  GPK_HIP(hipMemcpyAsync(Mdev, landmarks, sizeof(int64_t) * r, hipMemcpyHostToDevice, st));
  GPK_HIP(hipMemcpyAsync(scd, sc.data(), sizeof(double) * d, hipMemcpyHostToDevice, st));
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)((r + kNysTile - 1) / kNysTile));
  if (kern->kind == GP_MATERN52)
    kernel_cols_kernel<GP_MATERN52><<<grid, 256, 0, st>>>(X, n, d, scd, Mdev, r, kern->outputscale, KXM);
  else
    kernel_cols_kernel<GP_RBF><<<grid, 256, 0, st>>>(X, n, d, scd, Mdev, r, kern->outputscale, KXM);
  GPK_HIP(hipGetLastError());
  gather_landmark_rows_kernel<<<(unsigned)(((int64_t)r * r + 255) / 256), 256, 0, st>>>(KXM, n, Mdev, r, KMM);
  GPK_HIP(hipGetLastError());
  GPK_HIP(gram(KXM, r, KXM, r, n, G, part, st));
  std::vector<double> L((size_t)r * r), T((size_t)r * r);
  GPK_HIP(hipMemcpyAsync(L.data(), KMM, sizeof(double) * r * r, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipMemcpyAsync(T.data(), G, sizeof(double) * r * r, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipStreamSynchronize(st));
  for (size_t e = 0; e < L.size(); ++e)
    if (!std::isfinite(L[e]) || !std::isfinite(T[e])) return fail(GP_ENONFINITE, "gp_nystrom_precond: non-finite kernel");
  // K_MM is stored column by column; it is symmetric up to the order of its evaluation
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < i; ++j) L[(size_t)i * r + j] = L[(size_t)j * r + i] = 0.5 * (L[(size_t)i * r + j] + L[(size_t)j * r + i]);
  if (!host_cholesky(L, r)) return fail(GP_ENOTPD, "gp_nystrom_precond: K_MM is not positive definite (repeated landmarks?)");
  // T = L^{-1} G L^{-T}  (G symmetric: L^{-1} (L^{-1} G)^T)
  host_lower_solve(L, r, T, r);
  host_transpose(T, r);
  host_lower_solve(L, r, T, r);
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < i; ++j) T[(size_t)i * r + j] = T[(size_t)j * r + i] = 0.5 * (T[(size_t)i * r + j] + T[(size_t)j * r + i]);
  std::vector<double> S, V;
  if (!sym_eig(r, T, S, V)) return fail(GP_ENOTPD, "gp_nystrom_precond: eigen-decomposition did not converge");
  const double sig = std::sqrt(kern->noise);
  // K2 = V diag(g) V^T
  std::vector<double> K2((size_t)r * r, 0.0), gv(r);
  for (int m = 0; m < r; ++m) {
    const double sm = std::max(S[m], 0.0);
    const double q = std::sqrt(sm + kern->noise);
    gv[m] = -1.0 / (sig * q * (sig + q));
  }
  for (int i = 0; i < r; ++i)
    for (int m = 0; m < r; ++m) {
      const double vg = V[(size_t)i * r + m] * gv[m];
      double* row = &K2[(size_t)i * r];
      const double* vrow = &V[0];
      for (int j = 0; j < r; ++j) row[j] += vg * vrow[(size_t)j * r + m];
    }
  // H = L^{-T} K2 L^{-1}  (K2 symmetric: L^{-T} (L^{-T} K2)^T)
  host_upper_solve(L, r, K2, r);
  host_transpose(K2, r);
  host_upper_solve(L, r, K2, r);
  for (size_t e = 0; e < K2.size(); ++e)
    if (!std::isfinite(K2[e])) return fail(GP_ENONFINITE, "gp_nystrom_precond: non-finite H");
  GPK_HIP(hipMemcpyAsync(H, K2.data(), sizeof(double) * r * r, hipMemcpyHostToDevice, st));
  GPK_HIP(hipStreamSynchronize(st));
  return GP_OK;
}

// ---------------------------------------------------------------- apply P^{-1/2}

size_t nystrom_apply_ws_bytes(int64_t n, int r, int s) {
  return 2 * align256((size_t)r * s * 8) + align256(gram_partial_doubles(n, std::max(r, 1), s) * 8) + 1024;
}

// Y = sigma^{-1} V + K_XM (H (K_XM^T V)); Y may alias V.
static hipError_t nystrom_apply(const double* KXM, const double* H, int64_t n, int r, double noise, const double* V,
                                int64_t ldv, int s, double* Y, int64_t ldy, double* C1, double* C2, double* part,
                                hipStream_t st) {
  hipError_t e;
  if (ldv != n) return hipErrorInvalidValue;  // gram() takes ld = n
  if ((e = gram(KXM, r, V, s, n, C1, part, st)) != hipSuccess) return e;
  if ((e = tall_product(H, r, r, r, C1, s, 0.0, nullptr, 0, C2, 0, true, st)) != hipSuccess) return e;
  return tall_product(KXM, n, n, r, C2, s, 1.0 / std::sqrt(noise), V, ldv, Y, ldy, false, st);
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

// s x s: X = A^{-1} B with A symmetric positive definite (row-major); false on breakdown.
static bool host_spd_solve(std::vector<double> A, int s, const std::vector<double>& B, std::vector<double>& X) {
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < i; ++j) A[(size_t)i * s + j] = A[(size_t)j * s + i] = 0.5 * (A[(size_t)i * s + j] + A[(size_t)j * s + i]);
  if (!host_cholesky(A, s)) return false;
  X = B;
  host_lower_solve(A, s, X, s);
  host_upper_solve(A, s, X, s);
  for (double v : X)
    if (!std::isfinite(v)) return false;
  return true;
}

int run_bcg(const gp_kernel* kern, int precision, const double* X, int64_t n, const double* KXM, const double* H,
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
    if (pre) return nystrom_apply(KXM, H, n, r, kern->noise, in, n, s, out, n, C1, C2, part, st);
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
    if (!host_spd_solve(DtQ, s, RtR, alpha))
      return fail(GP_ENOTPD, "gp_bcg: D^T A D not positive definite at iteration %d (block breakdown)", it);
    nalpha = alpha;
    for (auto& v : nalpha) v = -v;
    GPK_HIP(hipMemcpyAsync(Ad, alpha.data(), sizeof(double) * s * s, hipMemcpyHostToDevice, st));
    GPK_HIP(hipMemcpyAsync(Bd, nalpha.data(), sizeof(double) * s * s, hipMemcpyHostToDevice, st));
    GPK_HIP(tall_product(D, n, n, s, Ad, s, 1.0, Z, n, Z, n, false, st));   // Z += D alpha
    GPK_HIP(tall_product(Q, n, n, s, Bd, s, 1.0, R, n, R, n, false, st));   // R -= Q alpha
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
    if (!host_spd_solve(RtR, s, RtRn, beta))
      return fail(GP_ENOTPD, "gp_bcg: R^T R singular at iteration %d (block breakdown)", it);
    GPK_HIP(hipMemcpyAsync(Bd, beta.data(), sizeof(double) * s * s, hipMemcpyHostToDevice, st));
    GPK_HIP(tall_product(D, n, n, s, Bd, s, 1.0, R, n, D, n, false, st));   // D = R + D beta
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
                                  int32_t r, double* KXM, double* H, void* ws, size_t ws_bytes, void* stream) {
  GPK_TRY(check_kernel(kern));
  if (!X || !landmarks || !KXM || !H) return fail(GP_EINVAL, "gp_nystrom_precond: NULL argument");
  if (n < 1) return fail(GP_EINVAL, "gp_nystrom_precond: n must be >= 1");
  if (r < 1 || r > kNysMaxR || r > n) return fail(GP_EINVAL, "gp_nystrom_precond: r=%d outside [1, min(n, %d)]", r, kNysMaxR);
  if (!(kern->noise > 0.0)) return fail(GP_EINVAL, "gp_nystrom_precond: the noise must be > 0");
  GPK_TRY(check_landmarks(landmarks, r, n));
  GPK_TRY(check_ws(ws, ws_bytes, nystrom_ws_bytes(kern->d, n, r), "gp_nystrom_precond"));
  return run_nystrom(kern, X, n, landmarks, r, KXM, H, ws, ws_bytes, (hipStream_t)stream);
}

extern "C" int gp_nystrom_apply(const double* KXM, const double* H, int64_t n, int32_t r, double noise,
                                const double* V, int32_t s, double* Y, void* ws, size_t ws_bytes, void* stream) {
  if (!KXM || !H || !V || !Y) return fail(GP_EINVAL, "gp_nystrom_apply: NULL argument");
  if (n < 1 || r < 1 || r > kNysMaxR || r > n) return fail(GP_EINVAL, "gp_nystrom_apply: bad n or r");
  if (s < 1 || s > kTallMaxS) return fail(GP_EINVAL, "gp_nystrom_apply: s=%d outside [1, %d]", s, kTallMaxS);
  if (!(noise > 0.0) || !std::isfinite(noise)) return fail(GP_EINVAL, "gp_nystrom_apply: noise must be > 0");
  GPK_TRY(check_ws(ws, ws_bytes, nystrom_apply_ws_bytes(n, r, s), "gp_nystrom_apply"));
  Carve cv(ws, ws_bytes);
  double* C1 = cv.take<double>((size_t)r * s);
  double* C2 = cv.take<double>((size_t)r * s);
  double* part = cv.take<double>(gram_partial_doubles(n, r, s));
  if (!part) return fail(GP_EWORKSPACE, "gp_nystrom_apply: workspace layout failed");
  GPK_HIP(nystrom_apply(KXM, H, n, r, noise, V, n, s, Y, n, C1, C2, part, (hipStream_t)stream));
  return GP_OK;
}

extern "C" int gp_bcg(const gp_kernel* kern, int32_t precision, const double* X, int64_t n, const double* KXM,
                      const double* H, int32_t r, const double* B, int64_t ldb, int32_t s, int32_t max_iter, double tol,
                      double* W, int64_t ldw, int32_t* iters, double* relres, void* ws, size_t ws_bytes, void* stream) {
  GPK_TRY(check_kernel(kern));
  GPK_TRY(check_precision(precision));
  if (!X || !B || !W || !iters || !relres) return fail(GP_EINVAL, "gp_bcg: NULL argument");
  if (n < 1) return fail(GP_EINVAL, "gp_bcg: n must be >= 1");
  if (s < 1 || s > kTallMaxS) return fail(GP_EINVAL, "gp_bcg: s=%d outside [1, %d]", s, kTallMaxS);
  if (ldb < n || ldw < n) return fail(GP_EINVAL, "gp_bcg: ldb and ldw must be >= n");
  if (max_iter < 1) return fail(GP_EINVAL, "gp_bcg: max_iter must be >= 1");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(GP_EINVAL, "gp_bcg: tol must be finite and >= 0");
  if (r < 0 || r > kNysMaxR || r > n) return fail(GP_EINVAL, "gp_bcg: r=%d outside [0, min(n, %d)]", r, kNysMaxR);
  if (r > 0 && (!KXM || !H)) return fail(GP_EINVAL, "gp_bcg: r > 0 needs KXM and H");
  if (r > 0 && !(kern->noise > 0.0)) return fail(GP_EINVAL, "gp_bcg: the preconditioner needs noise > 0");
  GPK_TRY(check_ws(ws, ws_bytes, bcg_ws_bytes(precision, kern->d, n, r, s), "gp_bcg"));
  return run_bcg(kern, precision, X, n, KXM, H, r, B, ldb, s, max_iter, tol, W, ldw, iters, relres, ws, ws_bytes,
                 (hipStream_t)stream);
}

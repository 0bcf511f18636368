/*
 * gpkmm.h - C ABI of an MI355X (gfx950) library for exact Gaussian-process
 * training and prediction with never-materialised kernel-matrix products.
 *
 * The method is BBMM as used by Sun, Cheng & Miller, "Molecular Energy
 * Learning Using Alternative Blackbox Matrix-Matrix Multiplication Algorithm
 * for Exact Gaussian Process": the log marginal likelihood (Eq. 2), its
 * gradient and the predictive equations (Eq. 1) are obtained from products
 * K_hat V with K_hat = K(X, X) + sigma^2 I (Sec. 2.2), inside preconditioned
 * modified batched CG (mBCG, Sec. 3.1-3.2) with a pivoted-Cholesky
 * preconditioner (Sec. 3.2).  K_hat is recomputed tile by tile and never
 * stored, so memory is O(N) (Sec. 3.2; the paper batches tiles of 4096 x 4096,
 * Sec. 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - X (n x d) and query rows Z (m x d) are FP64, row-major (point i occupies
 *   X[i*d .. i*d+d-1]), in device memory.
 * - A block of t vectors of length n ("columns") is FP64 and column-major:
 *   column c starts at V + c*ldv, ldv >= n.
 * - Every pointer documented "device" is a HIP device allocation owned by the
 *   caller; "host" pointers are ordinary host memory.  The library never
 *   frees, retains or reallocates caller memory after a call returns.
 * - Scratch memory is the caller's: ws / ws_bytes, at least
 *   gp_workspace_bytes(op, ...) bytes of device memory, 256-byte aligned.
 * - stream is a hipStream_t (NULL: the null stream).  Calls whose outputs are
 *   all in device memory are asynchronous on that stream; calls with host
 *   outputs synchronise the stream before they return.
 * - Return value: 0 on success, GP_WNOCONV (> 0) for a valid result that did
 *   not meet its tolerance, a negative GP_E* code on error (outputs are then
 *   unspecified).  Arguments are validated on the host before any GPU work;
 *   gp_last_error() returns a message for the last non-zero status of the
 *   calling thread.
 * - Hyperparameter gradients are taken with respect to
 *   (log l_1 .. log l_d, log s_f, log sigma^2), in that order (d + 2 values).
 */
#ifndef GPKMM_H
#define GPKMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define GP_OK 0
#define GP_WNOCONV 1       /* iteration limit hit; outputs valid */
#define GP_EINVAL (-1)     /* bad argument (checked before any GPU work) */
#define GP_EWORKSPACE (-2) /* ws NULL, misaligned or smaller than required */
#define GP_EHIP (-3)       /* HIP runtime error (message from the runtime) */
#define GP_ENOTPD (-4)     /* a curvature d^T K_hat d <= 0 or a factor not positive definite */
#define GP_ENONFINITE (-5) /* NaN or Inf met in a reduction */

/* ---- kernel families ---- */
#define GP_MATERN52 0 /* k(r) = s_f (1 + sqrt5 r + 5 r^2/3) exp(-sqrt5 r)  (Sec. 4) */
#define GP_RBF 1      /* k(r) = s_f exp(-r^2/2) */

/* ---- arithmetic of the kernel-matrix products ---- */
#define GP_PREC_FP32 0   /* FP32 matrix-core operands and accumulation */
/* Mixed: every operand split hi + lo in FP16 (22 significant bits), three products
 * hi.hi + hi.lo + lo.hi on the FP16 matrix cores, FP32 accumulation.  The distance uses
 * the scaled coordinates centred on the training points' column means m; the kernel
 * values enter as 2^15 m(r) and each column of V scaled by the power of two that puts
 * its largest entry in [2^14, 2^15), scalings undone exactly in FP64 (in gp_kmm_grad the
 * kernel-weighted values and the columns [x~ | x~^2] take FP16 halves after power-of-two
 * scalings per wave's rows and per column, the operands of C = U diag(w) W^T BF16 halves).
 * FP16 bounds the
 * scaled coordinates: |x_j - m_j| / l_j up to about 10^4
 * (Matern-5/2; about 3.8 10^4 for RBF), for training and query rows alike.  A point beyond
 * makes every product involving it NaN (gp_mbcg then fails with GP_ENONFINITE);
 * GP_PREC_FP32 has no such bound. */
#define GP_PREC_BF16X3 1
#define GP_PREC_FP64 2   /* FP64 throughout (low-noise regime); gp_kmm, gp_mbcg and gp_bcg only, d <= 64 */

#define GP_MAX_D 128 /* largest feature count d */

/* ---- workspace query operation codes ---- */
#define GP_OP_KMM 1
#define GP_OP_KMM_GRAD 2
#define GP_OP_PIVCHOL 3
#define GP_OP_MBCG 4
#define GP_OP_MLL 5
#define GP_OP_PREDICT 6
#define GP_OP_LANCZOS 7
#define GP_OP_PREDICT_RUN 8
#define GP_OP_NYSTROM 9
#define GP_OP_NYSTROM_APPLY 10
#define GP_OP_BCG 11
#define GP_OP_EXACT 12
#define GP_OP_NYSTROM_CHOL 13
#define GP_OP_BPCG 14

/*
 * ARD stationary kernel with r^2 = sum_j ((x_j - z_j) / l_j)^2 (Sec. 2.2;
 * Matern-5/2 per Sec. 4).  lengthscale: host, d entries, each finite and > 0.
 * outputscale s_f > 0.  noise: the total sigma^2 >= 0 on the diagonal of
 * K_hat (the paper adds a regulariser sigma^2_add to the optimised noise,
 * Sec. 4; pass the sum).
 */
typedef struct gp_kernel {
  int32_t kind;
  int32_t d;
  const double* lengthscale;
  double outputscale;
  double noise;
} gp_kernel;

/*
 * Preconditioner P = L L^T + sigma^2 I from a rank-k pivoted Cholesky factor
 * of K (Sec. 3.2).  rank = 0 means P = I (L and Cchol ignored).
 * L: device, n x rank, column-major with leading dimension n.
 * Cchol: device, rank x rank, column-major lower Cholesky factor of
 * C = sigma^2 I + L^T L (upper triangle ignored).
 */
typedef struct gp_precond {
  int32_t rank;
  const double* L;
  const double* Cchol;
} gp_precond;

/* Per-column record of an mBCG run (all host arrays, caller-allocated). */
typedef struct gp_mbcg_out {
  double* alpha;   /* nullable; max_iter x s, entry [j*s + c] = alpha of column c at iteration j */
  double* beta;    /* nullable; same layout (0 after a column froze) */
  int32_t* iters;  /* nullable; s entries: iterations J_c run by column c */
  double* relres;  /* nullable; s entries: final ||r_c|| / ||b_c|| of the recurrence */
  double* gamma0;  /* nullable; s entries: b_c^T P^{-1} b_c */
  int32_t total_iters; /* out: iterations of the whole block */
} gp_mbcg_out;

/* Options of one marginal-likelihood evaluation. */
typedef struct gp_mll_opts {
  int32_t probes;    /* t >= 1 probe vectors (block is [y | b_1..b_t]) */
  int32_t rank;      /* k >= 0 pivoted-Cholesky rank */
  int32_t max_iter;  /* >= 1 */
  int32_t precision; /* GP_PREC_* */
  double tol;        /* relative residual at which a column freezes (0: run max_iter) */
  uint64_t seed;     /* probe seed */
} gp_mll_opts;

/* Diagnostics of gp_mll_and_grad (host struct, nullable). */
typedef struct gp_mll_info {
  int32_t iters;      /* mBCG iterations run */
  int32_t rank;       /* preconditioner rank reached */
  double logdet;      /* SLQ estimate of log|K_hat| */
  double logdet_p;    /* log|P| */
  double quad;        /* y^T K_hat^{-1} y */
  double max_relres;  /* largest final relative residual over the block */
  double ms_precond, ms_mbcg, ms_grad; /* phase wall times */
} gp_mll_info;

/*
 * gp_kmm - the kernel-matrix product (Sec. 3.1: CG needs only products with
 * K_hat, each O(N^2), which are amenable to GPU acceleration).
 *   Z == NULL : out = K_hat V = (K(X, X) + sigma^2 I) V, m ignored, out is n x t.
 *   Z != NULL : out = K(Z, X) V (no noise), the cross-covariance product of the
 *               predictive equations (Eq. 1); out is m x t.
 * X: device n x d; Z: device m x d or NULL; V: device n x t (ldv >= n);
 * out: device (n or m) x t (ldo >= rows), must not overlap V.
 * n >= 1, 1 <= t <= 4096.  Asynchronous on stream.
 */
int gp_kmm(const gp_kernel* kern, int32_t precision,
           const double* X, int64_t n, const double* Z, int64_t m,
           const double* V, int64_t ldv, int32_t t,
           double* out, int64_t ldo,
           void* ws, size_t ws_bytes, void* stream);

/*
 * gp_kmm_noalloc - gp_kmm for callers that cannot allocate device memory at
 * call time (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same product, arguments and results as gp_kmm, with
 * its scratch in a fixed array of GP_KMM_NOALLOC_MAX_BYTES that the library
 * holds on every device it is loaded on until the process ends, instead of a
 * caller workspace.  The call itself allocates nothing.  Returns GP_EWORKSPACE
 * (before any GPU work) when the product needs more scratch than that, i.e.
 * gp_workspace_bytes(GP_OP_KMM, ...) > GP_KMM_NOALLOC_MAX_BYTES (every square
 * product with n <= 5,500, d <= 48 and t <= 16 fits, in either matrix-core
 * precision; larger ones may, depending on how the sweep splits).  All calls on one device share
 * that device's array: calls that overlap in time on one device (different host
 * threads, or streams not ordered with each other) race.  Asynchronous on
 * stream; the device is the stream's (the current device for NULL).
 */
#define GP_KMM_NOALLOC_MAX_BYTES (64ull << 20)
int gp_kmm_noalloc(const gp_kernel* kern, int32_t precision,
                   const double* X, int64_t n, const double* Z, int64_t m,
                   const double* V, int64_t ldv, int32_t t,
                   double* out, int64_t ldo, void* stream);

/*
 * gp_kmm_grad - derivative bilinear forms for the gradient of Eq. 2:
 *   grad[j] = sum_c colw[c] * U_c^T (dK_hat / dlog theta_j) W_c
 * with dK_ab/dlog l_j = psi(r_ab) ((x_aj - x_bj)/l_j)^2, dK_hat/dlog s_f = K
 * and dK_hat/dlog sigma^2 = sigma^2 I.  Tiles are recomputed, never stored.
 * U, W: device n x t with ldu = ldw = n, t <= 64, d <= 64; colw: host, t
 * weights; grad: host, d + 2 values.  precision selects the matrix-core form
 * of the tile products (distances, C = U diag(w) W^T and psi (.) C times the
 * columns [x~ | x~^2]) as for gp_kmm; the BF16X3 form visits each unordered
 * pair a < b once with C + C^T.  Synchronous.
 */
int gp_kmm_grad(const gp_kernel* kern, int32_t precision,
                const double* X, int64_t n,
                const double* U, int64_t ldu, const double* W, int64_t ldw, int32_t t,
                const double* colw, double* grad,
                void* ws, size_t ws_bytes, void* stream);

/*
 * gp_pivchol_precond - greedy rank-k pivoted Cholesky factor of K (without
 * noise), the BBMM preconditioner (Sec. 3.2).  Pivot m is the unpivoted row
 * with the largest residual diagonal (lowest index on ties); the factor stops
 * early when that residual is <= 1e-12 s_f.  Also forms C = sigma^2 I + L^T L,
 * its Cholesky factor, and log|P| = (n - rank) log sigma^2 + log|C|.
 * Requires sigma^2 > 0 and 1 <= k <= min(n, 1024).
 * L: device n x k (column-major, ld n; columns >= rank are zero);
 * Cchol: device k x k; piv: host k entries (nullable); rank, logdetP: host.
 * Synchronous.
 */
int gp_pivchol_precond(const gp_kernel* kern, const double* X, int64_t n, int32_t k,
                       double* L, double* Cchol, int64_t* piv, int32_t* rank, double* logdetP,
                       void* ws, size_t ws_bytes, void* stream);

/*
 * gp_mbcg - modified batched preconditioned CG (Sec. 3.2): s independent CG
 * recurrences on K_hat U = B sharing each product K_hat D.  Column c freezes
 * once ||r_c|| <= tol ||b_c||.  FP64 recurrences; products per `precision`.
 * pc: preconditioner (NULL: P = I); B: device n x s; U: device n x s output
 * (K_hat^{-1} B); Z0: device n x s output P^{-1} B (nullable).  s <= 256.
 * Synchronises once per iteration.  Returns GP_WNOCONV if some column had
 * not converged after max_iter iterations (tol > 0).
 */
int gp_mbcg(const gp_kernel* kern, int32_t precision,
            const double* X, int64_t n, const gp_precond* pc,
            const double* B, int32_t s, int32_t max_iter, double tol,
            double* U, double* Z0, gp_mbcg_out* out,
            void* ws, size_t ws_bytes, void* stream);

/*
 * gp_probe_block - the right-hand-side block [y | b_1..b_t] (Sec. 3.1 sets
 * y_0 = y and random y_i), with Rademacher probes b_i = L e1_i + sigma e2_i
 * (E[b b^T] = P) or b_i = e2_i when k = 0.  Signs: top bit of one SplitMix64
 * step from key ^ ((stream << 40) | row), key = one step from seed; probe i uses
 * stream i for e2 and i + 65536 for e1.
 * y: device n; L: device n x k (ld n) or NULL when k = 0; B: device n x (t+1).
 */
int gp_probe_block(const double* y, int64_t n, int32_t t, const double* L, int32_t k,
                   double noise, uint64_t seed, double* B, void* stream);

/*
 * gp_mll_and_grad - one BBMM evaluation of the log marginal likelihood (Eq. 2)
 * and of its gradient: pivoted-Cholesky preconditioner, probe block,
 * mBCG, stochastic Lanczos quadrature for log|K_hat| and stochastic trace
 * estimates for the gradient (Sec. 3.2).
 * X: device n x d; y: device n; mll: host; grad: host d + 2 (nullable: no
 * gradient); info: host (nullable).  Synchronous.
 */
int gp_mll_and_grad(const gp_kernel* kern, const gp_mll_opts* opts,
                    const double* X, const double* y, int64_t n,
                    double* mll, double* grad, gp_mll_info* info,
                    void* ws, size_t ws_bytes, void* stream);

/*
 * gp_lanczos_cache - rank-kc Lanczos decomposition K_hat Q = Q T (full FP64
 * re-orthogonalisation, start y / ||y||) and the variance cache
 * R = Q L_T^{-T} with T = L_T L_T^T, so that R R^T = Q T^{-1} Q^T ~ K_hat^{-1}
 * for the variance of Eq. 1.  R: device n x kc (ld n); kc_out: host, the rank
 * reached (< kc if the Krylov space closed).  Synchronous.
 */
int gp_lanczos_cache(const gp_kernel* kern, int32_t precision,
                     const double* X, const double* y, int64_t n, int32_t kc,
                     double* R, int32_t* kc_out,
                     void* ws, size_t ws_bytes, void* stream);

/*
 * gp_predict - predictive mean K(Z, X) alpha and latent variance
 * s_f - ||K(z, X) R||^2 at m query rows (Eq. 1, with the prior term that the
 * printed variance leaves out), from alpha = K_hat^{-1} y and a variance cache
 * R.  X: device n x d; alpha: device n; R: device n x kc (ld n) or NULL;
 * Z: device m x d; mean: device m; var: device m (nullable; needs R).
 * Each row's result depends only on that row (not on the other rows of the
 * call).  Asynchronous.  GP_EINVAL for a NULL X, alpha, Z or mean, m < 1, or
 * var without a cache, and GP_EWORKSPACE for a short workspace, all before
 * any GPU work.
 */
int gp_predict(const gp_kernel* kern, int32_t precision,
               const double* X, int64_t n, const double* alpha,
               const double* R, int32_t kc,
               const double* Z, int64_t m, double* mean, double* var,
               void* ws, size_t ws_bytes, void* stream);

/*
 * Prepared prediction model for serving (Eq. 1): the training-side operands of
 * K(Z, X) [alpha | R] (the split fragments of X and of the kc + 1 columns
 * [alpha | R]) computed once into a caller-owned device buffer `model`, so
 * that each batch of query rows pays only for its own rows.
 * gp_predict_model_bytes: size of `model` (0 for invalid arguments).
 * gp_predict_prepare: fills `model` from X (device n x d), alpha (device n)
 *   and R (device n x kc, ld n; NULL when kc = 0).  Asynchronous.
 * gp_predict_run: mean (device m) and, when var is non-NULL and kc >= 1, the
 *   latent variance s_f - ||K(z, X) R||^2 (device m) for query rows Z (device
 *   m x d).  Workspace: gp_workspace_bytes(GP_OP_PREDICT_RUN, n, m, d, 0, kc,
 *   precision).  Each row's result is bitwise independent of the other rows in
 *   the call.  Asynchronous; `model` must stay unchanged while it is in use.
 */
size_t gp_predict_model_bytes(const gp_kernel* kern, int32_t precision, int64_t n, int32_t kc);
int gp_predict_prepare(const gp_kernel* kern, int32_t precision, const double* X, int64_t n,
                       const double* alpha, const double* R, int32_t kc,
                       void* model, size_t model_bytes, void* stream);
int gp_predict_run(const gp_kernel* kern, int32_t precision, const void* model, int64_t n, int32_t kc,
                   const double* Z, int64_t m, double* mean, double* var,
                   void* ws, size_t ws_bytes, void* stream);

/*
 * gp_lanczos_quadrature - host utility of stochastic Lanczos quadrature:
 * e_1^T log(T) e_1 for the J x J Lanczos tridiagonal T built from one column's
 * CG coefficients (T_00 = 1/alpha_0, T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
 * T_j,j-1 = sqrt(beta_{j-1})/alpha_{j-1}), read as alpha[j*stride],
 * beta[j*stride].  Returns GP_ENOTPD if T is not positive definite.
 */
int gp_lanczos_quadrature(const double* alpha, const double* beta, int32_t J, int32_t stride, double* out);

/*
 * gp_nystrom_precond - the AltBBMM preconditioner (Sec. 3.2, Sec. 4): the
 * Nystrom approximation over r landmark rows M,
 *   P = K_XM K_MM^{-1} K_MX + sigma^2 I,
 * in the factored form of its inverse square root
 *   P^{-1/2} = sigma^{-1} I + Z^T diag(g) Z,
 * where Z^T = U_F S^{1/2} is the thin SVD factor of F = K_XM C, C C^T the
 * inverse of K_MM, and g_m = -1 / (sigma q_m (sigma + q_m)), q_m = sqrt(S_m +
 * sigma^2).  K_MM^{-1} is the pseudo-inverse over the eigenvalues of K_MM
 * above 1e-7 of the largest (nearly repeated landmarks make K_MM numerically
 * singular; the dropped directions are left to CG), so only the first k <= r
 * rows of Z are used: rows k..r-1 and g[k..r-1] are zero.
 * landmarks: host, r distinct indices in [0, n) (the paper draws them at
 * random; pass the draw).  Z: device, r x n row-major (row m = factor column
 * m; the sum of Z_m Z_m^T is the approximation K_XM K_MM^{-1} K_MX).  g:
 * device, r.  Both FP64, owned by the caller.
 * Requires sigma^2 > 0 and 1 <= r <= min(n, 1024).  Errors: GP_EINVAL (sizes,
 * repeated or out-of-range landmarks), GP_ENOTPD (K_MM numerically zero, or an
 * eigendecomposition that does not converge), GP_ENONFINITE, GP_EWORKSPACE,
 * GP_EHIP.  Synchronous (the two r x r eigendecompositions run on the host).
 * Workspace: gp_workspace_bytes(GP_OP_NYSTROM, n, 0, d, 0, r, any precision).
 */
int gp_nystrom_precond(const gp_kernel* kern, const double* X, int64_t n,
                       const int64_t* landmarks, int32_t r, double* Z, double* g,
                       void* ws, size_t ws_bytes, void* stream);

/*
 * gp_nystrom_apply - Y = P^{-1/2} V = sigma^{-1} V + Z^T (diag(g) (Z V)) for
 * a device n x s block V (column-major, ld = n), s <= 64; Y likewise (may
 * equal V).  Z, g from gp_nystrom_precond; noise = its sigma^2.  Asynchronous.
 * Workspace: gp_workspace_bytes(GP_OP_NYSTROM_APPLY, n, 0, 1, s, r, any precision).
 */
int gp_nystrom_apply(const double* Z, const double* g, int64_t n, int32_t r, double noise,
                     const double* V, int32_t s, double* Y,
                     void* ws, size_t ws_bytes, void* stream);

/*
 * gp_bcg - AltBBMM solve (Sec. 3.1 block CG, Sec. 3.2): block conjugate
 * gradients on the symmetrically preconditioned system
 *   P^{-1/2} K_hat P^{-1/2} U = P^{-1/2} B,   W = P^{-1/2} U  (= K_hat^{-1} B),
 * with P the Nystrom preconditioner of gp_nystrom_precond (r > 0) or the
 * identity (r = 0; Z, g ignored).  Iteration (O'Leary): Q = A D,
 * alpha = (D^T Q)^{-1} R^T R, U += D alpha, R -= Q alpha,
 * beta = (R_old^T R_old)^{-1} R^T R, D = R + D beta.  Stops when every column's
 * relative residual ||R_c|| / ||P^{-1/2} B_c|| <= tol (the paper: 1e-6 for all
 * s = 50 columns); GP_WNOCONV after max_iter.  K_hat products in `precision`
 * (as gp_kmm); recurrences, preconditioner and the s x s solves in FP64.
 * B: device n x s (ldb >= n), nonzero columns, s <= 64.  W: device n x s
 * (ldw >= n).  iters: host, the iterations run.  relres: host, s final
 * relative residuals.  The s x s systems are solved by pivoted LU on the host;
 * GP_ENOTPD on block breakdown (a singular D^T A D or R^T R).  Synchronises
 * twice per iteration.
 * Workspace: gp_workspace_bytes(GP_OP_BCG, n, 0, d, s, r, precision).
 */
int gp_bcg(const gp_kernel* kern, int32_t precision, const double* X, int64_t n,
           const double* Z, const double* g, int32_t r,
           const double* B, int64_t ldb, int32_t s, int32_t max_iter, double tol,
           double* W, int64_t ldw, int32_t* iters, double* relres,
           void* ws, size_t ws_bytes, void* stream);

/*
 * gp_nystrom_chol_precond - the AltBBMM Nystrom preconditioner (Sec. 3.2) at
 * large rank (the paper uses r = 10^4, Sec. 4), built from Cholesky factors
 * alone (no eigendecomposition):
 *   K_MM + delta I = L_M L_M^T,   delta = 1e-10 r s_f,
 *   F = K_XM L_M^{-T}  (n x r),   F^T F + sigma^2 I = L_G L_G^T,
 *   E = F L_G^{-T}     (n x r),
 * so that P = F F^T + sigma^2 I (the Nystrom approximation over the landmark
 * rows M, with K_MM's inverse regularised by delta) and
 *   P^{-1} = sigma^{-2} (I - E E^T),
 * positive definite for any rounding of the factors (E E^T has eigenvalues
 * below 1).  landmarks: host, r distinct indices in [0, n).  E: device n x r,
 * column-major (ld n), FP64, owned by the caller.  Requires sigma^2 > 0 and
 * 1 <= r <= min(n, 16384).  Errors: GP_EINVAL, GP_ENOTPD (a factorisation met
 * a non-positive pivot), GP_EWORKSPACE, GP_EHIP.  Synchronous.  The O(n r^2)
 * steps (F, F^T F, E) are FP64 matrix-core products.
 * Workspace: gp_workspace_bytes(GP_OP_NYSTROM_CHOL, n, 0, d, 0, r, any precision)
 * (an n x r FP64 buffer and two r x r ones).
 */
int gp_nystrom_chol_precond(const gp_kernel* kern, const double* X, int64_t n,
                            const int64_t* landmarks, int32_t r, double* E,
                            void* ws, size_t ws_bytes, void* stream);

/*
 * gp_bpcg - AltBBMM solve (Sec. 3.1 block CG, Sec. 3.2) with the preconditioner
 * of gp_nystrom_chol_precond: block preconditioned CG (O'Leary) on
 * K_hat W = B with P^{-1} = sigma^{-2} (I - E E^T) (r = 0: P = I, E ignored),
 *   Q = K_hat D;  alpha = (D^T Q)^{-1} (R^T Z);  W += D alpha;  R -= Q alpha;
 *   Z = P^{-1} R;  beta = (R_old^T Z_old)^{-1} (R^T Z);  D = Z + D beta,
 * whose iterates are those of block CG on P^{-1/2} K_hat P^{-1/2} (gp_bcg's
 * system).  Stops when every column's sqrt(r_c^T P^{-1} r_c) / sqrt(b_c^T P^{-1} b_c)
 * (that system's relative residual) is <= tol; GP_WNOCONV after max_iter.
 * K_hat products in `precision` (as gp_kmm); everything else FP64.  B: device
 * n x s (ldb >= n), nonzero columns, s <= 64; W: device n x s (ldw >= n);
 * iters: host; relres: host, s entries.  The s x s systems are solved by pivoted
 * LU on the host; GP_ENOTPD on block breakdown.  Synchronises twice per
 * iteration.  Workspace: gp_workspace_bytes(GP_OP_BPCG, n, 0, d, s, r, precision).
 */
int gp_bpcg(const gp_kernel* kern, int32_t precision, const double* X, int64_t n,
            const double* E, int32_t r,
            const double* B, int64_t ldb, int32_t s, int32_t max_iter, double tol,
            double* W, int64_t ldw, int32_t* iters, double* relres,
            void* ws, size_t ws_bytes, void* stream);

/*
 * gp_exact_mll_and_grad - the exact GP of the AltBBMM hyperparameter
 * protocol (Sec. 3.2, Sec. 4: hyperparameters from a full GP on a random
 * subset of the training molecules), dense FP64 on the device:
 *   K_hat = L L^T (Cholesky), omega = K_hat^{-1} y,
 *   mll = -1/2 y^T omega - 1/2 log|K_hat| - n/2 log 2 pi           (Eq. 2),
 *   grad_j = 1/2 omega^T dK_hat_j omega - 1/2 tr(K_hat^{-1} dK_hat_j)
 * over (log l_1 .. log l_d, log s_f, log sigma^2), the order of gp_kmm_grad.
 * X: device n x d row-major FP64; y: device n.  mll: host.  grad: host d + 2,
 * or NULL to skip the derivative sweep.  omega: device n, or NULL.
 * Requires 1 <= n <= 65536, d <= 64.  Errors: GP_EINVAL, GP_ENOTPD (K_hat not
 * numerically positive definite, e.g. repeated rows with sigma^2 = 0),
 * GP_ENONFINITE, GP_EWORKSPACE, GP_EHIP.  Synchronous.  O(n^3) flops; the
 * workspace holds two n x n FP64 matrices (K_hat's factor and its inverse).
 * Workspace: gp_workspace_bytes(GP_OP_EXACT, n, 0, d, 0, 0, any precision).
 */
int gp_exact_mll_and_grad(const gp_kernel* kern, const double* X, const double* y, int64_t n,
                          double* mll, double* grad, double* omega,
                          void* ws, size_t ws_bytes, void* stream);

/*
 * gp_workspace_bytes - device scratch needed by one call of `op`
 * (GP_OP_*), for n training rows, m query rows (GP_OP_KMM: m = 0 for the
 * square product), d features, t columns (GP_OP_MBCG: the block width s;
 * GP_OP_MLL: opts.probes), k the preconditioner rank (or kc for
 * GP_OP_LANCZOS / GP_OP_PREDICT / GP_OP_PREDICT_RUN).  Returns 0 for invalid
 * arguments.
 */
size_t gp_workspace_bytes(int32_t op, int64_t n, int64_t m, int32_t d, int32_t t,
                          int32_t k, int32_t precision);

/*
 * Kernel timing for profiling.  While enabled (process-wide), every launch of
 * the K_hat V / K(Z, X) V tile sweep records a pair of HIP events on its own
 * stream.  gp_profile_read waits for the recorded events and returns the
 * number of sweep launches, their summed duration (ms) and their summed
 * nominal flops 2 m n (d + t); reset != 0 clears the record.
 */
int gp_profile_enable(int32_t on);
int gp_profile_read(int64_t* launches, double* total_ms, double* nominal_flops, int32_t reset);
/* Per-launch view of the same record (up to cap launches, oldest first): the
 * product's n (training rows), m (output rows), t (columns) and duration (ms);
 * count receives the number written.  Call before a resetting gp_profile_read. */
int gp_profile_records(int64_t cap, int64_t* n, int64_t* m, int32_t* t, double* ms, int64_t* count);

/* Message of the last non-zero status returned to the calling thread. */
const char* gp_last_error(void);

/* Library version string. */
const char* gp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GPKMM_H */

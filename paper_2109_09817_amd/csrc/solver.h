// Internal interface of the FP64 solver kernels (blas.hip) used by the host
// orchestration (solver.cpp, predict.cpp, grad.hip).
#pragma once

#include "internal.h"

namespace gpk {

constexpr int64_t kDotBlocks = 1024;  // target blocks of the column reductions
constexpr int64_t kAtbBlocks = 256;   // target blocks of the tall-skinny A^T B products
constexpr uint64_t kEps1StreamOffset = 65536;

constexpr unsigned kStatusNotPD = 1u;
constexpr unsigned kStatusNonFinite = 2u;

inline uint64_t splitmix64_host(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct RowSplit {
  int64_t rows_per_blk;
  int64_t nblk;
};
RowSplit row_split(int64_t n, int64_t target_blocks);

// Device-resident per-column state of an mBCG run (arrays of s entries).
struct MbcgState {
  int s;
  double* gamma;      // r.z of the current residual
  double* gamma_new;  // r.z after the preconditioner step
  double* gamma0;     // b^T P^{-1} b
  double* delta;      // d.w
  double* alpha;      // current step sizes (copied to the host every iteration)
  double* beta;
  double* rnorm2;
  double* bnorm;      // ||b|| (holds ||b||^2 until init)
  double* relres;
  int* active;
  int* iters;
  int* num_active;
  unsigned* status;
};

struct Precond {
  int rank = 0;
  const double* L = nullptr;      // n x rank, ld n
  const double* Cchol = nullptr;  // rank x rank lower, column-major
  double noise = 0.0;
};

struct PivState {
  int64_t* piv;     // k pivots
  double* pivval;   // residual diagonal at each pivot
  int* rank;        // steps completed
};

hipError_t coldot(const double* A, const double* B, int64_t n, int s, double* out, double* partial, hipStream_t st);
size_t atb_partial_doubles(int64_t n, int pa, int qb);
hipError_t atb(const double* A, int pa, const double* B, int qb, int64_t n, double* out, double* partial,
               hipStream_t st);
// atb with the row split into (at most) nblk blocks; partial holds nblk * pa * qb doubles.
hipError_t atb_n(const double* A, int pa, const double* B, int qb, int64_t n, double* out, double* partial,
                 int64_t nblk, hipStream_t st);
// Z = P^{-1} R for an n x s block.  Y: rank x s scratch; partial: atb scratch.
hipError_t precond_apply(const Precond& pc, const double* R, double* Z, int64_t n, int s, double* Y,
                         double* partial, hipStream_t st);
hipError_t launch_probes(const double* y, int64_t n, int t, const double* L, int k, double noise, uint64_t seed,
                         double* B, hipStream_t st);
hipError_t launch_copy(const double* src, double* dst, int64_t count, hipStream_t st);
hipError_t launch_zero_words(void* dst, int64_t words, hipStream_t st);  // 32-bit words
hipError_t launch_gemv_sub(const double* Q, int64_t n, int jn, const double* h, double* w, hipStream_t st);
hipError_t launch_scale_rsqrt(const double* src, const double* s2, int64_t n, double* dst, hipStream_t st);
hipError_t launch_bidiag_solve(double* QR, int64_t n, int K, const double* lm, hipStream_t st);
hipError_t launch_predict_finish(const double* P, int64_t m, int kc, double sf, double* mean, double* var,
                                 hipStream_t st);
hipError_t launch_fill(double* dst, double v, int64_t count, hipStream_t st);

hipError_t mbcg_launch_init(const MbcgState& s, hipStream_t st);
hipError_t mbcg_launch_alpha(const MbcgState& s, hipStream_t st);
hipError_t mbcg_launch_update_ur(const MbcgState& s, const double* D, const double* W, double* U, double* R,
                                 int64_t n, double* partial, hipStream_t st);
hipError_t mbcg_launch_freeze(const MbcgState& s, int j, double tol, hipStream_t st);
hipError_t mbcg_launch_beta(const MbcgState& s, hipStream_t st);
hipError_t mbcg_launch_update_d(const MbcgState& s, const double* Z, double* D, int64_t n, hipStream_t st);

hipError_t pivchol_launch_argmax(const double* delta, int64_t n, double* pval, int64_t* pidx, const PivState& ps,
                                 int m, double stop_below, hipStream_t st);
hipError_t pivchol_launch_column(const double* X, int64_t n, const gp_kernel* kern, double* L, double* delta,
                                 const PivState& ps, int m, hipStream_t st);

// Dense FP64 pieces on the matrix cores (exact.hip).  Row-major matrices.
// C (m x nn, ldc) = A B with A(i, k) = ta ? A[k lda + i] : A[i lda + k] and
// B(k, j) = tb ? B[j ldb + k] : B[k ldb + j]; lower: only the tiles on and
// below the diagonal (m = nn).
hipError_t dense_gemm(bool ta, bool tb, bool lower, int64_t m, int64_t nn, int64_t kk, const double* A, int64_t lda,
                      const double* B, int64_t ldb, double* C, int64_t ldc, hipStream_t st);
// Doubles of the diagonal-block scratch of the two routines below.
size_t dense_dinv_doubles(int64_t n);
// In-place lower Cholesky factor of the symmetric n x n A (lower triangle read);
// *info (device, zeroed by the caller) receives 1 + the first non-positive pivot.
hipError_t dense_cholesky(double* A, int64_t n, int* info, double* Dinv, hipStream_t st);
// B = L^{-1} for a lower Cholesky factor L (zero above the diagonal).
hipError_t dense_lower_inverse(const double* L, double* B, double* Dinv, int64_t n, hipStream_t st);

// Host: e_1^T log(T) e_1 for the Lanczos tridiagonal of CG coefficients
// (alpha[j*stride], beta[j*stride], j < J).  Returns false if T is not
// positive definite or the eigen-iteration fails.
bool lanczos_log_quadrature(const double* alpha, const double* beta, int J, int stride, double* out);
// Host: eigenvalues (ascending not guaranteed) and first eigenvector components of a
// symmetric tridiagonal matrix (diag a[0..n-1], off-diagonal b[0..n-2]).
bool tridiag_eig_first(int n, double* a, double* b, double* z);
// Host: in-place lower Cholesky factor of the symmetric k x k matrix A (row-major);
// false if A is not positive definite.
bool host_cholesky(std::vector<double>& A, int k);
// Host: all eigenpairs of the dense symmetric n x n matrix A (row-major, destroyed):
// A = Q diag(w) Q^T, Q row-major with the eigenvectors as columns.  False if the
// iteration does not converge.
bool sym_eig(int n, std::vector<double>& A, std::vector<double>& w, std::vector<double>& Q);

}  // namespace gpk

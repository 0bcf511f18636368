// C ABI: pivoted-Cholesky preconditioner, probe block, mBCG and the BBMM
// marginal-likelihood evaluation (host orchestration of the HIP kernels).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "api_common.h"
#include "solver.h"

namespace gpk {

constexpr double kPivStopRel = 1e-12;   // pivoted Cholesky stops at residual <= 1e-12 s_f
constexpr double kFreezeFloor = 1e-12;  // mBCG columns also freeze at ||r|| <= 1e-12 ||b||
constexpr int kMaxBlock = 256;          // largest mBCG block width
constexpr int kMaxRank = 1024;

static double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- workspace

static size_t dot_partial_doubles(int64_t n, int s) { return (size_t)row_split(n, kDotBlocks).nblk * s; }

size_t pivchol_ws_bytes(int64_t n, int k) {
  const size_t nb = (size_t)row_split(n, kDotBlocks).nblk;
  size_t b = 0;
  b += align256(n * 8);                                   // delta
  b += align256(nb * 8) + align256(nb * 8);               // argmax partials
  b += align256((size_t)k * 8) * 2 + align256(8);         // piv, pivval, rank
  b += align256((size_t)k * k * 8);                       // C
  b += align256(atb_partial_doubles(n, k, k) * 8);        // atb partial
  return b;
}

size_t mbcg_ws_bytes(int precision, int d, int64_t n, int s, int rank) {
  size_t b = kmm_plan_bytes(precision, d, n, n, true, s);
  b += 4 * align256((size_t)n * s * 8);  // R, Z, D, W
  b += 16 * align256((size_t)s * 8);     // per-column state
  b += align256((size_t)(2 * s + 2) * 8);
  const size_t part = std::max(dot_partial_doubles(n, s), rank > 0 ? atb_partial_doubles(n, rank, s) : 0);
  b += align256(part * 8);
  b += align256((size_t)std::max(rank, 1) * s * 8);  // Woodbury Y
  return b + 4096;
}

// ------------------------------------------------------------- pivoted Cholesky

bool host_cholesky(std::vector<double>& A, int k) {
  // in place, lower, row-major k x k (A symmetric)
  for (int j = 0; j < k; ++j) {
    double v = A[(size_t)j * k + j];
    for (int i = 0; i < j; ++i) v -= A[(size_t)j * k + i] * A[(size_t)j * k + i];
    if (!(v > 0.0) || !std::isfinite(v)) return false;
    const double ljj = std::sqrt(v);
    A[(size_t)j * k + j] = ljj;
    for (int r = j + 1; r < k; ++r) {
      double w = A[(size_t)r * k + j];
      for (int i = 0; i < j; ++i) w -= A[(size_t)r * k + i] * A[(size_t)j * k + i];
      A[(size_t)r * k + j] = w / ljj;
    }
    for (int i = j + 1; i < k; ++i) A[(size_t)j * k + i] = 0.0;
  }
  return true;
}

int run_pivchol(const gp_kernel* kern, const double* X, int64_t n, int k, double* L, double* Cchol,
                int64_t* piv_host, int* rank_host, double* logdet_host, void* ws, size_t ws_bytes, hipStream_t st) {
  Carve cv(ws, ws_bytes);
  const int64_t nb = row_split(n, kDotBlocks).nblk;
  double* delta = cv.take<double>(n);
  double* pval = cv.take<double>(nb);
  int64_t* pidx = cv.take<int64_t>(nb);
  int64_t* piv = cv.take<int64_t>(k);
  double* pivval = cv.take<double>(k);
  int* rank = cv.take<int>(2);
  double* C = cv.take<double>((size_t)k * k);
  double* part = cv.take<double>(atb_partial_doubles(n, k, k));
  if (!part) return fail(GP_EWORKSPACE, "gp_pivchol_precond: workspace layout failed");
  PivState ps{piv, pivval, rank};
  GPK_HIP(launch_fill(L, 0.0, n * (int64_t)k, st));
  GPK_HIP(launch_fill(delta, kern->outputscale, n, st));
  GPK_HIP(launch_zero_words(rank, 1, st));
  GPK_HIP(launch_zero_words(piv, 2 * (int64_t)k, st));
  for (int m = 0; m < k; ++m) {
    GPK_HIP(pivchol_launch_argmax(delta, n, pval, pidx, ps, m, kPivStopRel * kern->outputscale, st));
    GPK_HIP(pivchol_launch_column(X, n, kern, L, delta, ps, m, st));
  }
  GPK_HIP(atb(L, k, L, k, n, C, part, st));
  std::vector<double> Ch((size_t)k * k);
  int r = 0;
  std::vector<int64_t> pv(k);
  GPK_HIP(hipMemcpyAsync(Ch.data(), C, Ch.size() * 8, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipMemcpyAsync(&r, rank, sizeof(int), hipMemcpyDeviceToHost, st));
  GPK_HIP(hipMemcpyAsync(pv.data(), piv, sizeof(int64_t) * k, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipStreamSynchronize(st));
  const double s2 = kern->noise;
  for (int j = 0; j < k; ++j) {
    Ch[(size_t)j * k + j] += s2;
    for (int i = 0; i < k; ++i)
      if (!std::isfinite(Ch[(size_t)j * k + i])) return fail(GP_ENONFINITE, "gp_pivchol_precond: non-finite L^T L");
  }
  if (!host_cholesky(Ch, k)) return fail(GP_ENOTPD, "gp_pivchol_precond: sigma^2 I + L^T L is not positive definite");
  double ld = (double)(n - k) * std::log(s2);
  for (int j = 0; j < k; ++j) ld += 2.0 * std::log(Ch[(size_t)j * k + j]);
  // column-major copy of the lower factor: entry (row i, col j) at [j*k + i]
  std::vector<double> Lc((size_t)k * k);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) Lc[(size_t)j * k + i] = Ch[(size_t)i * k + j];
  GPK_HIP(hipMemcpyAsync(Cchol, Lc.data(), Lc.size() * 8, hipMemcpyHostToDevice, st));
  GPK_HIP(hipStreamSynchronize(st));
  if (piv_host)
    for (int j = 0; j < k; ++j) piv_host[j] = j < r ? pv[j] : -1;
  if (rank_host) *rank_host = r;
  if (logdet_host) *logdet_host = ld;
  return GP_OK;
}

// ----------------------------------------------------------------------- mBCG

struct MbcgHost {
  std::vector<double> alpha, beta;  // total_iters x s
  std::vector<int> iters;
  std::vector<double> relres, gamma0;
  int total_iters = 0;
};

int run_mbcg(const gp_kernel* kern, int precision, const double* X, int64_t n, const Precond& pc, const double* B,
             int s, int max_iter, double tol, double* U, double* Z0, MbcgHost& out, void* ws, size_t ws_bytes,
             hipStream_t st) {
  const size_t kb = kmm_plan_bytes(precision, kern->d, n, n, true, s);
  KmmPlan plan;
  if (!kmm_plan_init(plan, kern, precision, n, n, true, s, ws, kb))
    return fail(GP_EWORKSPACE, "gp_mbcg: workspace too small for the product plan");
  Carve cv((char*)ws + align256(kb), ws_bytes - align256(kb));
  const size_t ns = (size_t)n * s;
  double* R = cv.take<double>(ns);
  double* Z = cv.take<double>(ns);
  double* D = cv.take<double>(ns);
  double* W = cv.take<double>(ns);
  MbcgState S;
  S.s = s;
  S.gamma = cv.take<double>(s);
  S.gamma_new = cv.take<double>(s);
  S.gamma0 = cv.take<double>(s);
  S.delta = cv.take<double>(s);
  S.rnorm2 = cv.take<double>(s);
  S.bnorm = cv.take<double>(s);
  S.relres = cv.take<double>(s);
  S.active = cv.take<int>(s);
  S.iters = cv.take<int>(s);
  double* xfer = cv.take<double>(2 * s + 2);  // [alpha | beta | num_active, status]
  const size_t part_n = std::max(dot_partial_doubles(n, s), pc.rank > 0 ? atb_partial_doubles(n, pc.rank, s) : 0);
  double* part = cv.take<double>(part_n);
  double* Y = cv.take<double>((size_t)std::max(pc.rank, 1) * s);
  if (!Y || !xfer) return fail(GP_EWORKSPACE, "gp_mbcg: workspace layout failed");
  S.alpha = xfer;
  S.beta = xfer + s;
  S.num_active = (int*)(xfer + 2 * s);
  S.status = (unsigned*)(S.num_active + 1);
  // the step sizes of every iteration are copied to the host; the device keeps no history

  GPK_HIP(kmm_prepare(plan, kern, X, nullptr, st));
  GPK_HIP(launch_copy(B, R, (int64_t)ns, st));
  GPK_HIP(launch_fill(U, 0.0, (int64_t)ns, st));
  GPK_HIP(launch_zero_words(S.status, 1, st));
  GPK_HIP(precond_apply(pc, R, Z, n, s, Y, part, st));
  if (Z0) GPK_HIP(launch_copy(Z, Z0, (int64_t)ns, st));
  GPK_HIP(launch_copy(Z, D, (int64_t)ns, st));
  GPK_HIP(coldot(R, Z, n, s, S.gamma, part, st));
  GPK_HIP(coldot(B, B, n, s, S.bnorm, part, st));
  GPK_HIP(mbcg_launch_init(S, st));
  struct {
    int num_active;
    unsigned status;
  } flags{0, 0};
  std::vector<double> ab(2 * s);
  GPK_HIP(hipMemcpyAsync(&flags, S.num_active, sizeof flags, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipStreamSynchronize(st));
  if (flags.status & kStatusNonFinite) return fail(GP_ENONFINITE, "gp_mbcg: non-finite right-hand side or P^{-1}B");
  const double ftol = std::max(tol, kFreezeFloor);
  out.alpha.clear();
  out.beta.clear();
  out.total_iters = 0;
  for (int j = 0; j < max_iter && flags.num_active > 0; ++j) {
    GPK_HIP(kmm_apply(plan, D, n, s, W, n, st));
    GPK_HIP(coldot(D, W, n, s, S.delta, part, st));
    GPK_HIP(mbcg_launch_alpha(S, st));
    GPK_HIP(mbcg_launch_update_ur(S, D, W, U, R, n, part, st));
    GPK_HIP(mbcg_launch_freeze(S, j, ftol, st));
    GPK_HIP(precond_apply(pc, R, Z, n, s, Y, part, st));
    GPK_HIP(coldot(R, Z, n, s, S.gamma_new, part, st));
    GPK_HIP(mbcg_launch_beta(S, st));
    GPK_HIP(mbcg_launch_update_d(S, Z, D, n, st));
    GPK_HIP(hipMemcpyAsync(ab.data(), xfer, sizeof(double) * 2 * s, hipMemcpyDeviceToHost, st));
    GPK_HIP(hipMemcpyAsync(&flags, S.num_active, sizeof flags, hipMemcpyDeviceToHost, st));
    GPK_HIP(hipStreamSynchronize(st));
    out.alpha.insert(out.alpha.end(), ab.begin(), ab.begin() + s);
    out.beta.insert(out.beta.end(), ab.begin() + s, ab.end());
    out.total_iters = j + 1;
    if (flags.status & kStatusNonFinite) return fail(GP_ENONFINITE, "gp_mbcg: non-finite value at iteration %d", j);
    if (flags.status & kStatusNotPD) return fail(GP_ENOTPD, "gp_mbcg: d^T K_hat d <= 0 at iteration %d", j);
  }
  out.iters.assign(s, 0);
  out.relres.assign(s, 0.0);
  out.gamma0.assign(s, 0.0);
  GPK_HIP(hipMemcpyAsync(out.iters.data(), S.iters, sizeof(int) * s, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipMemcpyAsync(out.relres.data(), S.relres, sizeof(double) * s, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipMemcpyAsync(out.gamma0.data(), S.gamma0, sizeof(double) * s, hipMemcpyDeviceToHost, st));
  GPK_HIP(hipStreamSynchronize(st));
  return (flags.num_active > 0 && tol > 0.0) ? GP_WNOCONV : GP_OK;
}

static int check_common(const gp_kernel* kern, int precision, const double* X, int64_t n, const char* op,
                        bool fp64_ok = false) {
  GPK_TRY(check_kernel(kern));
  GPK_TRY(fp64_ok ? check_product_precision(precision) : check_precision(precision));
  if (!X) return fail(GP_EINVAL, "%s: X is NULL", op);
  if (n < 1) return fail(GP_EINVAL, "%s: n=%lld must be >= 1", op, (long long)n);
  return GP_OK;
}

}  // namespace gpk

using namespace gpk;

extern "C" int gp_pivchol_precond(const gp_kernel* kern, const double* X, int64_t n, int32_t k, double* L,
                                  double* Cchol, int64_t* piv, int32_t* rank, double* logdetP, void* ws,
                                  size_t ws_bytes, void* stream) {
  GPK_TRY(check_common(kern, GP_PREC_FP32, X, n, "gp_pivchol_precond"));
  if (k < 1 || k > kMaxRank || k > n) return fail(GP_EINVAL, "gp_pivchol_precond: k=%d outside [1, min(n, %d)]", k, kMaxRank);
  if (!(kern->noise > 0.0)) return fail(GP_EINVAL, "gp_pivchol_precond: needs noise > 0");
  if (!L || !Cchol || !rank || !logdetP) return fail(GP_EINVAL, "gp_pivchol_precond: NULL output");
  GPK_TRY(check_ws(ws, ws_bytes, pivchol_ws_bytes(n, k), "gp_pivchol_precond"));
  int r = 0;
  GPK_TRY(run_pivchol(kern, X, n, k, L, Cchol, piv, &r, logdetP, ws, ws_bytes, (hipStream_t)stream));
  *rank = r;
  return GP_OK;
}

extern "C" int gp_probe_block(const double* y, int64_t n, int32_t t, const double* L, int32_t k, double noise,
                              uint64_t seed, double* B, void* stream) {
  if (!y || !B) return fail(GP_EINVAL, "gp_probe_block: y or B is NULL");
  if (n < 1 || t < 0 || t + 1 > kMaxBlock) return fail(GP_EINVAL, "gp_probe_block: bad n=%lld or t=%d", (long long)n, t);
  if (k < 0 || k > kMaxRank || (k > 0 && !L)) return fail(GP_EINVAL, "gp_probe_block: bad k=%d or L", k);
  if (!std::isfinite(noise) || noise < 0.0) return fail(GP_EINVAL, "gp_probe_block: bad noise");
  GPK_HIP(launch_probes(y, n, t, L, k, noise, seed, B, (hipStream_t)stream));
  return GP_OK;
}

extern "C" int gp_mbcg(const gp_kernel* kern, int32_t precision, const double* X, int64_t n, const gp_precond* pc,
                       const double* B, int32_t s, int32_t max_iter, double tol, double* U, double* Z0,
                       gp_mbcg_out* out, void* ws, size_t ws_bytes, void* stream) {
  GPK_TRY(check_common(kern, precision, X, n, "gp_mbcg", /*fp64_ok=*/true));
  if (!B || !U) return fail(GP_EINVAL, "gp_mbcg: B or U is NULL");
  if (s < 1 || s > kMaxBlock) return fail(GP_EINVAL, "gp_mbcg: s=%d outside [1, %d]", s, kMaxBlock);
  if (max_iter < 1) return fail(GP_EINVAL, "gp_mbcg: max_iter=%d must be >= 1", max_iter);
  if (!std::isfinite(tol) || tol < 0.0) return fail(GP_EINVAL, "gp_mbcg: tol must be finite and >= 0");
  Precond P;
  P.noise = kern->noise;
  if (pc && pc->rank > 0) {
    if (pc->rank > kMaxRank || pc->rank > n || !pc->L || !pc->Cchol)
      return fail(GP_EINVAL, "gp_mbcg: bad preconditioner (rank %d)", pc->rank);
    if (!(kern->noise > 0.0)) return fail(GP_EINVAL, "gp_mbcg: a preconditioner needs noise > 0");
    P.rank = pc->rank;
    P.L = pc->L;
    P.Cchol = pc->Cchol;
  }
  GPK_TRY(check_ws(ws, ws_bytes, mbcg_ws_bytes(precision, kern->d, n, s, P.rank), "gp_mbcg"));
  MbcgHost h;
  const int rc = run_mbcg(kern, precision, X, n, P, B, s, max_iter, tol, U, Z0, h, ws, ws_bytes,
                          (hipStream_t)stream);
  if (rc < 0) return rc;
  if (out) {
    out->total_iters = h.total_iters;
    for (int j = 0; j < h.total_iters; ++j)
      for (int c = 0; c < s; ++c) {
        if (out->alpha) out->alpha[(size_t)j * s + c] = h.alpha[(size_t)j * s + c];
        if (out->beta) out->beta[(size_t)j * s + c] = h.beta[(size_t)j * s + c];
      }
    for (int c = 0; c < s; ++c) {
      if (out->iters) out->iters[c] = h.iters[c];
      if (out->relres) out->relres[c] = h.relres[c];
      if (out->gamma0) out->gamma0[c] = h.gamma0[c];
    }
  }
  if (rc == GP_WNOCONV) fail(GP_WNOCONV, "gp_mbcg: %d iterations without reaching tol=%g", max_iter, tol);
  return rc;
}

// ------------------------------------------------------------ mll and gradient

namespace gpk {
size_t grad_ws_bytes(int precision, int d, int64_t n, int t);
int run_kmm_grad(const gp_kernel* kern, int precision, const double* X, int64_t n, const double* U, int64_t ldu,
                 const double* W, int64_t ldw, int t, const double* colw, double* grad, void* ws, size_t ws_bytes,
                 hipStream_t st);

size_t mll_ws_bytes(int precision, int d, int64_t n, int t, int k) {
  const int s = t + 1;
  size_t b = 0;
  b += align256((size_t)n * std::max(k, 1) * 8);     // L
  b += align256((size_t)std::max(k, 1) * std::max(k, 1) * 8);  // Cchol
  b += 3 * align256((size_t)n * s * 8);              // B, U, Z0
  b += align256(16 * 8);                             // quad
  size_t inner = mbcg_ws_bytes(precision, d, n, s, k);
  if (k > 0) inner = std::max(inner, pivchol_ws_bytes(n, k));
  inner = std::max(inner, grad_ws_bytes(precision, d, n, s));
  inner = std::max(inner, (size_t)row_split(n, kDotBlocks).nblk * 8 + 256);
  return b + inner + 4096;
}
}  // namespace gpk

extern "C" int gp_mll_and_grad(const gp_kernel* kern, const gp_mll_opts* opts, const double* X, const double* y,
                               int64_t n, double* mll, double* grad, gp_mll_info* info, void* ws, size_t ws_bytes,
                               void* stream) {
  if (!opts) return fail(GP_EINVAL, "gp_mll_and_grad: opts is NULL");
  GPK_TRY(check_common(kern, opts->precision, X, n, "gp_mll_and_grad"));
  if (!y || !mll) return fail(GP_EINVAL, "gp_mll_and_grad: y or mll is NULL");
  const int t = opts->probes, k = opts->rank;
  if (t < 1 || t + 1 > kMaxBlock) return fail(GP_EINVAL, "gp_mll_and_grad: probes=%d outside [1, %d]", t, kMaxBlock - 1);
  if (k < 0 || k > kMaxRank || k > n) return fail(GP_EINVAL, "gp_mll_and_grad: rank=%d outside [0, min(n, %d)]", k, kMaxRank);
  if (opts->max_iter < 1) return fail(GP_EINVAL, "gp_mll_and_grad: max_iter must be >= 1");
  if (!std::isfinite(opts->tol) || opts->tol < 0.0) return fail(GP_EINVAL, "gp_mll_and_grad: bad tol");
  if (!(kern->noise > 0.0)) return fail(GP_EINVAL, "gp_mll_and_grad: needs noise > 0");
  GPK_TRY(check_ws(ws, ws_bytes, mll_ws_bytes(opts->precision, kern->d, n, t, k), "gp_mll_and_grad"));
  hipStream_t st = (hipStream_t)stream;
  const int s = t + 1;
  Carve cv(ws, ws_bytes);
  double* L = cv.take<double>((size_t)n * std::max(k, 1));
  double* Cc = cv.take<double>((size_t)std::max(k, 1) * std::max(k, 1));
  double* B = cv.take<double>((size_t)n * s);
  double* U = cv.take<double>((size_t)n * s);
  double* Z0 = cv.take<double>((size_t)n * s);
  double* q = cv.take<double>(16);
  void* inner = cv.p;
  const size_t inner_bytes = cv.left;
  if (!q) return fail(GP_EWORKSPACE, "gp_mll_and_grad: workspace layout failed");

  const double t0 = now_ms();
  Precond P;
  P.noise = kern->noise;
  double logdet_p = 0.0;
  int rank = 0;
  if (k > 0) {
    GPK_TRY(run_pivchol(kern, X, n, k, L, Cc, nullptr, &rank, &logdet_p, inner, inner_bytes, st));
    P.rank = k;  // columns past the reached rank are zero and harmless
    P.L = L;
    P.Cchol = Cc;
  }
  GPK_HIP(launch_probes(y, n, t, L, k, kern->noise, opts->seed, B, st));
  const double t1 = now_ms();
  MbcgHost h;
  const int rc = run_mbcg(kern, opts->precision, X, n, P, B, s, opts->max_iter, opts->tol, U, Z0, h, inner,
                          inner_bytes, st);
  if (rc < 0) return rc;
  const double t2 = now_ms();
  // stochastic Lanczos quadrature over the probe columns
  double acc = 0.0;
  for (int c = 1; c < s; ++c) {
    double qc = 0.0;
    if (!lanczos_log_quadrature(h.alpha.data() + c, h.beta.data() + c, h.iters[c], s, &qc))
      return fail(GP_ENOTPD, "gp_mll_and_grad: Lanczos tridiagonal of probe %d not positive definite", c);
    acc += h.gamma0[c] * qc;
  }
  const double logdet = logdet_p + acc / t;
  // quad = y^T u_0
  double* part = (double*)inner;
  GPK_HIP(coldot(y, U, n, 1, q, part, st));
  double quad = 0.0;
  GPK_HIP(hipMemcpyAsync(&quad, q, sizeof(double), hipMemcpyDeviceToHost, st));
  GPK_HIP(hipStreamSynchronize(st));
  *mll = -0.5 * quad - 0.5 * logdet - 0.5 * (double)n * std::log(2.0 * M_PI);
  double t3 = now_ms();
  if (grad) {
    // W = [u_0 | z0_1 .. z0_t], weights [1/2, -1/(2t) ...]
    GPK_HIP(launch_copy(U, Z0, n, st));
    std::vector<double> w(s, -0.5 / t);
    w[0] = 0.5;
    GPK_TRY(run_kmm_grad(kern, opts->precision, X, n, U, n, Z0, n, s, w.data(), grad, inner, inner_bytes, st));
  }
  const double t4 = now_ms();
  if (info) {
    info->iters = h.total_iters;
    info->rank = rank;
    info->logdet = logdet;
    info->logdet_p = logdet_p;
    info->quad = quad;
    double mr = 0.0;
    for (double r : h.relres) mr = std::max(mr, r);
    info->max_relres = mr;
    info->ms_precond = t1 - t0;
    info->ms_mbcg = t2 - t1;
    info->ms_grad = grad ? t4 - t3 : 0.0;
  }
  if (rc == GP_WNOCONV) fail(GP_WNOCONV, "gp_mll_and_grad: mBCG hit max_iter=%d", opts->max_iter);
  return rc;
}

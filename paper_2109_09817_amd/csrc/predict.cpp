// C ABI: predictive mean and variance (Eq. 1) from a resident model, and the
// Lanczos variance cache; plus gp_workspace_bytes for every operation.
#include <algorithm>
#include <cmath>
#include <vector>

#include "api_common.h"
#include "solver.h"

namespace gpk {

size_t pivchol_ws_bytes(int64_t n, int k);
size_t mbcg_ws_bytes(int precision, int d, int64_t n, int s, int rank);
size_t mll_ws_bytes(int precision, int d, int64_t n, int t, int k);
size_t grad_ws_bytes(int precision, int d, int64_t n, int t);
size_t nystrom_ws_bytes(int d, int64_t n, int r);
size_t nystrom_apply_ws_bytes(int64_t n, int r, int s);
size_t bcg_ws_bytes(int precision, int d, int64_t n, int r, int s);
size_t exact_ws_bytes(int d, int64_t n);
size_t nystrom_chol_ws_bytes(int d, int64_t n, int r);
size_t bpcg_ws_bytes(int precision, int d, int64_t n, int r, int s);

constexpr int kMaxCache = 4095;  // kc + 1 <= 4096 product columns

size_t predict_run_bytes(int precision, int d, int64_t n, int64_t m, int kc) {
  const int t = kc + 1;
  return kmm_query_bytes(precision, d, n, m, t) + align256((size_t)m * t * 8) + 4096;
}

size_t lanczos_ws_bytes(int precision, int d, int64_t n, int kc) {
  size_t b = kmm_plan_bytes(precision, d, n, n, true, 1);
  b += align256((size_t)n * 8);                                      // w
  b += align256((size_t)std::max(kc, 1) * 8) + align256(64);         // h, scalars
  b += align256(std::max(atb_partial_doubles(n, std::max(kc, 1), 1),
                         (size_t)row_split(n, kDotBlocks).nblk) * 8);  // reductions
  b += align256((size_t)2 * std::max(kc, 1) * 8);                    // bidiagonal factor
  return b + 4096;
}

static int check_predict_common(const gp_kernel* kern, int precision, int64_t n, int kc) {
  GPK_TRY(check_kernel(kern));
  GPK_TRY(check_precision(precision));
  if (n < 1) return fail(GP_EINVAL, "predict: n must be >= 1");
  if (kc < 0 || kc > kMaxCache) return fail(GP_EINVAL, "predict: kc=%d outside [0, %d]", kc, kMaxCache);
  return GP_OK;
}

}  // namespace gpk

using namespace gpk;

extern "C" size_t gp_predict_model_bytes(const gp_kernel* kern, int32_t precision, int64_t n, int32_t kc) {
  if (!kern || kern->d < 1 || kern->d > GP_MAX_D || n < 1 || kc < 0 || kc > kMaxCache) return 0;
  if (precision != GP_PREC_FP32 && precision != GP_PREC_BF16X3) return 0;
  return kmm_model_bytes(precision, kern->d, n, kc + 1);
}

extern "C" int gp_predict_prepare(const gp_kernel* kern, int32_t precision, const double* X, int64_t n,
                                  const double* alpha, const double* R, int32_t kc, void* model, size_t model_bytes,
                                  void* stream) {
  GPK_TRY(check_predict_common(kern, precision, n, kc));
  if (!X || !alpha || (kc > 0 && !R)) return fail(GP_EINVAL, "gp_predict_prepare: NULL X, alpha or R");
  const size_t need = kmm_model_bytes(precision, kern->d, n, kc + 1);
  GPK_TRY(check_ws(model, model_bytes, need, "gp_predict_prepare (model)"));
  KmmPlan p;
  if (!kmm_plan_model(p, kern, precision, n, 0, kc + 1, model, model_bytes, nullptr, 0))
    return fail(GP_EWORKSPACE, "gp_predict_prepare: model layout failed");
  hipStream_t st = (hipStream_t)stream;
  GPK_HIP(kmm_prepare_rows(p, kern, X, st));
  GPK_HIP(kmm_prepare_v(p, kc > 0 ? R : alpha, n, kc + 1, /*row_independent=*/true, st, alpha));
  return GP_OK;
}

extern "C" int gp_predict_run(const gp_kernel* kern, int32_t precision, const void* model, int64_t n, int32_t kc,
                              const double* Z, int64_t m, double* mean, double* var, void* ws, size_t ws_bytes,
                              void* stream) {
  GPK_TRY(check_predict_common(kern, precision, n, kc));
  if (!model || !Z || !mean) return fail(GP_EINVAL, "gp_predict_run: NULL model, Z or mean");
  if (m < 1) return fail(GP_EINVAL, "gp_predict_run: m must be >= 1");
  if (var && kc < 1) return fail(GP_EINVAL, "gp_predict_run: variance needs a cache (kc >= 1)");
  const size_t need = predict_run_bytes(precision, kern->d, n, m, kc);
  GPK_TRY(check_ws(ws, ws_bytes, need, "gp_predict_run"));
  const int t = kc + 1;
  KmmPlan p;
  const size_t qb = kmm_query_bytes(precision, kern->d, n, m, t);
  if (!kmm_plan_model(p, kern, precision, n, m, t, (void*)model, kmm_model_bytes(precision, kern->d, n, t), ws, qb))
    return fail(GP_EWORKSPACE, "gp_predict_run: workspace layout failed");
  double* P = (double*)((char*)ws + align256(qb));
  hipStream_t st = (hipStream_t)stream;
  GPK_HIP(kmm_prepare_cols(p, kern, Z, st));
  GPK_HIP(kmm_sweep(p, t, nullptr, n, P, m, st, /*row_independent=*/true));
  GPK_HIP(launch_predict_finish(P, m, var ? kc : 0, kern->outputscale, mean, var, st));
  return GP_OK;
}

extern "C" int gp_predict(const gp_kernel* kern, int32_t precision, const double* X, int64_t n, const double* alpha,
                          const double* R, int32_t kc, const double* Z, int64_t m, double* mean, double* var, void* ws,
                          size_t ws_bytes, void* stream) {
  GPK_TRY(check_predict_common(kern, precision, n, kc));
  if (!R) kc = 0;
  // every argument is checked before the preparation's GPU work
  if (!X || !alpha || !Z || !mean) return fail(GP_EINVAL, "gp_predict: NULL X, alpha, Z or mean");
  if (m < 1) return fail(GP_EINVAL, "gp_predict: m must be >= 1");
  if (var && kc < 1) return fail(GP_EINVAL, "gp_predict: variance needs a cache (R and kc >= 1)");
  const size_t mb = kmm_model_bytes(precision, kern->d, n, kc + 1);
  const size_t rb = predict_run_bytes(precision, kern->d, n, m, kc);
  GPK_TRY(check_ws(ws, ws_bytes, align256(mb) + rb, "gp_predict"));
  GPK_TRY(gp_predict_prepare(kern, precision, X, n, alpha, R, kc, ws, mb, stream));
  return gp_predict_run(kern, precision, ws, n, kc, Z, m, mean, var, (char*)ws + align256(mb),
                        ws_bytes - align256(mb), stream);
}

extern "C" int gp_lanczos_cache(const gp_kernel* kern, int32_t precision, const double* X, const double* y, int64_t n,
                                int32_t kc, double* R, int32_t* kc_out, void* ws, size_t ws_bytes, void* stream) {
  GPK_TRY(check_kernel(kern));
  GPK_TRY(check_precision(precision));
  if (!X || !y || !R) return fail(GP_EINVAL, "gp_lanczos_cache: NULL X, y or R");
  if (n < 1) return fail(GP_EINVAL, "gp_lanczos_cache: n must be >= 1");
  if (kc < 1 || kc > kMaxCache || kc > n) return fail(GP_EINVAL, "gp_lanczos_cache: kc=%d outside [1, min(n, %d)]", kc, kMaxCache);
  GPK_TRY(check_ws(ws, ws_bytes, lanczos_ws_bytes(precision, kern->d, n, kc), "gp_lanczos_cache"));
  hipStream_t st = (hipStream_t)stream;
  const size_t kb = kmm_plan_bytes(precision, kern->d, n, n, true, 1);
  KmmPlan plan;
  if (!kmm_plan_init(plan, kern, precision, n, n, true, 1, ws, kb))
    return fail(GP_EWORKSPACE, "gp_lanczos_cache: workspace layout failed");
  Carve cv((char*)ws + align256(kb), ws_bytes - align256(kb));
  double* w = cv.take<double>(n);
  double* h = cv.take<double>(std::max(kc, 1));
  double* sc = cv.take<double>(8);
  double* part = cv.take<double>(std::max(atb_partial_doubles(n, std::max(kc, 1), 1),
                                          (size_t)row_split(n, kDotBlocks).nblk));
  double* lm = cv.take<double>(2 * (size_t)std::max(kc, 1));
  if (!lm) return fail(GP_EWORKSPACE, "gp_lanczos_cache: workspace layout failed");
  GPK_HIP(kmm_prepare(plan, kern, X, nullptr, st));
  // q_0 = y / ||y||
  GPK_HIP(coldot(y, y, n, 1, sc, part, st));
  GPK_HIP(launch_scale_rsqrt(y, sc, n, R, st));
  std::vector<double> a(kc), b(kc);
  int K = 0;
  for (int j = 0; j < kc; ++j) {
    double* q = R + (int64_t)j * n;
    GPK_HIP(kmm_apply(plan, q, n, 1, w, n, st));
    GPK_HIP(coldot(q, w, n, 1, sc + 1, part, st));
    for (int pass = 0; pass < 2; ++pass) {  // full re-orthogonalisation, twice
      GPK_HIP(atb(R, j + 1, w, 1, n, h, part, st));
      GPK_HIP(launch_gemv_sub(R, n, j + 1, h, w, st));
    }
    GPK_HIP(coldot(w, w, n, 1, sc + 2, part, st));
    double hv[3];
    GPK_HIP(hipMemcpyAsync(hv, sc, sizeof hv, hipMemcpyDeviceToHost, st));
    GPK_HIP(hipStreamSynchronize(st));
    if (!std::isfinite(hv[1]) || !std::isfinite(hv[2])) return fail(GP_ENONFINITE, "gp_lanczos_cache: non-finite at step %d", j);
    a[j] = hv[1];
    K = j + 1;
    const double bj = std::sqrt(hv[2]);
    if (j + 1 < kc) {
      if (bj <= 1e-12 * std::fabs(a[j])) break;  // Krylov space closed
      b[j] = bj;
      GPK_HIP(launch_scale_rsqrt(w, sc + 2, n, R + (int64_t)(j + 1) * n, st));
    }
  }
  // Cholesky of the K x K tridiagonal: diagonal l_j, subdiagonal m_j
  std::vector<double> lmh(2 * K);
  double prev_l = 0.0;
  for (int j = 0; j < K; ++j) {
    const double mj = j > 0 ? b[j - 1] / prev_l : 0.0;
    const double v = a[j] - mj * mj;
    if (!(v > 0.0)) return fail(GP_ENOTPD, "gp_lanczos_cache: Lanczos tridiagonal not positive definite at %d", j);
    const double lj = std::sqrt(v);
    lmh[2 * j] = lj;
    lmh[2 * j + 1] = mj;
    prev_l = lj;
  }
  GPK_HIP(hipMemcpyAsync(lm, lmh.data(), sizeof(double) * 2 * K, hipMemcpyHostToDevice, st));
  GPK_HIP(launch_bidiag_solve(R, n, K, lm, st));
  if (K < kc) GPK_HIP(launch_fill(R + (int64_t)K * n, 0.0, (int64_t)(kc - K) * n, st));
  GPK_HIP(hipStreamSynchronize(st));
  if (kc_out) *kc_out = K;
  return GP_OK;
}

extern "C" size_t gp_workspace_bytes(int32_t op, int64_t n, int64_t m, int32_t d, int32_t t, int32_t k,
                                     int32_t precision) {
  if (n < 1 || d < 1 || d > GP_MAX_D) return 0;
  if (precision != GP_PREC_FP32 && precision != GP_PREC_BF16X3 && precision != GP_PREC_FP64) return 0;
  if (precision == GP_PREC_FP64 && op != GP_OP_KMM && op != GP_OP_MBCG && op != GP_OP_BCG && op != GP_OP_EXACT &&
      op != GP_OP_BPCG && op != GP_OP_NYSTROM_CHOL)
    return 0;
  switch (op) {
    case GP_OP_KMM:
      if (t < 1) return 0;
      return kmm_plan_bytes(precision, d, n, m > 0 ? m : n, m <= 0, t);
    case GP_OP_KMM_GRAD:
      if (t < 1 || t > 64 || d > 64) return 0;
      return grad_ws_bytes(precision, d, n, t);
    case GP_OP_PIVCHOL:
      if (k < 1) return 0;
      return pivchol_ws_bytes(n, k);
    case GP_OP_MBCG:
      if (t < 1) return 0;
      return mbcg_ws_bytes(precision, d, n, t, std::max(k, 0));
    case GP_OP_MLL:
      if (t < 1) return 0;
      return mll_ws_bytes(precision, d, n, t, std::max(k, 0));
    case GP_OP_PREDICT:
      if (m < 1 || k < 0) return 0;
      return align256(kmm_model_bytes(precision, d, n, k + 1)) + predict_run_bytes(precision, d, n, m, k);
    case GP_OP_PREDICT_RUN:
      if (m < 1 || k < 0) return 0;
      return predict_run_bytes(precision, d, n, m, k);
    case GP_OP_LANCZOS:
      if (k < 1) return 0;
      return lanczos_ws_bytes(precision, d, n, k);
    case GP_OP_NYSTROM:
      if (k < 1 || k > 1024 || k > n) return 0;
      return nystrom_ws_bytes(d, n, k);
    case GP_OP_NYSTROM_APPLY:
      if (k < 1 || k > 1024 || k > n || t < 1 || t > 64) return 0;
      return nystrom_apply_ws_bytes(n, k, t);
    case GP_OP_BCG:
      if (k < 0 || k > 1024 || k > n || t < 1 || t > 64) return 0;
      return bcg_ws_bytes(precision, d, n, k, t);
    case GP_OP_EXACT:
      return exact_ws_bytes(d, n);
    case GP_OP_NYSTROM_CHOL:
      if (k < 1 || k > 16384 || k > n) return 0;
      return nystrom_chol_ws_bytes(d, n, k);
    case GP_OP_BPCG:
      if (k < 0 || k > 16384 || k > n || t < 1 || t > 64) return 0;
      return bpcg_ws_bytes(precision, d, n, k, t);
    default:
      return 0;
  }
}

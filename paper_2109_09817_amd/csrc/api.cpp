// C ABI: argument validation, error reporting, workspace sizing and gp_kmm.
#include <algorithm>

#include "api_common.h"
#include "internal.h"

namespace gpk {

std::string& last_error() {
  static thread_local std::string msg;
  return msg;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  last_error() = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what, int line) {
  return fail(GP_EHIP, "HIP error %d (%s) at %s [line %d]", (int)e, hipGetErrorString(e), what, line);
}

int check_kernel(const gp_kernel* k) {
  if (!k) return fail(GP_EINVAL, "kernel descriptor is NULL");
  if (k->kind != GP_MATERN52 && k->kind != GP_RBF) return fail(GP_EINVAL, "unknown kernel kind %d", k->kind);
  if (k->d < 1 || k->d > GP_MAX_D) return fail(GP_EINVAL, "feature count d=%d outside [1, %d]", k->d, GP_MAX_D);
  if (!k->lengthscale) return fail(GP_EINVAL, "lengthscale pointer is NULL");
  for (int j = 0; j < k->d; ++j)
    if (!std::isfinite(k->lengthscale[j]) || !(k->lengthscale[j] > 0.0))
      return fail(GP_EINVAL, "lengthscale[%d]=%g must be finite and > 0", j, k->lengthscale[j]);
  if (!std::isfinite(k->outputscale) || !(k->outputscale > 0.0))
    return fail(GP_EINVAL, "outputscale=%g must be finite and > 0", k->outputscale);
  if (!std::isfinite(k->noise) || k->noise < 0.0) return fail(GP_EINVAL, "noise=%g must be finite and >= 0", k->noise);
  return GP_OK;
}

int check_precision(int32_t p) {
  if (p == GP_PREC_FP64) return fail(GP_EINVAL, "GP_PREC_FP64 is available for gp_kmm, gp_mbcg and gp_bcg only");
  if (p != GP_PREC_FP32 && p != GP_PREC_BF16X3) return fail(GP_EINVAL, "unknown precision %d", p);
  return GP_OK;
}

int check_product_precision(int32_t p) {
  if (p == GP_PREC_FP64) return GP_OK;
  return check_precision(p);
}

int check_ws(const void* ws, size_t have, size_t need, const char* op) {
  if (need == 0) return GP_OK;
  if (!ws) return fail(GP_EWORKSPACE, "%s: workspace is NULL (%zu bytes needed)", op, need);
  if (((uintptr_t)ws & 255) != 0) return fail(GP_EWORKSPACE, "%s: workspace not 256-byte aligned", op);
  if (have < need) return fail(GP_EWORKSPACE, "%s: workspace has %zu bytes, %zu needed", op, have, need);
  return GP_OK;
}

}  // namespace gpk

using namespace gpk;

extern "C" const char* gp_last_error(void) { return last_error().c_str(); }

extern "C" const char* gp_version(void) { return "gpkmm 0.1 (gfx950)"; }

namespace gpk {

int kmm_checked(const gp_kernel* kern, int32_t precision, const double* X, int64_t n, const double* Z, int64_t m,
                const double* V, int64_t ldv, int32_t t, double* out, int64_t ldo, size_t* need) {
  GPK_TRY(check_kernel(kern));
  GPK_TRY(check_product_precision(precision));
  if (!X) return fail(GP_EINVAL, "gp_kmm: X is NULL");
  if (n < 1) return fail(GP_EINVAL, "gp_kmm: n=%lld must be >= 1", (long long)n);
  if (Z && m < 1) return fail(GP_EINVAL, "gp_kmm: m=%lld must be >= 1 when Z is given", (long long)m);
  if (!V || !out) return fail(GP_EINVAL, "gp_kmm: V or out is NULL");
  if (t < 1 || t > 4096) return fail(GP_EINVAL, "gp_kmm: t=%d outside [1, 4096]", t);
  if (ldv < n) return fail(GP_EINVAL, "gp_kmm: ldv=%lld < n=%lld", (long long)ldv, (long long)n);
  const int64_t rows = Z ? m : n;
  if (ldo < rows) return fail(GP_EINVAL, "gp_kmm: ldo=%lld < %lld output rows", (long long)ldo, (long long)rows);
  if ((const void*)out == (const void*)V) return fail(GP_EINVAL, "gp_kmm: out must not alias V");
  *need = kmm_plan_bytes(precision, kern->d, n, rows, Z == nullptr, t);
  return GP_OK;
}

int kmm_run(const gp_kernel* kern, int32_t precision, const double* X, int64_t n, const double* Z, int64_t m,
            const double* V, int64_t ldv, int32_t t, double* out, int64_t ldo, void* ws, size_t ws_bytes,
            hipStream_t st, bool no_timing) {
  const bool square = Z == nullptr;
  KmmPlan p;
  if (!kmm_plan_init(p, kern, precision, n, square ? n : m, square, t, ws, ws_bytes))
    return fail(GP_EWORKSPACE, "gp_kmm: workspace layout failed");
  p.no_timing = no_timing;
  GPK_HIP(kmm_prepare(p, kern, X, Z, st));
  GPK_HIP(kmm_apply(p, V, ldv, t, out, ldo, st, /*row_independent=*/!square));
  return GP_OK;
}

}  // namespace gpk

extern "C" int gp_kmm(const gp_kernel* kern, int32_t precision, const double* X, int64_t n, const double* Z,
                      int64_t m, const double* V, int64_t ldv, int32_t t, double* out, int64_t ldo, void* ws,
                      size_t ws_bytes, void* stream) {
  size_t need = 0;
  GPK_TRY(kmm_checked(kern, precision, X, n, Z, m, V, ldv, t, out, ldo, &need));
  GPK_TRY(check_ws(ws, ws_bytes, need, "gp_kmm"));
  return kmm_run(kern, precision, X, n, Z, m, V, ldv, t, out, ldo, ws, ws_bytes, (hipStream_t)stream, false);
}

extern "C" int gp_profile_enable(int32_t on) {
  profile_enable(on != 0);
  return GP_OK;
}

extern "C" int gp_profile_read(int64_t* launches, double* total_ms, double* nominal_flops, int32_t reset) {
  if (!launches || !total_ms || !nominal_flops) return fail(GP_EINVAL, "gp_profile_read: NULL output");
  if (profile_read(launches, total_ms, nominal_flops, reset != 0) != 0)
    return fail(GP_EHIP, "gp_profile_read: event query failed");
  return GP_OK;
}

extern "C" int gp_profile_records(int64_t cap, int64_t* n, int64_t* m, int32_t* t, double* ms, int64_t* count) {
  if (cap < 0 || !n || !m || !t || !ms || !count) return fail(GP_EINVAL, "gp_profile_records: bad arguments");
  if (profile_records(cap, n, m, t, ms, count) != 0) return fail(GP_EHIP, "gp_profile_records: event query failed");
  return GP_OK;
}

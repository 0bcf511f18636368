// temporary: entry points not yet implemented
#include "api_common.h"
#include "internal.h"
using namespace gpk;
extern "C" {
int gp_kmm_grad(const gp_kernel*, int32_t, const double*, int64_t, const double*, int64_t, const double*, int64_t, int32_t, const double*, double*, void*, size_t, void*) { return fail(GP_EINVAL, "not implemented"); }
int gp_pivchol_precond(const gp_kernel*, const double*, int64_t, int32_t, double*, double*, int64_t*, int32_t*, double*, void*, size_t, void*) { return fail(GP_EINVAL, "not implemented"); }
int gp_mbcg(const gp_kernel*, int32_t, const double*, int64_t, const gp_precond*, const double*, int32_t, int32_t, double, double*, double*, gp_mbcg_out*, void*, size_t, void*) { return fail(GP_EINVAL, "not implemented"); }
int gp_probe_block(const double*, int64_t, int32_t, const double*, int32_t, double, uint64_t, double*, void*) { return fail(GP_EINVAL, "not implemented"); }
int gp_mll_and_grad(const gp_kernel*, const gp_mll_opts*, const double*, const double*, int64_t, double*, double*, gp_mll_info*, void*, size_t, void*) { return fail(GP_EINVAL, "not implemented"); }
int gp_lanczos_cache(const gp_kernel*, int32_t, const double*, const double*, int64_t, int32_t, double*, int32_t*, void*, size_t, void*) { return fail(GP_EINVAL, "not implemented"); }
int gp_predict(const gp_kernel*, int32_t, const double*, int64_t, const double*, const double*, int32_t, const double*, int64_t, double*, double*, void*, size_t, void*) { return fail(GP_EINVAL, "not implemented"); }
size_t gp_workspace_bytes(int32_t op, int64_t n, int64_t m, int32_t d, int32_t t, int32_t k, int32_t precision) {
  if (op == GP_OP_KMM) return kmm_plan_bytes(precision, d, n, m > 0 ? m : n, m <= 0, t);
  return 0;
}
}

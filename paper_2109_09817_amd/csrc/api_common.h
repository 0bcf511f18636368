// Host-side helpers of the C ABI: status/error reporting and argument checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/gpkmm.h"

namespace gpk {

std::string& last_error();
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char* what, int line);

#define GPK_HIP(expr)                                          \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) return ::gpk::hip_fail(_e, #expr, __LINE__); \
  } while (0)

#define GPK_TRY(expr)        \
  do {                       \
    int _s = (expr);         \
    if (_s < 0) return _s;   \
  } while (0)

int check_kernel(const gp_kernel* k);
int check_precision(int32_t p);
// Also accepts GP_PREC_FP64 (the entry points whose only tile product is K_hat V).
int check_product_precision(int32_t p);
int check_ws(const void* ws, size_t have, size_t need, const char* op);

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// gp_kmm in two steps: argument checks (need receives the workspace bytes), then the
// product in the given workspace (no_timing: never record profiling events).
int kmm_checked(const gp_kernel* kern, int32_t precision, const double* X, int64_t n, const double* Z, int64_t m,
                const double* V, int64_t ldv, int32_t t, double* out, int64_t ldo, size_t* need);
int kmm_run(const gp_kernel* kern, int32_t precision, const double* X, int64_t n, const double* Z, int64_t m,
            const double* V, int64_t ldv, int32_t t, double* out, int64_t ldo, void* ws, size_t ws_bytes,
            hipStream_t st, bool no_timing);

// Bump allocator over the caller's workspace.
struct Carve {
  char* p;
  size_t left;
  explicit Carve(void* ws, size_t bytes) : p((char*)ws), left(bytes) {}
  template <class T>
  T* take(size_t count) {
    const size_t b = align256(count * sizeof(T));
    if (b > left) return nullptr;
    T* r = (T*)p;
    p += b;
    left -= b;
    return r;
  }
};

}  // namespace gpk

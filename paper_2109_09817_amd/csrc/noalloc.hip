// gp_kmm_noalloc: the kernel-matrix product of gp_kmm with its scratch memory in
// a fixed device array of the library instead of a caller workspace, for
// callers that cannot allocate device memory at call time.
//
// The array is a file-scope __device__ object, so every device the library is
// loaded on holds one copy of kNoAllocScratchBytes until the process ends.  In
// host code the array's name is only a host-side stand-in: its device address
// is looked up once per device, with that device current, through
// hipGetSymbolAddress, and only that address is handed to kernels.
//
// Every call on one device uses that device's single copy: calls that overlap
// in time on one device (two host threads, or two streams without an ordering
// between them) race on it.  Nothing in the array has to start at zero: the
// product's preparation writes every operand fragment before the sweep reads it,
// and the sweep writes every partial sum before the epilogue reads it.
#include <mutex>

#include "api_common.h"
#include "internal.h"

namespace gpk {

constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;  // GP_KMM_NOALLOC_MAX_BYTES
static_assert(kNoAllocScratchBytes == (size_t)GP_KMM_NOALLOC_MAX_BYTES, "header and library disagree");

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

struct ScratchTable {
  std::mutex mu;
  void* ptr[kMaxDevices] = {};
};

ScratchTable& table() {
  static ScratchTable t;
  return t;
}

// Device address of `scratch` on the device that runs work submitted to `st`.
int scratch_on(hipStream_t st, void** out) {
  int cur = -1;
  GPK_HIP(hipGetDevice(&cur));
  int dev = cur;
  if (st != nullptr) GPK_HIP(hipStreamGetDevice(st, &dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GP_EINVAL, "gp_kmm_noalloc: device %d out of range", dev);
  ScratchTable& t = table();
  std::lock_guard<std::mutex> lock(t.mu);
  if (!t.ptr[dev]) {
    if (dev != cur) GPK_HIP(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) GPK_HIP(hipSetDevice(cur));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)", __LINE__);
    if (!p || ((uintptr_t)p & 255) != 0) return fail(GP_EHIP, "gp_kmm_noalloc: bad scratch address %p", p);
    t.ptr[dev] = p;
  }
  *out = t.ptr[dev];
  return GP_OK;
}

}  // namespace
}  // namespace gpk

using namespace gpk;

extern "C" int gp_kmm_noalloc(const gp_kernel* kern, int32_t precision, const double* X, int64_t n,
                              const double* Z, int64_t m, const double* V, int64_t ldv, int32_t t, double* out,
                              int64_t ldo, void* stream) {
  size_t need = 0;
  GPK_TRY(kmm_checked(kern, precision, X, n, Z, m, V, ldv, t, out, ldo, &need));
  if (need > kNoAllocScratchBytes)
    return fail(GP_EWORKSPACE,
                "gp_kmm_noalloc: this product needs %zu bytes of scratch, more than the library's fixed %zu "
                "(use gp_kmm with a caller workspace)",
                need, kNoAllocScratchBytes);
  hipStream_t st = (hipStream_t)stream;
  void* ws = nullptr;
  GPK_TRY(scratch_on(st, &ws));
  return kmm_run(kern, precision, X, n, Z, m, V, ldv, t, out, ldo, ws, kNoAllocScratchBytes, st, true);
}

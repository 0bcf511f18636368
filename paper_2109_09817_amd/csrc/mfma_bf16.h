// Register types and helpers shared by the mixed-precision tile sweeps (K_hat V,
// the hyperparameter forms and prediction).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace gpk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x8 __attribute__((ext_vector_type(8)));

// log2(e) * sqrt(5) scales x/l so that S = u^2 with u = sqrt5 r log2(e):
// exp(-sqrt5 r) = exp2(-u) and 1 + sqrt5 r + 5r^2/3 = 1 + u ln2 + (u ln2)^2 / 3.
// (The scales are evaluated on the host from M_LOG2E; see make_scale.)
constexpr float kMaternC1 = (float)M_LN2;                  // ln 2
constexpr float kMaternC2 = (float)(M_LN2 * M_LN2 / 3.0);  // (ln 2)^2 / 3
// RBF: S = r^2 log2(e) / 2 so that exp(-r^2/2) = exp2(-S).

// Kernel values and vectors in the K_hat V products of the mixed form are FP16
// hi + lo pairs of scaled values: the kernel value m in [0, 1] enters as
// kMScale m (so that entries down to ~1e-9 stay in FP16's normal range) and each
// column of V is scaled by a power of two that puts its largest entry in
// [2^14, 2^15).  The partial sums are scaled back exactly in FP64.
constexpr float kMScale = 32768.f;  // 2^15
constexpr float kMaternC1s = (float)(32768.0 * M_LN2);              // 2^15 ln 2
constexpr float kMaternC2s = (float)(32768.0 * M_LN2 * M_LN2 / 3.0);  // 2^15 (ln 2)^2 / 3

// Split 8 FP32 values into FP16 hi = RNE(m) (two values per v_cvt_pk_f16_f32)
// and lo = RNE(m - hi): v_fma_mixlo_f16 / v_fma_mixhi_f16 take hi's FP16 half as
// an operand, form m - hi exactly in FP32 and round it into the low or high half
// of the packed result, one instruction per value.  |m - hi| <= 2^-11 |m|, so
// hi + lo holds m to 2^-22 relative (FP16 subnormals: absolute 2^-25 below 2^-14).
// The two results are 16-byte units of the BF16 vector type (reinterpreted, as
// for the point fragments).
__device__ __forceinline__ uint32_t f16_residual_pair(uint32_t h, float m0, float m1) {
  uint32_t l;
  asm("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixhi_f16 %0, %1, -1.0, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
      : "=&v"(l)
      : "v"(h), "v"(m0), "v"(m1));
  return l;
}

__device__ __forceinline__ void split_f16x8(const f32x8& m, bf16x8& H, bf16x8& L) {
  typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  u32x4 h, l;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const f32x2 v = {m[2 * p], m[2 * p + 1]};
    h[p] = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
    l[p] = f16_residual_pair(h[p], v[0], v[1]);
  }
  H = __builtin_bit_cast(bf16x8, h);
  L = __builtin_bit_cast(bf16x8, l);
}

// Value product on the FP16 matrix cores, operands held as 16-byte units.
__device__ __forceinline__ f32x4 mfma_val(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0,
                                                0, 0);
}

// Distance tile on the matrix cores: the point operands are FP16 (see the
// preparation of the point fragments) and travel through registers and LDS as
// 16-byte units of the BF16 vector type; they are reinterpreted, not converted.
__device__ __forceinline__ f32x4 mfma_dist(const bf16x8& b, const bf16x8& a, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, b), __builtin_bit_cast(f16x8, a), c, 0,
                                                0, 0);
}

// K position -> point of a 32-point chunk, for an operand built from the two
// 16x16 distance accumulators of the chunk (lane l holds rows 4(l/16)+i of
// each): K = 8(l/16) + j takes point vperm(l/16, j).
__device__ __forceinline__ int vperm(int g, int j) { return j < 4 ? 4 * g + j : 12 + 4 * g + j; }

}  // namespace gpk

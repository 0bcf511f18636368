// Register types and helpers shared by the BF16X3 tile sweeps (K_hat V, the
// hyperparameter forms and prediction).
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

// Split 8 FP32 values into BF16 hi = RNE(m) and lo = RNE(m - hi), two values per
// v_cvt_pk_bf16_f32; hi is widened back with one shift or mask per value.
__device__ __forceinline__ void split_bf16x8(const f32x8& m, bf16x8& H, bf16x8& L) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const f32x2 v = {m[2 * p], m[2 * p + 1]};
    const bf16x2 h = __builtin_convertvector(v, bf16x2);
    const uint32_t hb = __builtin_bit_cast(uint32_t, h);
    const float h0 = __builtin_bit_cast(float, hb << 16);
    const float h1 = __builtin_bit_cast(float, hb & 0xffff0000u);
    const f32x2 r = {v[0] - h0, v[1] - h1};
    const bf16x2 l = __builtin_convertvector(r, bf16x2);
    H[2 * p] = h[0];
    H[2 * p + 1] = h[1];
    L[2 * p] = l[0];
    L[2 * p + 1] = l[1];
  }
}

// The same split with m - hi (exact in FP32) taken in one instruction
// per value as the BF16 dot product of the packed hi pair with (-1, 0) or
// (0, -1), added to m (an input below FP32's normal range may come out as m
// itself; such a kernel value is far below any tolerance).  The (-1, 0) pair
// is kept in a register: as an immediate the compiler encodes it as the inline
// constant -1.0, whose bit pattern the hardware reads as (0, -1).
__device__ __forceinline__ void split_bf16x8_dot2(const f32x8& m, bf16x8& H, bf16x8& L) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  uint32_t neg_lo_bits = 0x0000bf80u;  // bf16 (-1, 0): low half -1, high half 0
  asm("" : "+v"(neg_lo_bits));        // opaque to constant folding
  const bf16x2 neg_lo = __builtin_bit_cast(bf16x2, neg_lo_bits);
  const bf16x2 neg_hi = __builtin_bit_cast(bf16x2, 0xbf800000u);  // bf16 (0, -1): the FP32 pattern of -1.0
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const f32x2 v = {m[2 * p], m[2 * p + 1]};
    const bf16x2 h = __builtin_convertvector(v, bf16x2);
    const f32x2 r = {__builtin_amdgcn_fdot2_f32_bf16(h, neg_lo, v[0], false),
                     __builtin_amdgcn_fdot2_f32_bf16(h, neg_hi, v[1], false)};
    const bf16x2 l = __builtin_convertvector(r, bf16x2);
    H[2 * p] = h[0];
    H[2 * p + 1] = h[1];
    L[2 * p] = l[0];
    L[2 * p + 1] = l[1];
  }
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

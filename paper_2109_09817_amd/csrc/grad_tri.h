// Upper-triangle tile sweep of the hyperparameter bilinear forms (BF16X3).
//
// The mBCG gradient estimate (Sec. 3.2, the derivative of Eq. 2) needs, for
// every lengthscale j,
//   g_j = sum_{a != b} psi(r_ab) C_ab (x~_aj - x~_bj)^2,   C_ab = sum_c w_c U_ac W_bc,
// and g_{s_f} = sum_{a != b} k(r_ab) C_ab.  psi, k and the squared difference are
// symmetric in (a, b), so both sums run over the pairs a < b only, with C
// replaced by its symmetric part C^s_ab = C_ab + C_ba
//   = sum_c w_c (U_ac W_bc + W_ac U_bc).
// Each unordered pair is evaluated once: half the distance products, half the
// kernel evaluations of the full-matrix sweep.
//
// Work unit: a row group of 64 or 128 rows a (4 waves x one or two 16-row
// blocks, held in registers) against a range of 32-point chunks b at or after the group's own
// first chunk; pairs with b <= a inside a chunk that straddles a block are
// masked.  Per (16 rows) x (32 points) tile, on the matrix cores:
//   S    = |x~_a - x~_b|^2          (distance, K = 3d + 6: FP16 hi/lo coordinates
//                                    centred on the column means, the products
//                                    hi.hi + hi.lo + lo.hi and the norm digits)
//   C^s  = [W_b | U_b] . [w U_a | w W_a]^T   (K = 2t, split three ways)
//   P    = psi(S) C^s, its row sums, and sum k(S) C^s   (registers, FP32)
//   Q, T = P . [x~_b | x~_b^2]       (2 ceil(d/16) blocks of 16 columns; P and the
//                                    columns as FP16 hi/lo of power-of-two scaled values)
// Every 32 chunks the FP32 sums are folded into per-lane FP64 partials of
//   g_j += sum_a x~_aj^2 R_a - 2 x~_aj Q_aj + T_aj,  R_a = sum_b P_ab.
// The b-side fragments of each chunk are staged in LDS, double-buffered, and
// shared by the workgroup's waves.
#pragma once

#include "internal.h"

namespace gpk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct GradTriArgs {
  const bf16x8* xr;     // b-stream FP16 distance fragments (A operand)
  const bf16x8* xc;     // a-row FP16 distance fragments (B operand)
  const bf16x8* cb;     // b-stream fragments of [W | U]        (A operand, K = 6t: hi | hi | lo)
  const bf16x8* ca;     // a-row fragments of [s_P w U | s_P w W]  (B operand, K = 6t: hi | lo | hi)
  const bf16x8* gv;     // b-stream FP16 fragments of the scaled [x~ | x~^2]  (B operand of the forms, hi and lo)
  const int2* units;    // per workgroup: (row group, first chunk)
  const double* X;      // n x d row-major
  const double* mu;     // column means (d)
  const double* inv_ell;  // 1 / lengthscale (d)
  int d;
  int64_t n;
  int64_t nchunks;
  int cps;              // chunk-range alignment of the units
  const double* scal;   // column scalings of the FP16 forms (layout below)
  const double* grpinv; // 1 / s for each wave's group of 16 NA rows (mpad / (16 NA) values)
  double* part;         // per unit: g_1..g_d, g_{s_f} (unscaled)
};

// Scalings of the mixed form's FP16 forms product P . [x~ | x~^2], P = psi (.) C^s.
// The rows of C^s held by one wave (a group of 16 NA rows) enter scaled by the group's
// s, the power of two that puts the largest of the rows' bounds
// sum_c |w_c| (|U_ac| max|W_c| + |W_ac| max|U_c|) >= max_b |C^s_ab| in [2^14, 2^15) (one
// scale per group: the wave's partial sums share it), and each form column by its own
// power of two (largest entry in [2^14, 2^15)); the partial sums are scaled back
// exactly.  Layout of the column array (4 d doubles):
//   [j] scale of x~_j, [d + j] scale of x~_j^2, [2d + j] and [3d + j] their inverses.
inline int grad_scale_doubles(int d) { return 4 * d; }

// Waves per workgroup.  Two 4-wave workgroups share a CU: the per-chunk
// barrier then keeps only half the CU's waves in step, and the other
// workgroup's waves fill the matrix cores while these run their VALU phase.
constexpr int kTriWaves = 4;
constexpr int kTriFlush = 32;  // chunks per FP32 accumulation window

// 16-row blocks per wave: two while they fit in 256 registers without spilling
// (the staged b-side fragments then serve two tiles per LDS read), else one.
// The largest C K-step count with two blocks per (KS, NJ) instantiation is read
// off the compiled register counts.
constexpr int tri_max_ksc2(int ks, int nj) {
  return ks <= 4 && nj == 1 ? 12 : (ks <= 4 && nj == 2 ? 8 : (ks == 5 && nj == 3 ? 8 : (ks == 7 && nj == 4 ? 2 : 0)));
}
constexpr int tri_na(int ks, int ksc, int nj) { return ksc <= tri_max_ksc2(ks, nj) ? 2 : 1; }
// The C^s phase runs for both row blocks at once (each staged C fragment read
// once, the next K step's fragments read during the current MFMAs) where the
// extra accumulators still fit; otherwise it runs block by block.
constexpr int tri_max_ksc_joint(int ks, int nj) {
  return ks <= 4 && nj == 1 ? 12 : (ks <= 4 && nj <= 2 ? 8 : (ks == 5 && nj == 3 ? 4 : (ks == 7 && nj == 4 ? 1 : 0)));
}
constexpr bool tri_joint_c(int ks, int ksc, int nj) {
  return tri_na(ks, ksc, nj) == 1 || ksc <= tri_max_ksc_joint(ks, nj);
}
// Rows of one row group (a workgroup's register-resident rows).
constexpr int tri_rows(int ks, int ksc, int nj) { return 16 * kTriWaves * tri_na(ks, ksc, nj); }

// K steps of 32 of the distance operands for d features (K = 3d + 6), one
// instantiated count per number of 16-feature form blocks nj = ceil(d / 16):
// 2, 4, 5, 7 for nj = 1..4 (each covers the largest d of its nj); -1 above
// d = 64.  The zero K padding is exact.
inline int tri_ks_of(int d) {
  static const int kByNj[] = {2, 4, 5, 7};
  if (d < 1 || d > 64) return -1;
  const int ks = kByNj[(d + 15) / 16 - 1];
  return ks * 32 >= 3 * d + 6 ? ks : -1;
}

// Launch one instantiation; false if (ks, nj, ksc) has none.
bool launch_grad_tri_matern(int ks, int nj, int ksc, unsigned units, const GradTriArgs& a, hipStream_t st);
bool launch_grad_tri_rbf(int ks, int nj, int ksc, unsigned units, const GradTriArgs& a, hipStream_t st);

// Instantiated chunk widths of the C^s product (K steps of 32 for 6t terms).
int grad_tri_ksc(int t);

}  // namespace gpk

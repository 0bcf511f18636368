// Internal declarations shared by the host orchestration and the HIP kernels
// of libgpkmm.  Not part of the public ABI (see include/gpkmm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/gpkmm.h"

namespace gpk {

// Feature scaling passed by value to the preparation kernels: x~_j = x_j * s[j].
struct Scale {
  double s[GP_MAX_D];
};

// Geometry of one prepared kernel-matrix product (square K_hat V or cross K(Z, X) V).
//
// Operand streams (all in caller workspace):
//   xr   "row side" fragments of the n training points: they play the column
//        (summation) index b of the product and feed the distance MFMA as its
//        A operand; the stream every workgroup sweeps.
//   xc   "column side" fragments of the output rows a (training points for
//        the square product, query rows for the cross product); they stay in
//        registers for a workgroup's whole sweep.
//   vf   the right-hand sides V split into MFMA B-operand fragments.
//   part FP64 partial sums per split of the b range.
struct KmmPlan {
  int precision = 0;  // GP_PREC_*
  int kind = 0;       // GP_MATERN52 / GP_RBF
  int d = 0;
  bool square = true;
  int64_t n = 0, m = 0;         // training rows, output rows
  int64_t npad = 0, mpad = 0;   // n rounded to 32, m rounded to 256
  int64_t nchunks = 0;          // npad / 32
  int ks = 0;                   // K steps: 32-wide (BF16X3) or 16-wide float4 groups (FP32)
  int tmax = 0;                 // columns the plan was sized for
  int ntb = 0;                  // 16-column blocks for tmax
  double sf = 1.0, noise = 0.0;
  bool no_timing = false;       // never record profiling events (the allocation-free entry point)
  // workspace carve-out
  void* xr = nullptr;
  void* xc = nullptr;
  float* nrm_b = nullptr;   // FP32 form: norms of the b stream
  float* nrm_a = nullptr;   // FP32 form: norms of the output rows
  double* nrm64 = nullptr;  // FP64 norms scratch (n or m entries)
  double* ctr = nullptr;    // mixed form: the centre of the coordinates (the b stream's column means, d values)
  double* cpart = nullptr;  // scratch of the column means (colmean_scratch_doubles(n, d))
  void* vf = nullptr;
  double* vscale = nullptr;  // mixed form: per-column power-of-two scale of V's fragments (tpad values)
  double* vinv = nullptr;    // mixed form: 2^-15 / vscale, applied to the partial sums (tpad values)
  double* vpart = nullptr;   // mixed form: column-max partials (scratch of kmm_prepare_v)
  double* part = nullptr;
  int64_t part_splits = 0;  // splits the partial buffer can hold
  // FP64 form: the points themselves (caller memory), prescaled features and norms
  const double* x64 = nullptr;  // b stream (training points), n x d
  const double* z64 = nullptr;  // output rows, m x d
  double* sc64 = nullptr;       // d feature scales
  double* nb64 = nullptr;       // n squared norms of the scaled b points
  double* na64 = nullptr;       // m squared norms of the scaled output rows
};

// Number of 32-wide K steps (BF16X3) or 16-wide groups (FP32) for d features.
int kmm_ksteps(int precision, int d);
// Bytes of workspace for a plan (square: Z == X).
size_t kmm_plan_bytes(int precision, int d, int64_t n, int64_t m, bool square, int tmax);
// Carve a plan out of ws (no GPU work).  Returns false if ws is too small.
bool kmm_plan_init(KmmPlan& p, const gp_kernel* kern, int precision, int64_t n, int64_t m,
                   bool square, int tmax, void* ws, size_t ws_bytes);
// Prepare the point operands (X, and Z for a cross product).
hipError_t kmm_prepare(KmmPlan& p, const gp_kernel* kern, const double* X, const double* Z,
                       hipStream_t st);
// Prepare only the b stream (training points) or only the output rows.
hipError_t kmm_prepare_rows(KmmPlan& p, const gp_kernel* kern, const double* X, hipStream_t st);
hipError_t kmm_prepare_cols(KmmPlan& p, const gp_kernel* kern, const double* Z, hipStream_t st);
// Split V (column-major, ldv, t columns) into the plan's V fragments.
// col0 (optional): column 0 taken from col0, columns c >= 1 from V column c - 1.
hipError_t kmm_prepare_v(const KmmPlan& p, const double* V, int64_t ldv, int t, bool row_independent,
                         hipStream_t st, const double* col0 = nullptr);
// The sweep and epilogue on already-prepared operands (Vdiag: V for the exact
// diagonal term of the square product, ignored for cross products).
hipError_t kmm_sweep(const KmmPlan& p, int t, const double* Vdiag, int64_t ldv, double* out, int64_t ldo,
                     hipStream_t st, bool row_independent);
// The factor c of the prescaled coordinates x' = c (x - centre) / l, chosen so that the
// profile reads r^2 through exp2: sqrt(5) log2(e) for Matern-5/2, sqrt(log2(e) / 2) for RBF.
double profile_coordinate_scale(int kind);
// The mixed form's FP16 distance operands of a square product (prep_frag_f16x3_kernel)
// at ks K steps of 32 (ks * 32 >= 3d + 6), centred on ctr (d device values, the
// column means of X): the b-side (xr) and a-side (xc) fragments of rows_pad points
// (a multiple of 64; points >= n are zero), with nrm64 (rows_pad doubles) as
// scratch for the squared norms.
hipError_t prep_dist(const gp_kernel* kern, const double* X, int64_t n, int64_t rows_pad, int ks, const double* ctr,
                     void* xr, void* xc, double* nrm64, hipStream_t st);
// Column means of the row-major n x d matrix X into mu (d doubles), deterministic;
// part: colmean_scratch_doubles(n, d) doubles of scratch.
size_t colmean_scratch_doubles(int64_t n, int d);
hipError_t column_means(const double* X, int64_t n, int d, double* part, double* mu, hipStream_t st);
// Largest |V| of each of the t columns of V (column-major, ldv, n rows) into out (t
// doubles, device); part: column_absmax_scratch_doubles(t) doubles of scratch.  NaN
// entries are skipped.
size_t column_absmax_scratch_doubles(int t);
hipError_t column_absmax(const double* V, int64_t ldv, int64_t n, int t, double* part, double* out, hipStream_t st);
// Bytes of the V fragments for t columns.
size_t kmm_vfrag_bytes(int64_t n, int t);
// A cross-product plan split in two: the training-side operands (b stream and V
// fragments) in a long-lived `model` buffer, the query side in `ws`.
size_t kmm_model_bytes(int precision, int d, int64_t n, int tmax);
size_t kmm_query_bytes(int precision, int d, int64_t n, int64_t m, int tmax);
bool kmm_plan_model(KmmPlan& p, const gp_kernel* kern, int precision, int64_t n, int64_t m, int tmax, void* model,
                    size_t model_bytes, void* ws, size_t ws_bytes);
// out = K_hat V (square) or K(Z, X) V (cross), V column-major (ldv), t <= tmax columns.
// Splits of the b range are chosen from n only when `row_independent` is set,
// so that each output row's arithmetic does not depend on m.
hipError_t kmm_apply(const KmmPlan& p, const double* V, int64_t ldv, int t, double* out,
                     int64_t ldo, hipStream_t st, bool row_independent = false);

// Sweep timing (see gp_profile_enable / gp_profile_read).
void profile_enable(bool on);
int profile_read(int64_t* launches, double* total_ms, double* flops, bool reset);
int profile_records(int64_t cap, int64_t* n, int64_t* m, int* t, double* ms, int64_t* count);

}  // namespace gpk

// FP64 kernels of the solver: column reductions, the mBCG recurrences, the
// pivoted-Cholesky preconditioner (build and Woodbury apply) and the probe
// generator.  These passes stream O(n s) or O(n k) data per call and are
// bound by HBM bandwidth; all reductions are two-pass with a fixed order
// (per-block partials, then one block per output), so results are bitwise
// reproducible run to run.
//
// Layout: every block of vectors is column-major with leading dimension n
// (column c of an n x s block starts at c*n).
#include "solver.h"

namespace gpk {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block-wide sum in a fixed order; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;
}

// partial[blk * s + c] = sum over this block's rows of A[c*n+i] * B[c*n+i].
// grid = (nblk, s).  Rows are split in contiguous ranges per block.
__global__ void coldot_partial_kernel(const double* __restrict__ A, const double* __restrict__ B, int64_t n,
                                      int64_t rows_per_blk, int s, double* __restrict__ partial) {
  __shared__ double sh[kThreads / 64];
  const int c = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < n ? r0 + rows_per_blk : n;
  const double* a = A + (int64_t)c * n;
  const double* b = B + (int64_t)c * n;
  double acc = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) acc += a[i] * b[i];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * s + c] = r;
}

// out[c] = sum_blk partial[blk * s + c] (fixed order).  grid = (s).
__global__ void reduce_partials_kernel(const double* __restrict__ partial, int64_t nblk, int s,
                                       double* __restrict__ out) {
  __shared__ double sh[kThreads / 64];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (int64_t b = threadIdx.x; b < nblk; b += blockDim.x) acc += partial[b * s + c];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) out[c] = r;
}

// ------------------------------------------------------------------ mBCG steps

// alpha = gamma / (d.w) for active columns (0 for frozen ones); flags breakdown.
__global__ void mbcg_alpha_kernel(MbcgState st) {
  const int c = threadIdx.x;
  if (c >= st.s) return;
  double a = 0.0;
  if (st.active[c]) {
    const double dl = st.delta[c];
    if (!isfinite(dl) || !isfinite(st.gamma[c])) {
      atomicOr(st.status, kStatusNonFinite);
    } else if (!(dl > 0.0)) {
      atomicOr(st.status, kStatusNotPD);
    } else {
      a = st.gamma[c] / dl;
    }
  }
  st.alpha[c] = a;
}

// U += alpha D ; R -= alpha W ; partial ||R||^2.  grid = (nblk, s).
__global__ void mbcg_update_ur_kernel(MbcgState st, const double* __restrict__ D, const double* __restrict__ W,
                                      double* __restrict__ U, double* __restrict__ R, int64_t n,
                                      int64_t rows_per_blk, double* __restrict__ partial) {
  __shared__ double sh[kThreads / 64];
  const int c = blockIdx.y;
  const double a = st.alpha[c];
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < n ? r0 + rows_per_blk : n;
  const int64_t off = (int64_t)c * n;
  double acc = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const double r = R[off + i] - a * W[off + i];
    U[off + i] += a * D[off + i];
    R[off + i] = r;
    acc += r * r;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * st.s + c] = s;
}

// Convergence bookkeeping after the residual update of iteration j.
__global__ void mbcg_freeze_kernel(MbcgState st, int j, double tol) {
  const int c = threadIdx.x;
  if (c < st.s && st.active[c]) {
    const double rn = sqrt(st.rnorm2[c]);
    st.iters[c] = j + 1;
    st.relres[c] = st.bnorm[c] > 0.0 ? rn / st.bnorm[c] : 0.0;
    if (!isfinite(rn)) atomicOr(st.status, kStatusNonFinite);
    if (rn <= tol * st.bnorm[c]) st.active[c] = 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int na = 0;
    for (int i = 0; i < st.s; ++i) na += st.active[i];
    *st.num_active = na;
  }
}

// beta = gamma'/gamma for active columns (0 for frozen ones); gamma <- gamma'.
__global__ void mbcg_beta_kernel(MbcgState st) {
  const int c = threadIdx.x;
  if (c >= st.s) return;
  double b = 0.0;
  if (st.active[c]) {
    const double gn = st.gamma_new[c];
    if (!isfinite(gn)) atomicOr(st.status, kStatusNonFinite);
    b = gn / st.gamma[c];
    st.gamma[c] = gn;
  }
  st.beta[c] = b;
}

// D = Z + beta D for active columns, 0 for frozen ones.  grid = (nblk, s).
__global__ void mbcg_update_d_kernel(MbcgState st, const double* __restrict__ Z, double* __restrict__ D,
                                     int64_t n, int64_t rows_per_blk) {
  const int c = blockIdx.y;
  const bool act = st.active[c] != 0;
  const double b = st.beta[c];
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < n ? r0 + rows_per_blk : n;
  const int64_t off = (int64_t)c * n;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) D[off + i] = act ? Z[off + i] + b * D[off + i] : 0.0;
}

// Initial state: gamma0 = gamma, active = ||b|| > 0, counters cleared.
__global__ void mbcg_init_kernel(MbcgState st) {
  const int c = threadIdx.x;
  if (c < st.s) {
    st.gamma0[c] = st.gamma[c];
    st.bnorm[c] = sqrt(st.bnorm[c]);
    st.active[c] = st.bnorm[c] > 0.0 ? 1 : 0;
    st.iters[c] = 0;
    st.relres[c] = st.bnorm[c] > 0.0 ? 1.0 : 0.0;
    if (!isfinite(st.gamma[c]) || !isfinite(st.bnorm[c])) atomicOr(st.status, kStatusNonFinite);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int na = 0;
    for (int i = 0; i < st.s; ++i) na += st.active[i];
    *st.num_active = na;
  }
}

// -------------------------------------------------------- tall-skinny products

// partial[blk][p][q] of G = A^T B over this block's rows, A (n x pa), B (n x qb),
// both column-major with ld n.  grid = (nblk, ceil(pa/64), ceil(qb/(4 MQ))),
// 256 threads, 64-row tiles staged in LDS; each thread owns MQ outputs
// (q = q0 + tid / 64 + 4 m, m < MQ), so a narrow B carries no idle columns.
template <int MQ>
__global__ void __launch_bounds__(256) atb_partial_kernel(const double* __restrict__ A, int pa,
                                                          const double* __restrict__ B, int qb, int64_t n,
                                                          int64_t rows_per_blk, double* __restrict__ partial) {
  __shared__ double As[64][65];
  __shared__ double Bs[4 * MQ][65];
  const int p0 = blockIdx.y * 64, q0 = blockIdx.z * (4 * MQ);
  const int tid = threadIdx.x;
  const int pl = tid & 63;        // this thread's p (local)
  const int qg = tid >> 6;        // q = q0 + qg + 4 m, m = 0..MQ-1
  double acc[MQ];
#pragma unroll
  for (int m = 0; m < MQ; ++m) acc[m] = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < n ? r0 + rows_per_blk : n;
  for (int64_t t0 = r0; t0 < r1; t0 += 64) {
    // stage A[t0..t0+63][p0..p0+63] and B likewise (zero outside): this thread
    // stages row t0 + tid % 64 of columns tid / 64 + 4 u, all 32 loads issued
    // before the first store (indexes clamped into the matrices)
    const int r = tid & 63;
    const int64_t row = t0 + r;
    const int64_t rowc = row < n ? row : n - 1;
    double av[16], bv[MQ];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int col = (tid >> 6) + 4 * u;
      av[u] = A[(int64_t)(p0 + col < pa ? p0 + col : pa - 1) * n + rowc];
      if (u < MQ) bv[u] = B[(int64_t)(q0 + col < qb ? q0 + col : qb - 1) * n + rowc];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int col = (tid >> 6) + 4 * u;
      As[col][r] = (row < r1 && p0 + col < pa) ? av[u] : 0.0;
      if (u < MQ) Bs[col][r] = (row < r1 && q0 + col < qb) ? bv[u] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int r = 0; r < 64; ++r) {
      const double av = As[pl][r];
#pragma unroll
      for (int m = 0; m < MQ; ++m) acc[m] += av * Bs[qg + 4 * m][r];
    }
    __syncthreads();
  }
  const int64_t base = (int64_t)blockIdx.x * pa * qb;
#pragma unroll
  for (int m = 0; m < MQ; ++m) {
    const int p = p0 + pl, q = q0 + qg + 4 * m;
    if (p < pa && q < qb) partial[base + (int64_t)p * qb + q] = acc[m];
  }
}

// out[p*qb + q] = sum_blk partial (fixed order).  One thread per output.
__global__ void atb_reduce_kernel(const double* __restrict__ partial, int64_t nblk, int64_t pq,
                                  double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= pq) return;
  double acc = 0.0;
  int64_t b = 0;
  for (; b + 8 <= nblk; b += 8) {  // eight loads in flight, added in block order
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = partial[(b + u) * pq + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; b < nblk; ++b) acc += partial[b * pq + e];
  out[e] = acc;
}

// Y := C^{-1} Y for the k x s right-hand sides Y (row-major k x s, entry [j*s + c]),
// with the lower Cholesky factor Lc (column-major k x k).  One thread per column.
__global__ void chol_solve_kernel(const double* __restrict__ Lc, int k, double* __restrict__ Y, int s) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= s) return;
  // The terms of each dot product are subtracted in index order; their loads
  // are issued eight at a time so that the chain waits once per eight terms.
  // forward: Lc z = y
  for (int j = 0; j < k; ++j) {
    double v = Y[(int64_t)j * s + c];
    int i = 0;
    for (; i + 8 <= j; i += 8) {
      double lv[8], yv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        lv[u] = Lc[(int64_t)(i + u) * k + j];
        yv[u] = Y[(int64_t)(i + u) * s + c];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) v -= lv[u] * yv[u];
    }
    for (; i < j; ++i) v -= Lc[(int64_t)i * k + j] * Y[(int64_t)i * s + c];
    Y[(int64_t)j * s + c] = v / Lc[(int64_t)j * k + j];
  }
  // backward: Lc^T x = z
  for (int j = k - 1; j >= 0; --j) {
    double v = Y[(int64_t)j * s + c];
    int i = j + 1;
    for (; i + 8 <= k; i += 8) {
      double lv[8], yv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        lv[u] = Lc[(int64_t)j * k + i + u];
        yv[u] = Y[(int64_t)(i + u) * s + c];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) v -= lv[u] * yv[u];
    }
    for (; i < k; ++i) v -= Lc[(int64_t)j * k + i] * Y[(int64_t)i * s + c];
    Y[(int64_t)j * s + c] = v / Lc[(int64_t)j * k + j];
  }
}

// Z = inv_noise * (R - L Y) for columns [c0, c0 + sc), sc <= SC, Y row-major k x s.
// One thread per row with SC accumulators; Y staged in LDS in chunks of 64 rows.
template <int SC>
__global__ __launch_bounds__(256) void woodbury_finish_kernel(const double* __restrict__ L, int k,
                                                              const double* __restrict__ Y, int s, int c0, int sc,
                                                              const double* __restrict__ R, double* __restrict__ Z,
                                                              int64_t n, double inv_noise) {
  __shared__ double Ys[64 * SC];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[SC];
#pragma unroll
  for (int c = 0; c < SC; ++c) acc[c] = 0.0;
  for (int j0 = 0; j0 < k; j0 += 64) {
    const int jn = k - j0 < 64 ? k - j0 : 64;
    __syncthreads();
    for (int e = threadIdx.x; e < jn * sc; e += blockDim.x) {
      const int jj = e / sc, c = e - jj * sc;
      Ys[jj * SC + c] = Y[(int64_t)(j0 + jj) * s + c0 + c];
    }
    __syncthreads();
    if (i < n) {
      for (int jj = 0; jj < jn; ++jj) {
        const double l = L[(int64_t)(j0 + jj) * n + i];
#pragma unroll
        for (int c = 0; c < SC; ++c)
          if (c < sc) acc[c] += l * Ys[jj * SC + c];
      }
    }
  }
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < SC; ++c)
    if (c < sc) {
      const int64_t o = (int64_t)(c0 + c) * n + i;
      Z[o] = inv_noise * (R[o] - acc[c]);
    }
}

__global__ void copy_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}

__global__ void zero_words_kernel(uint32_t* __restrict__ dst, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = 0u;
}

__global__ void fill_kernel(double* __restrict__ dst, double v, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = v;
}

// w -= Q h  (Q: n x jn column-major, h: jn values).  One thread per row.
__global__ void gemv_sub_kernel(const double* __restrict__ Q, int64_t n, int jn, const double* __restrict__ h,
                                double* __restrict__ w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int j = 0; j < jn; ++j) acc += Q[(int64_t)j * n + i] * h[j];
  w[i] -= acc;
}

// dst = src * (*scale_inv_sqrt)^(-1/2): dst = src / sqrt(*s2)
__global__ void scale_rsqrt_kernel(const double* __restrict__ src, const double* __restrict__ s2, int64_t n,
                                   double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i] / sqrt(*s2);
}

// In place Q -> R = Q L_T^{-T} for the lower bidiagonal Cholesky factor L_T of
// the Lanczos tridiagonal (diagonal l_j, subdiagonal m_j):
//   R[:, j] = (Q[:, j] - m_j R[:, j-1]) / l_j.   One thread per row.
__global__ void bidiag_solve_kernel(double* __restrict__ QR, int64_t n, int K, const double* __restrict__ lm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double prev = 0.0;
  for (int j = 0; j < K; ++j) {
    const double v = (QR[(int64_t)j * n + i] - (j > 0 ? lm[2 * j + 1] * prev : 0.0)) / lm[2 * j];
    QR[(int64_t)j * n + i] = v;
    prev = v;
  }
}

// mean[q] = P[q]; var[q] = s_f - sum_{c=1..kc} P[c*m + q]^2.  One wave per
// query row: lane l adds the columns 1 + l, 65 + l, ... in order, then an XOR
// butterfly adds the lanes (the same order on every lane, fixed by kc alone).
__global__ __launch_bounds__(256) void predict_finish_kernel(const double* __restrict__ P, int64_t m, int kc,
                                                             double sf, double* __restrict__ mean,
                                                             double* __restrict__ var) {
  const int lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= m) return;  // whole wave
  if (lane == 0) mean[q] = P[q];
  if (var) {
    double s = 0.0;
    for (int c = 1 + lane; c <= kc; c += 64) {
      const double v = P[(int64_t)c * m + q];
      s += v * v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) var[q] = sf - s;
  }
}

// --------------------------------------------------------------------- probes

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double rademacher(uint64_t key, uint64_t stream, uint64_t row) {
  return (splitmix64(key ^ ((stream << 40) | row)) >> 63) ? -1.0 : 1.0;
}

// Column c >= 1 of B: L e1_c + sqrt(noise) e2_c (or e2_c when k == 0); column 0 = y.
// grid = (ceil(n/256), t+1).  e1 signs are recomputed per thread from the hash.
__global__ void probe_kernel(const double* __restrict__ y, int64_t n, const double* __restrict__ L, int k,
                             double sigma, uint64_t key, double* __restrict__ B) {
  __shared__ double e1[1024];
  const int c = blockIdx.y;
  if (c > 0 && k > 0) {
    for (int j = threadIdx.x; j < k; j += blockDim.x)
      e1[j] = rademacher(key, (uint64_t)c + kEps1StreamOffset, (uint64_t)j);
    __syncthreads();
  }
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v;
  if (c == 0) {
    v = y[i];
  } else {
    const double e2 = rademacher(key, (uint64_t)c, (uint64_t)i);
    if (k == 0) {
      v = e2;
    } else {
      double acc = 0.0;
      for (int j = 0; j < k; ++j) acc += L[(int64_t)j * n + i] * e1[j];
      v = acc + sigma * e2;
    }
  }
  B[(int64_t)c * n + i] = v;
}

// ------------------------------------------------------------ pivoted Cholesky

// Per-block argmax of delta (largest value, lowest index on ties) -> partial.
__global__ void argmax_partial_kernel(const double* __restrict__ delta, int64_t n, int64_t rows_per_blk,
                                      double* __restrict__ pval, int64_t* __restrict__ pidx) {
  __shared__ double sv[kThreads];
  __shared__ int64_t si[kThreads];
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < n ? r0 + rows_per_blk : n;
  double bv = -1.0;
  int64_t bi = -1;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    const double v = delta[i];
    if (v > bv) {  // strictly greater: the first (lowest) index of a tie wins within a thread
      bv = v;
      bi = i;
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const double ov = sv[threadIdx.x + off];
      const int64_t oi = si[threadIdx.x + off];
      const double mv = sv[threadIdx.x];
      const int64_t mi = si[threadIdx.x];
      if (ov > mv || (ov == mv && oi >= 0 && (mi < 0 || oi < mi))) {
        sv[threadIdx.x] = ov;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pval[blockIdx.x] = sv[0];
    pidx[blockIdx.x] = si[0];
  }
}

// Final argmax over block partials; records the pivot of step m or stops.
// Largest value, lowest index on ties: the answer does not depend on the order
// in which partials are combined, so one block reduces them as a tree.
__global__ __launch_bounds__(kThreads) void argmax_final_kernel(const double* __restrict__ pval,
                                                                const int64_t* __restrict__ pidx, int64_t nblk,
                                                                PivState ps, int m, double stop_below) {
  __shared__ double sv[kThreads];
  __shared__ int64_t si[kThreads];
  if (*ps.rank < m) return;  // already stopped (the same for every thread)
  double bv = -1.0;
  int64_t bi = -1;
  for (int64_t b = threadIdx.x; b < nblk; b += kThreads) {
    const double v = pval[b];
    const int64_t i = pidx[b];
    if (i >= 0 && (bi < 0 || v > bv || (v == bv && i < bi))) {
      bv = v;
      bi = i;
    }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const double ov = sv[threadIdx.x + off];
      const int64_t oi = si[threadIdx.x + off];
      const double mv = sv[threadIdx.x];
      const int64_t mi = si[threadIdx.x];
      if (oi >= 0 && (mi < 0 || ov > mv || (ov == mv && oi < mi))) {
        sv[threadIdx.x] = ov;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  bv = sv[0];
  bi = si[0];
  if (!(bv > stop_below) || bi < 0) {
    return;  // rank stays m
  }
  ps.piv[m] = bi;
  ps.pivval[m] = bv;
  *ps.rank = m + 1;
}

// Column m of L for all rows: l_a = (K(x_a, x_p) - L[a, :m] L[p, :m]^T) / sqrt(delta_p),
// delta_a -= l_a^2, delta_p = 0.  Kernel values in FP64 by direct differences.
__global__ void pivchol_column_kernel(const double* __restrict__ X, int64_t n, int d, Scale inv_ell, int kind,
                                      double sf, double* __restrict__ L, double* __restrict__ delta, PivState ps,
                                      int m) {
  __shared__ double xp[GP_MAX_D];
  __shared__ double lp[1024];
  if (*ps.rank <= m) return;  // stopped before step m
  const int64_t p = ps.piv[m];
  for (int j = threadIdx.x; j < d; j += blockDim.x) xp[j] = X[p * d + j];
  for (int j = threadIdx.x; j < m; j += blockDim.x) lp[j] = L[(int64_t)j * n + p];
  __syncthreads();
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  double r2 = 0.0;
  for (int j = 0; j < d; ++j) {
    const double df = (X[a * d + j] - xp[j]) * inv_ell.s[j];
    r2 += df * df;
  }
  double kv;
  if (kind == GP_MATERN52) {
    const double s = sqrt(5.0 * r2);
    kv = sf * (1.0 + s + s * s / 3.0) * exp(-s);
  } else {
    kv = sf * exp(-0.5 * r2);
  }
  double acc = 0.0;
  for (int j = 0; j < m; ++j) acc += L[(int64_t)j * n + a] * lp[j];
  const double l = (kv - acc) / sqrt(ps.pivval[m]);
  L[(int64_t)m * n + a] = l;
  delta[a] = (a == p) ? 0.0 : delta[a] - l * l;
}

// --------------------------------------------------------------- host helpers

static unsigned blocks_for(int64_t count, int thr = kThreads) { return (unsigned)((count + thr - 1) / thr); }

RowSplit row_split(int64_t n, int64_t target_blocks) {
  RowSplit r;
  int64_t per = (n + target_blocks - 1) / target_blocks;
  per = (per + kThreads - 1) / kThreads * kThreads;
  if (per < kThreads) per = kThreads;
  r.rows_per_blk = per;
  r.nblk = (n + per - 1) / per;
  return r;
}

hipError_t coldot(const double* A, const double* B, int64_t n, int s, double* out, double* partial,
                  hipStream_t st) {
  const RowSplit rs = row_split(n, kDotBlocks);
  coldot_partial_kernel<<<dim3((unsigned)rs.nblk, (unsigned)s), kThreads, 0, st>>>(A, B, n, rs.rows_per_blk, s,
                                                                                   partial);
  reduce_partials_kernel<<<s, kThreads, 0, st>>>(partial, rs.nblk, s, out);
  return hipGetLastError();
}

static void launch_atb_partial(const double* A, int pa, const double* B, int qb, int64_t n, const RowSplit& rs,
                               double* partial, hipStream_t st) {
  const unsigned gy = (unsigned)((pa + 63) / 64);
  if (qb <= 4) {
    atb_partial_kernel<1><<<dim3((unsigned)rs.nblk, gy, 1), 256, 0, st>>>(A, pa, B, qb, n, rs.rows_per_blk, partial);
  } else if (qb <= 16) {
    atb_partial_kernel<4><<<dim3((unsigned)rs.nblk, gy, 1), 256, 0, st>>>(A, pa, B, qb, n, rs.rows_per_blk, partial);
  } else {
    atb_partial_kernel<16><<<dim3((unsigned)rs.nblk, gy, (unsigned)((qb + 63) / 64)), 256, 0, st>>>(
        A, pa, B, qb, n, rs.rows_per_blk, partial);
  }
}

size_t atb_partial_doubles(int64_t n, int pa, int qb) {
  const RowSplit rs = row_split(n, kAtbBlocks);
  return (size_t)rs.nblk * pa * qb;
}

hipError_t atb(const double* A, int pa, const double* B, int qb, int64_t n, double* out, double* partial,
               hipStream_t st) {
  const RowSplit rs = row_split(n, kAtbBlocks);
  launch_atb_partial(A, pa, B, qb, n, rs, partial, st);
  const int64_t pq = (int64_t)pa * qb;
  atb_reduce_kernel<<<blocks_for(pq), kThreads, 0, st>>>(partial, rs.nblk, pq, out);
  return hipGetLastError();
}

hipError_t atb_n(const double* A, int pa, const double* B, int qb, int64_t n, double* out, double* partial,
                 int64_t nblk, hipStream_t st) {
  const RowSplit rs = row_split(n, nblk);
  launch_atb_partial(A, pa, B, qb, n, rs, partial, st);
  const int64_t pq = (int64_t)pa * qb;
  atb_reduce_kernel<<<blocks_for(pq), kThreads, 0, st>>>(partial, rs.nblk, pq, out);
  return hipGetLastError();
}

hipError_t precond_apply(const Precond& pc, const double* R, double* Z, int64_t n, int s, double* Y,
                         double* partial, hipStream_t st) {
  if (pc.rank == 0) {
    copy_kernel<<<blocks_for(n * s), kThreads, 0, st>>>(R, Z, n * s);
    return hipGetLastError();
  }
  // Y = L^T R  (k x s, row-major [j*s + c])
  hipError_t e = atb(pc.L, pc.rank, R, s, n, Y, partial, st);
  if (e != hipSuccess) return e;
  chol_solve_kernel<<<blocks_for(s, 64), 64, 0, st>>>(pc.Cchol, pc.rank, Y, s);
  for (int c0 = 0; c0 < s; c0 += 64) {
    const int sc = s - c0 < 64 ? s - c0 : 64;
    const double inv = 1.0 / pc.noise;
    if (sc <= 16)
      woodbury_finish_kernel<16><<<blocks_for(n), kThreads, 0, st>>>(pc.L, pc.rank, Y, s, c0, sc, R, Z, n, inv);
    else if (sc <= 32)
      woodbury_finish_kernel<32><<<blocks_for(n), kThreads, 0, st>>>(pc.L, pc.rank, Y, s, c0, sc, R, Z, n, inv);
    else
      woodbury_finish_kernel<64><<<blocks_for(n), kThreads, 0, st>>>(pc.L, pc.rank, Y, s, c0, sc, R, Z, n, inv);
  }
  return hipGetLastError();
}

hipError_t launch_probes(const double* y, int64_t n, int t, const double* L, int k, double noise, uint64_t seed,
                         double* B, hipStream_t st) {
  const uint64_t key = splitmix64_host(seed);
  probe_kernel<<<dim3(blocks_for(n), (unsigned)(t + 1)), kThreads, 0, st>>>(y, n, L, k, std::sqrt(noise), key, B);
  return hipGetLastError();
}

hipError_t launch_gemv_sub(const double* Q, int64_t n, int jn, const double* h, double* w, hipStream_t st) {
  gemv_sub_kernel<<<blocks_for(n), kThreads, 0, st>>>(Q, n, jn, h, w);
  return hipGetLastError();
}

hipError_t launch_scale_rsqrt(const double* src, const double* s2, int64_t n, double* dst, hipStream_t st) {
  scale_rsqrt_kernel<<<blocks_for(n), kThreads, 0, st>>>(src, s2, n, dst);
  return hipGetLastError();
}

hipError_t launch_bidiag_solve(double* QR, int64_t n, int K, const double* lm, hipStream_t st) {
  bidiag_solve_kernel<<<blocks_for(n), kThreads, 0, st>>>(QR, n, K, lm);
  return hipGetLastError();
}

hipError_t launch_predict_finish(const double* P, int64_t m, int kc, double sf, double* mean, double* var,
                                 hipStream_t st) {
  predict_finish_kernel<<<(unsigned)((m + 3) / 4), 256, 0, st>>>(P, m, kc, sf, mean, var);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, int64_t count, hipStream_t st) {
  copy_kernel<<<blocks_for(count), kThreads, 0, st>>>(src, dst, count);
  return hipGetLastError();
}

hipError_t launch_zero_words(void* dst, int64_t words, hipStream_t st) {
  zero_words_kernel<<<blocks_for(words), kThreads, 0, st>>>((uint32_t*)dst, words);
  return hipGetLastError();
}

hipError_t launch_fill(double* dst, double v, int64_t count, hipStream_t st) {
  fill_kernel<<<blocks_for(count), kThreads, 0, st>>>(dst, v, count);
  return hipGetLastError();
}

hipError_t mbcg_launch_init(const MbcgState& s, hipStream_t st) {
  mbcg_init_kernel<<<1, 256, 0, st>>>(s);
  return hipGetLastError();
}
hipError_t mbcg_launch_alpha(const MbcgState& s, hipStream_t st) {
  mbcg_alpha_kernel<<<1, 256, 0, st>>>(s);
  return hipGetLastError();
}
hipError_t mbcg_launch_update_ur(const MbcgState& s, const double* D, const double* W, double* U, double* R,
                                 int64_t n, double* partial, hipStream_t st) {
  const RowSplit rs = row_split(n, kDotBlocks);
  mbcg_update_ur_kernel<<<dim3((unsigned)rs.nblk, (unsigned)s.s), kThreads, 0, st>>>(s, D, W, U, R, n,
                                                                                      rs.rows_per_blk, partial);
  reduce_partials_kernel<<<s.s, kThreads, 0, st>>>(partial, rs.nblk, s.s, s.rnorm2);
  return hipGetLastError();
}
hipError_t mbcg_launch_freeze(const MbcgState& s, int j, double tol, hipStream_t st) {
  mbcg_freeze_kernel<<<1, 256, 0, st>>>(s, j, tol);
  return hipGetLastError();
}
hipError_t mbcg_launch_beta(const MbcgState& s, hipStream_t st) {
  mbcg_beta_kernel<<<1, 256, 0, st>>>(s);
  return hipGetLastError();
}
hipError_t mbcg_launch_update_d(const MbcgState& s, const double* Z, double* D, int64_t n, hipStream_t st) {
  const RowSplit rs = row_split(n, kDotBlocks);
  mbcg_update_d_kernel<<<dim3((unsigned)rs.nblk, (unsigned)s.s), kThreads, 0, st>>>(s, Z, D, n, rs.rows_per_blk);
  return hipGetLastError();
}

hipError_t pivchol_launch_argmax(const double* delta, int64_t n, double* pval, int64_t* pidx, const PivState& ps,
                                 int m, double stop_below, hipStream_t st) {
  const RowSplit rs = row_split(n, kDotBlocks);
  argmax_partial_kernel<<<(unsigned)rs.nblk, kThreads, 0, st>>>(delta, n, rs.rows_per_blk, pval, pidx);
  argmax_final_kernel<<<1, kThreads, 0, st>>>(pval, pidx, rs.nblk, ps, m, stop_below);
  return hipGetLastError();
}

hipError_t pivchol_launch_column(const double* X, int64_t n, const gp_kernel* kern, double* L, double* delta,
                                 const PivState& ps, int m, hipStream_t st) {
  Scale inv{};
  for (int j = 0; j < kern->d; ++j) inv.s[j] = 1.0 / kern->lengthscale[j];
  pivchol_column_kernel<<<blocks_for(n), kThreads, 0, st>>>(X, n, kern->d, inv, kern->kind, kern->outputscale, L,
                                                            delta, ps, m);
  return hipGetLastError();
}

}  // namespace gpk

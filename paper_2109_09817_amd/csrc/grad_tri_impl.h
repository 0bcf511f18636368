// Kernel template of the upper-triangle hyperparameter-form sweep (see grad_tri.h)
// and its instantiation table; included by one translation unit per kernel kind.
#pragma once

#include "grad_tri.h"
#include "mfma_bf16.h"

namespace gpk {

// LDS image of one 32-point chunk, in 64-lane units of 16 bytes:
// [2 KS distance fragments | 2 KSC C fragments | 2 NJ (hi, lo) pairs of form fragments].
template <int KS, int KSC, int NJ>
struct TriChunk {
  static constexpr int kDist = 2 * KS * 64;
  static constexpr int kC = 2 * KSC * 64;
  static constexpr int kG = 2 * (2 * NJ) * 64;
  static constexpr int kAll = kDist + kC + kG;
};

template <int KS, int KSC, int NJ, int NA, int KIND>
__global__ __launch_bounds__(64 * kTriWaves, 2) void grad_tri_bf16x3_kernel(GradTriArgs a) {
  constexpr int NG = 2 * NJ;
  using TC = TriChunk<KS, KSC, NJ>;
  __shared__ bf16x8 stage[2][TC::kAll];
  static_assert(sizeof(stage) >= sizeof(double) * kTriWaves * (GP_MAX_D + 1), "reduction scratch");
  double(*red)[GP_MAX_D + 1] = reinterpret_cast<double(*)[GP_MAX_D + 1]>(&stage[0][0]);  // after the loop only
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 4;
  const int c16 = lane & 15;
  const int2 unit = a.units[blockIdx.x];
  const int64_t ablk0 = ((int64_t)unit.x * kTriWaves + wave) * NA;  // this wave's first 16-row block
  const int64_t c_begin = unit.y;
  const int64_t c_lim = (c_begin / a.cps + 1) * a.cps;
  const int64_t c_end = c_lim < a.nchunks ? c_lim : a.nchunks;

  bf16x8 A[NA][KS], CA[NA][KSC];
#pragma unroll
  for (int ab = 0; ab < NA; ++ab) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) A[ab][ks] = a.xc[((ablk0 + ab) * KS + ks) * 64 + lane];
#pragma unroll
    for (int q = 0; q < KSC; ++q) CA[ab][q] = a.ca[((ablk0 + ab) * KSC + q) * 64 + lane];
  }

  f32x4 acc[NA][NG];
  float racc[NA];
#pragma unroll
  for (int ab = 0; ab < NA; ++ab) {
    racc[ab] = 0.f;
#pragma unroll
    for (int nb = 0; nb < NG; ++nb) acc[ab][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  float sfacc = 0.f;  // Matern: sum of S e C^s over this wave's rows (in the wave's row scale)
  double g64[NJ];
#pragma unroll
  for (int cb = 0; cb < NJ; ++cb) g64[cb] = 0.0;
  double sf64 = 0.0;

  // Copy the chunks into stage[buf] with direct global-to-LDS loads: the 64-lane
  // units (16 bytes per lane, lane-contiguous in LDS) of each of the three
  // streams are dealt to the waves in turn (unit j of a stream to wave j mod 4),
  // so the source stream and LDS slot of every load are fixed at compile time
  // up to the wave index, which is held in a scalar register; the three stream
  // pointers start at chunk c_begin and advance by one chunk per fetch.
  // Completion is awaited (vmcnt) and published by the barrier that ends the
  // iteration.
  const int wu = __builtin_amdgcn_readfirstlane(wave);
  const int lofs = lane + 64 * wave;  // this lane's element of the wave's first unit
  const bf16x8* px = a.xr + c_begin * (2 * KS * 64);
  const bf16x8* pc = a.cb + c_begin * (2 * KSC * 64);
  const bf16x8* pg = a.gv + c_begin * (2 * NG * 64);
  auto load_stream = [&](const bf16x8* src, int units, int first, int buf) {
#pragma unroll
    for (int r = 0; r < (units + kTriWaves - 1) / kTriWaves; ++r) {
      const int j = wu + kTriWaves * r;  // unit of the stream
      if (j < units)
        __builtin_amdgcn_global_load_lds((const void*)(src + lofs + 64 * kTriWaves * r),
                                         (__attribute__((address_space(3))) void*)&stage[buf][first + 64 * j], 16, 0,
                                         0);
    }
  };
  auto fetch = [&](int buf) {
    load_stream(px, 2 * KS, 0, buf);
    load_stream(pc, 2 * KSC, TC::kDist, buf);
    load_stream(pg, 2 * NG, TC::kDist + TC::kC, buf);
    px += 2 * KS * 64;
    pc += 2 * KSC * 64;
    pg += 2 * NG * 64;
  };
  // Fold the FP32 window into the FP64 partials of g_j (j = 16 cb + c16).
  auto flush = [&]() {
    const double bi = a.grpinv[ablk0 / NA];  // 1 / s of this wave's 16 NA rows
    // the s_f form: sum k C^s = sum p + kMaternC2 sum S e C^s (Matern), sum p (RBF)
    double sfw = 0.0;
#pragma unroll
    for (int ab = 0; ab < NA; ++ab) sfw += (double)racc[ab];
    if constexpr (KIND == GP_MATERN52) sfw += (double)kMaternC2 * (double)sfacc;
    sf64 += sfw * bi;
    sfacc = 0.f;
#pragma unroll
    for (int ab = 0; ab < NA; ++ab) {
      const int64_t ar = (ablk0 + ab) * 16;
      float rf = racc[ab];  // row sums of P: lane holds row ar + c16 over 8 of the points
      rf += __shfl_xor(rf, 16, 64);
      rf += __shfl_xor(rf, 32, 64);
      double Ri[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) Ri[i] = (double)__shfl(rf, 4 * g + i, 64);
#pragma unroll
      for (int cb = 0; cb < NJ; ++cb) {
        const int j = 16 * cb + c16;
        if (j < a.d) {
          const double m = a.mu[j], s = a.inv_ell[j];
          const double qs = a.scal[2 * a.d + j], ts = a.scal[3 * a.d + j];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int64_t row = ar + 4 * g + i;
            if (row < a.n) {
              const double x = (a.X[row * a.d + j] - m) * s;
              g64[cb] += (x * x * Ri[i] - 2.0 * x * ((double)acc[ab][cb][i] * qs) + (double)acc[ab][NJ + cb][i] * ts) * bi;
            }
          }
        }
      }
      racc[ab] = 0.f;
#pragma unroll
      for (int nb = 0; nb < NG; ++nb) acc[ab][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };

  fetch(0);  // chunk c_begin
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int window = 0;
  for (int64_t ch = c_begin; ch < c_end; ++ch) {
    const int cur = (int)((ch - c_begin) & 1);
    const bool more = ch + 1 < c_end;
    if (more) fetch(cur ^ 1);  // chunk ch + 1
    const int64_t b0 = ch * 32;
    if (b0 + 31 > ablk0 * 16) {  // the first block's tile holds some pair b > a
      // A later block with no pair b > a in this chunk (only where the chunk meets
      // the wave's first rows) has all its pairs masked to zero below, so where
      // the C^s phase runs for both blocks at once every block's tiles are
      // computed and the MFMAs stay unconditional; the block-by-block form skips
      // such a block (unconditional, it spills).
      constexpr bool kJoint = tri_joint_c(KS, KSC, NJ);
      bool live[NA];
      f32x4 s0[NA], s1[NA];
#pragma unroll
      for (int ab = 0; ab < NA; ++ab) {
        live[ab] = kJoint || b0 + 31 > (ablk0 + ab) * 16;
        s0[ab] = f32x4{0.f, 0.f, 0.f, 0.f};
        s1[ab] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      // distance tiles of the NA blocks, one staged K step at a time (each LDS
      // read feeds NA MFMAs); the fragments of step ks + 1 are read while the
      // MFMAs of step ks run
      bf16x8 b0f = stage[cur][lane];
      bf16x8 b1f = stage[cur][KS * 64 + lane];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        bf16x8 n0f, n1f;
        if (ks + 1 < KS) {
          n0f = stage[cur][(ks + 1) * 64 + lane];
          n1f = stage[cur][(KS + ks + 1) * 64 + lane];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ab = 0; ab < NA; ++ab) {
          if (!live[ab]) continue;
          s0[ab] = mfma_dist(b0f, A[ab][ks], s0[ab]);
          s1[ab] = mfma_dist(b1f, A[ab][ks], s1[ab]);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (ks + 1 < KS) {
          b0f = n0f;
          b1f = n1f;
        }
      }
      // C^s tiles: both blocks one staged K step at a time, the next step's
      // fragments read while these MFMAs run, where the registers allow;
      // otherwise block by block (the fragments re-read per block)
      f32x4 q0a[NA], q1a[NA];
      if constexpr (kJoint) {
#pragma unroll
        for (int ab = 0; ab < NA; ++ab) {
          q0a[ab] = f32x4{0.f, 0.f, 0.f, 0.f};
          q1a[ab] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        bf16x8 c0f = stage[cur][TC::kDist + lane];
        bf16x8 c1f = stage[cur][TC::kDist + KSC * 64 + lane];
#pragma unroll
        for (int q = 0; q < KSC; ++q) {
          bf16x8 d0f, d1f;
          if (q + 1 < KSC) {
            d0f = stage[cur][TC::kDist + (q + 1) * 64 + lane];
            d1f = stage[cur][TC::kDist + (KSC + q + 1) * 64 + lane];
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int ab = 0; ab < NA; ++ab) {
              if (!live[ab]) continue;
            q0a[ab] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c0f, CA[ab][q], q0a[ab], 0, 0, 0);
            q1a[ab] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(c1f, CA[ab][q], q1a[ab], 0, 0, 0);
          }
          __builtin_amdgcn_sched_barrier(0);
          if (q + 1 < KSC) {
            c0f = d0f;
            c1f = d1f;
          }
        }
      }
      bf16x8 H[NA], L[NA];
#pragma unroll
      for (int ab = 0; ab < NA; ++ab) {
        const int64_t ar = (ablk0 + ab) * 16;
        if (!live[ab]) continue;
        f32x4 q0 = {0.f, 0.f, 0.f, 0.f}, q1 = {0.f, 0.f, 0.f, 0.f};
        if constexpr (kJoint) {
          q0 = q0a[ab];
          q1 = q1a[ab];
        } else {
#pragma unroll
          for (int q = 0; q < KSC; ++q) {
            q0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(stage[cur][TC::kDist + q * 64 + lane], CA[ab][q], q0, 0, 0, 0);
            q1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(stage[cur][TC::kDist + (KSC + q) * 64 + lane], CA[ab][q],
                                                         q1, 0, 0, 0);
          }
        }
        if (b0 < ar + 16) {  // meets or passes the block: keep b > a only
          // point b0 + k against row ar + c16, in 32-bit offsets from b0 (ar - b0 lies in
          // (-16, 16 NA + 15)); a block with b0 + 31 <= ar has every pair masked
          const int am = (int)(ar - b0) + c16;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if (4 * g + i <= am) q0[i] = 0.f;
            if (16 + 4 * g + i <= am) q1[i] = 0.f;
          }
        }
        f32x8 pv;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const float S = __builtin_fabsf(k < 4 ? s0[ab][k] : s1[ab][k - 4]);
          const float cs = k < 4 ? q0[k] : q1[k - 4];
          float p;  // psi C^s
          if constexpr (KIND == GP_MATERN52) {
            // psi = (1 + sqrt5 r) e^{-sqrt5 r} and k = psi + (5 r^2 / 3) e^{-sqrt5 r}, so that
            // k C^s = p + kMaternC2 S e C^s: the s_f sum keeps only S e C^s (added to the
            // row sums of p at the flush)
            const float u = __builtin_amdgcn_sqrtf(S);
            const float ec = __builtin_amdgcn_exp2f(-u) * cs;
            p = __builtin_fmaf(u, kMaternC1, 1.0f) * ec;
            sfacc = __builtin_fmaf(S, ec, sfacc);
          } else {
            p = __builtin_amdgcn_exp2f(-S) * cs;  // psi = k: the s_f sum is the row sums of p
          }
          pv[k] = p;
          racc[ab] += p;
        }
        split_f16x8(pv, H[ab], L[ab]);
      }
      bf16x8 Gh = stage[cur][TC::kDist + TC::kC + lane];
      bf16x8 Gl = stage[cur][TC::kDist + TC::kC + 64 + lane];
#pragma unroll
      for (int nb = 0; nb < NG; ++nb) {
        bf16x8 Nh, Nl;
        if (nb + 1 < NG) {
          Nh = stage[cur][TC::kDist + TC::kC + (2 * nb + 2) * 64 + lane];
          Nl = stage[cur][TC::kDist + TC::kC + (2 * nb + 3) * 64 + lane];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int ab = 0; ab < NA; ++ab) {
          if (!live[ab]) continue;
          acc[ab][nb] = mfma_val(H[ab], Gh, acc[ab][nb]);
          acc[ab][nb] = mfma_val(H[ab], Gl, acc[ab][nb]);
          acc[ab][nb] = mfma_val(L[ab], Gh, acc[ab][nb]);
        }
        __builtin_amdgcn_sched_barrier(0);
        if (nb + 1 < NG) {
          Gh = Nh;
          Gl = Nl;
        }
      }
    }
    if (++window == kTriFlush || !more) {
      flush();
      window = 0;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  // unit partial: sum over the rows of every wave, then over the waves
#pragma unroll
  for (int cb = 0; cb < NJ; ++cb) {
    double v = g64[cb];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (g == 0 && 16 * cb + c16 < a.d) red[wave][16 * cb + c16] = v;
  }
  double s = sf64;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) red[wave][a.d] = s;
  __syncthreads();
  if (tid <= a.d) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kTriWaves; ++w) t += red[w][tid];
    a.part[(int64_t)blockIdx.x * (a.d + 1) + tid] = t;
  }
}

template <int KS, int NJ, int KSC, int KIND>
static void tri_launch(unsigned units, const GradTriArgs& a, hipStream_t st) {
  constexpr int NA = tri_na(KS, KSC, NJ);
  grad_tri_bf16x3_kernel<KS, KSC, NJ, NA, KIND><<<units, 64 * kTriWaves, 0, st>>>(a);
}

template <int KS, int NJ, int KIND>
static bool tri_ksc(int ksc, unsigned units, const GradTriArgs& a, hipStream_t st) {
  switch (ksc) {
    case 1: tri_launch<KS, NJ, 1, KIND>(units, a, st); return true;
    case 2: tri_launch<KS, NJ, 2, KIND>(units, a, st); return true;
    case 3: tri_launch<KS, NJ, 3, KIND>(units, a, st); return true;
    case 4: tri_launch<KS, NJ, 4, KIND>(units, a, st); return true;
    case 6: tri_launch<KS, NJ, 6, KIND>(units, a, st); return true;
    case 8: tri_launch<KS, NJ, 8, KIND>(units, a, st); return true;
    case 12: tri_launch<KS, NJ, 12, KIND>(units, a, st); return true;
    default: return false;
  }
}

// (KS, NJ) pairs for d <= 64 (see tri_ks_of):
//   d <= 16: (2, 1)   d <= 32: (4, 2)   d <= 48: (5, 3)   d <= 64: (7, 4)
template <int KIND>
static bool tri_dispatch(int ks, int nj, int ksc, unsigned units, const GradTriArgs& a, hipStream_t st) {
  if (ks == 2 && nj == 1) return tri_ksc<2, 1, KIND>(ksc, units, a, st);
  if (ks == 4 && nj == 2) return tri_ksc<4, 2, KIND>(ksc, units, a, st);
  if (ks == 5 && nj == 3) return tri_ksc<5, 3, KIND>(ksc, units, a, st);
  if (ks == 7 && nj == 4) return tri_ksc<7, 4, KIND>(ksc, units, a, st);
  return false;
}

}  // namespace gpk

// Sampling, scaled gather and Householder QR of the sample (Algorithm
// rpCholesky-QR, lines 2-3), in one workgroup of 16 waves.
//
// Ownership: wave w owns the sample columns j = w, w+16, w+32, ...; lane l owns
// the sample rows r = l, l+64, l+128, ...  Every element of the working matrix
// is touched by exactly one thread, so only the Householder vector, tau and the
// R factor are shared (through LDS).
//
// Dot products over rows r >= k use the fixed order of lane_tree_sum: lane l
// accumulates its rows in ascending order with fma, then the 64 partials are
// combined pairwise.  With beta = -sign(alpha) * nu, d = 1/(alpha - beta),
// v = (1, y_1 d, ...), tau = (beta - alpha)/beta and the update
// w_r = fma(-tau*(v.w), v_r, w_r), this fixes every rounding of R_s.
#pragma once

#include "device_common.h"

namespace rpq {

constexpr int kSketchWaves = 16;
constexpr int kSketchThreads = kSketchWaves * kWave;
constexpr int kSketchMaxN = 64;  // R_s is staged in LDS as 64 x 65
constexpr int kSketchLdr = kSketchMaxN + 1;

struct SketchArgs {
  int64_t m;
  int32_t n, s;
  uint64_t seed;
  double scale;  // sqrt(m/s), correctly rounded on the host
  const double* A;
  int64_t lda;
  double* tri;    // out: packed R_s for the row solves (see Tri), nmax rows
  double* Rs;     // out: R_s, n x n column-major (ld n)
  int32_t nmax;
  int32_t* info;  // {code, index}
  double* W;      // global working copy of A_s (s x n, ld s), used by the generic kernel only
  int64_t* idx_out;  // optional
  double* As_out;    // optional, s x n, ld s
  double* Rs_out;    // optional, n x n, ld n
};

// Sign-normalize R_s (negate rows with a negative diagonal; exact) and write
// the packed triangle for the row solves, the column-major copy and the
// optional output.
__device__ __forceinline__ void sketch_finish(const SketchArgs& a, const double* Rl) {
  const int n = a.n, nmax = a.nmax;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e % n, j = e / n;
    double v = 0.0;
    if (i <= j) {
      v = Rl[i * kSketchLdr + j];
      if (Rl[i * kSketchLdr + i] < 0.0) v = -v;
    }
    a.Rs[e] = v;
    if (a.Rs_out) a.Rs_out[e] = v;
  }
  for (int e = threadIdx.x; e < nmax * nmax; e += blockDim.x) {
    const int k = e / nmax, j = e - k * nmax;
    if (j < k) continue;
    double v;
    if (k < n && j < n) {
      const double rkk = Rl[k * kSketchLdr + k];
      if (j == k) {
        v = 1.0 / (rkk < 0.0 ? -rkk : rkk);
      } else {
        v = Rl[k * kSketchLdr + j];
        if (rkk < 0.0) v = -v;
      }
    } else {
      v = (j == k) ? 1.0 : 0.0;
    }
    a.tri[tri_row_start(k, nmax) + (j - k)] = v;
  }
}

// Register-resident variant: each lane keeps CPW x RPL entries of A_s.
// Requires n <= 16*CPW <= 64 and s <= 64*RPL.
template <int CPW, int RPL>
__global__ __launch_bounds__(kSketchThreads) void k_sketch_reg(SketchArgs a) {
  __shared__ double vbuf[2][RPL * kWave];
  __shared__ double tau_s[2];
  __shared__ double Rl[kSketchMaxN * kSketchLdr];
  __shared__ int bad_k;

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6;
  const int n = a.n, s = a.s;

  for (int e = threadIdx.x; e < kSketchMaxN * kSketchLdr; e += kSketchThreads) Rl[e] = 0.0;
  if (threadIdx.x == 0) bad_k = -1;

  // Line 2: indices of my rows, then the scaled gather.
  int64_t rowidx[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int r = lane + kWave * t;
    rowidx[t] = (r < s) ? sample_index(a.seed, (uint64_t)r, (uint64_t)a.m) : 0;
    if (a.idx_out && wave == 0 && r < s) a.idx_out[r] = rowidx[t];
  }
  double W[CPW][RPL];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const int j = wave + kSketchWaves * c;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int r = lane + kWave * t;
      double v = 0.0;
      if (j < n && r < s) {
        v = a.scale * a.A[rowidx[t] + (int64_t)j * a.lda];
        if (a.As_out) a.As_out[r + (int64_t)j * s] = v;
      }
      W[c][t] = v;
    }
  }
  __syncthreads();

  // Line 3: Householder QR, R only.
  for (int k = 0; k < n; ++k) {
    const int owner = k & (kSketchWaves - 1), kc = k >> 4, kt = k >> 6, kl = k & (kWave - 1);
    const int buf = k & 1;
    if (wave == owner) {
      double col[RPL];
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        double v = W[0][t];
#pragma unroll
        for (int c = 1; c < CPW; ++c)
          if (c == kc) v = W[c][t];
        col[t] = v;
      }
      double p = 0.0;
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = lane + kWave * t;
        if (r >= k && r < s) p = __builtin_fma(col[t], col[t], p);
      }
      const double nu2 = lane_tree_sum(p);
      double ak = col[0];
#pragma unroll
      for (int t = 1; t < RPL; ++t)
        if (t == kt) ak = col[t];
      const double alpha = __shfl(ak, kl, kWave);
      if (nu2 == 0.0 || !__builtin_isfinite(nu2)) {
        if (lane == 0) bad_k = k;
      } else {
        const double nu = __builtin_sqrt(nu2);
        const double beta = (alpha >= 0.0) ? -nu : nu;
        const double d = 1.0 / (alpha - beta);
        const double tau = (beta - alpha) / beta;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int r = lane + kWave * t;
          if (r >= k && r < s) vbuf[buf][r] = (r == k) ? 1.0 : col[t] * d;
        }
        if (lane == 0) {
          tau_s[buf] = tau;
          Rl[k * kSketchLdr + k] = beta;
        }
      }
    }
    __syncthreads();
    if (bad_k >= 0) break;
    const double tau = tau_s[buf];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const int j = wave + kSketchWaves * c;
      if (j > k && j < n) {
        double p = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int r = lane + kWave * t;
          if (r >= k && r < s) p = __builtin_fma(vbuf[buf][r], W[c][t], p);
        }
        const double tt = tau * lane_tree_sum(p);
        double rk = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          const int r = lane + kWave * t;
          if (r >= k && r < s) W[c][t] = __builtin_fma(-tt, vbuf[buf][r], W[c][t]);
          if (t == kt) rk = W[c][t];
        }
        if (lane == kl) Rl[k * kSketchLdr + j] = rk;
      }
    }
  }
  __syncthreads();
  if (bad_k >= 0) {
    if (threadIdx.x == 0) {
      a.info[0] = 1;
      a.info[1] = bad_k;
    }
    return;
  }
  if (threadIdx.x == 0) {
    a.info[0] = 0;
    a.info[1] = -1;
  }
  sketch_finish(a, Rl);
}

// Generic variant: the working copy of A_s lives in global memory (a.W, s x n,
// ld s); the Householder vector in dynamic LDS (2*s doubles).  Same ownership
// and the same operation order as k_sketch_reg.  Requires n <= 64.
__global__ __launch_bounds__(kSketchThreads) void k_sketch_global(SketchArgs a) {
  extern __shared__ double vdyn[];  // [2][s]
  __shared__ double tau_s[2];
  __shared__ double Rl[kSketchMaxN * kSketchLdr];
  __shared__ int bad_k;

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x >> 6;
  const int n = a.n, s = a.s;
  double* W = a.W;

  for (int e = threadIdx.x; e < kSketchMaxN * kSketchLdr; e += kSketchThreads) Rl[e] = 0.0;
  if (threadIdx.x == 0) bad_k = -1;
  for (int r = lane; r < s; r += kWave) {
    const int64_t ir = sample_index(a.seed, (uint64_t)r, (uint64_t)a.m);
    if (a.idx_out && wave == 0) a.idx_out[r] = ir;
    for (int j = wave; j < n; j += kSketchWaves) {
      const double v = a.scale * a.A[ir + (int64_t)j * a.lda];
      W[r + (int64_t)j * s] = v;
      if (a.As_out) a.As_out[r + (int64_t)j * s] = v;
    }
  }
  __syncthreads();

  for (int k = 0; k < n; ++k) {
    const int owner = k & (kSketchWaves - 1);
    const int buf = k & 1;
    double* vb = vdyn + (size_t)buf * s;
    if (wave == owner) {
      const double* col = W + (int64_t)k * s;
      double p = 0.0;
      for (int r = lane; r < s; r += kWave)
        if (r >= k) p = __builtin_fma(col[r], col[r], p);
      const double nu2 = lane_tree_sum(p);
      const double alpha = col[k];
      if (nu2 == 0.0 || !__builtin_isfinite(nu2)) {
        if (lane == 0) bad_k = k;
      } else {
        const double nu = __builtin_sqrt(nu2);
        const double beta = (alpha >= 0.0) ? -nu : nu;
        const double d = 1.0 / (alpha - beta);
        const double tau = (beta - alpha) / beta;
        for (int r = lane; r < s; r += kWave)
          if (r >= k) vb[r] = (r == k) ? 1.0 : col[r] * d;
        if (lane == 0) {
          tau_s[buf] = tau;
          Rl[k * kSketchLdr + k] = beta;
        }
      }
    }
    __syncthreads();
    if (bad_k >= 0) break;
    const double tau = tau_s[buf];
    for (int j = wave; j < n; j += kSketchWaves) {
      if (j <= k) continue;
      double* wj = W + (int64_t)j * s;
      double p = 0.0;
      for (int r = lane; r < s; r += kWave)
        if (r >= k) p = __builtin_fma(vb[r], wj[r], p);
      const double tt = tau * lane_tree_sum(p);
      for (int r = lane; r < s; r += kWave)
        if (r >= k) wj[r] = __builtin_fma(-tt, vb[r], wj[r]);
      if (lane == (k & (kWave - 1))) Rl[k * kSketchLdr + j] = wj[k];
    }
  }
  __syncthreads();
  if (bad_k >= 0) {
    if (threadIdx.x == 0) {
      a.info[0] = 1;
      a.info[1] = bad_k;
    }
    return;
  }
  if (threadIdx.x == 0) {
    a.info[0] = 0;
    a.info[1] = -1;
  }
  sketch_finish(a, Rl);
}

}  // namespace rpq

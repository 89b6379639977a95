// The n x n steps between the passes (Algorithm Preconditioned Cholesky-QR,
// lines 4-5 and 8): fixed-order reduction of the per-workgroup partial Gram
// matrices, Cholesky G1 = R2^T R2, and R = R2 R_s.
#pragma once

#include "device_common.h"

namespace rpq {

constexpr int kReduceThreads = 256;
constexpr int kReduceChunk = 64;  // partials summed per thread in the first level
constexpr int kMaxPartial2 = 8;   // second-level partials (first-level chunks) at most
constexpr int kCholThreads = 256;
constexpr int kCholMaxN = 64;
constexpr int kCholLdg = kCholMaxN + 1;

// First level: partial2[g][e] = sum of partials[p][e] over p in chunk g, in
// ascending p.  Grid: (ceil(E/256), ceil(P/kReduceChunk)).
__global__ __launch_bounds__(kReduceThreads) void k_reduce_partials(const double* __restrict__ partials,
                                                                    int P, int E,
                                                                    double* __restrict__ partial2,
                                                                    const int32_t* __restrict__ info) {
  if (info[0] != 0) return;
  const int e = blockIdx.x * kReduceThreads + threadIdx.x;
  if (e >= E) return;
  const int p0 = blockIdx.y * kReduceChunk;
  const int cnt = min(P - p0, kReduceChunk);
  // All loads first (independent), then the sum in ascending p.
  double v[kReduceChunk];
#pragma unroll
  for (int q = 0; q < kReduceChunk; ++q) v[q] = (q < cnt) ? partials[(int64_t)(p0 + q) * E + e] : 0.0;
  double acc = v[0];
#pragma unroll
  for (int q = 1; q < kReduceChunk; ++q)
    if (q < cnt) acc = acc + v[q];
  partial2[(int64_t)blockIdx.y * E + e] = acc;
}

struct CholArgs {
  const double* partial2;  // [G2][E]
  int32_t G2, E, NB;       // number of second-level partials, doubles per Gram, 16-blocks
  int32_t n, nmax;
  const double* Rs;     // R_s, n x n column-major
  double* T2;           // out: R2^{-1}, nmax x nmax row-major, zero outside the n x n upper triangle
  double* R;            // out: n x n, ld ldr
  int64_t ldr;
  int32_t* info;
  double* G1_out;       // optional n x n, ld n (upper triangle)
  double* R2_out;       // optional n x n, ld n
};

// One workgroup.  The second-level partials are summed by all threads; the
// Cholesky factorization runs in wave 0 with lane j holding column j of G1 in
// registers (right-looking: at step k the pivot row is scaled by 1/sqrt(G(k,k))
// and broadcast through LDS, then every lane j updates G(i,j) -= R(k,i) R(k,j)
// for i > k).  A non-positive or non-finite pivot gives ECHOL(k).
__global__ __launch_bounds__(kCholThreads) void k_cholesky(CholArgs a) {
  __shared__ double G[kCholMaxN * kCholLdg];
  __shared__ double Rs_l[kCholMaxN * kCholLdg];  // R_s row-major
  __shared__ double rowk[2][kCholMaxN];
  __shared__ int bad_s;
  if (a.info[0] != 0) return;
  const int n = a.n, tid = threadIdx.x;
  if (tid == 0) bad_s = -1;

  // Stage R_s for the R product and assemble G1 from the second-level
  // partials (independent loads first, then the sum in ascending g).
  for (int e = tid; e < n * n; e += kCholThreads) Rs_l[(e % n) * kCholLdg + e / n] = a.Rs[e];
  constexpr int kEntries = 4;  // entries per thread per round: all their loads in flight together
  for (int e0 = tid; e0 < a.E; e0 += kEntries * kCholThreads) {
    double v[kEntries][kMaxPartial2];
#pragma unroll
    for (int u = 0; u < kEntries; ++u) {
      const int e = e0 + u * kCholThreads;
#pragma unroll
      for (int g = 0; g < kMaxPartial2; ++g)
        v[u][g] = (e < a.E && g < a.G2) ? a.partial2[(int64_t)g * a.E + e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kEntries; ++u) {
      const int e = e0 + u * kCholThreads;
      if (e >= a.E) break;
      const int tile = e >> 8, w = e & 255;
      int bi = 0, rem = tile;
      while (rem >= a.NB - bi) {
        rem -= a.NB - bi;
        ++bi;
      }
      const int bj = bi + rem;
      const int i = 16 * bi + (w >> 4), j = 16 * bj + (w & 15);
      double acc = v[u][0];
#pragma unroll
      for (int g = 1; g < kMaxPartial2; ++g)
        if (g < a.G2) acc = acc + v[u][g];
      if (i <= j && j < n) G[i * kCholLdg + j] = acc;
    }
  }
  __syncthreads();
  if (a.G1_out) {
    for (int e = tid; e < n * n; e += kCholThreads) {
      const int i = e % n, j = e / n;
      a.G1_out[e] = (i <= j) ? G[i * kCholLdg + j] : 0.0;
    }
  }

  if (tid < kWave) {
    const int lane = tid;
    double g[kCholMaxN];
#pragma unroll
    for (int i = 0; i < kCholMaxN; ++i) g[i] = (i <= lane && lane < n) ? G[i * kCholLdg + lane] : 0.0;
    int bad = -1;
#pragma unroll
    for (int k = 0; k < kCholMaxN; ++k) {
      if (k >= n || bad >= 0) break;
      const double d = readlane_d(g[k], k);
      if (!(d > 0.0) || !__builtin_isfinite(d)) {
        bad = k;
        break;
      }
      const double rkk = __builtin_sqrt(d);
      const double rinv = 1.0 / rkk;
      g[k] = (lane == k) ? rkk : g[k] * rinv;
      // Row k of R2 to every lane through LDS (two buffers: the next step's
      // write cannot overtake this step's reads of the same address).
      rowk[k & 1][lane] = g[k];
#pragma unroll
      for (int i = k + 1; i < kCholMaxN; ++i) g[i] = __builtin_fma(-rowk[k & 1][i], g[k], g[i]);
    }
    // Write R2 back into G's upper triangle (lane j owns column j).
    if (lane < n) {
#pragma unroll
      for (int i = 0; i < kCholMaxN; ++i)
        if (i <= lane) G[i * kCholLdg + lane] = g[i];
    }
    if (lane == 0) bad_s = bad;
  }
  __syncthreads();
  if (bad_s >= 0) {
    if (tid == 0) {
      a.info[0] = 2;
      a.info[1] = bad_s;
    }
    return;
  }

  if (a.R2_out) {
    for (int e = tid; e < n * n; e += kCholThreads) {
      const int i = e % n, j = e / n;
      a.R2_out[e] = (i <= j) ? G[i * kCholLdg + j] : 0.0;
    }
  }

  // T2 = R2^{-1} for pass B: lane i of wave 0 solves x R2 = e_i (row i of T2)
  // with the row-wise substitution; R2 is read from LDS (broadcast).
  const int nmax = a.nmax;
  if (tid < kWave) {
    const int lane = tid;
    double x[kCholMaxN];
#pragma unroll
    for (int k = 0; k < kCholMaxN; ++k) x[k] = (k == lane) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < kCholMaxN; ++k) {
      if (k < n) {
        x[k] = x[k] / G[k * kCholLdg + k];
#pragma unroll
        for (int j = k + 1; j < kCholMaxN; ++j)
          if (j < n) x[j] = __builtin_fma(-x[k], G[k * kCholLdg + j], x[j]);
      }
    }
    if (lane < nmax) {
#pragma unroll
      for (int j = 0; j < kCholMaxN; ++j)
        if (j < nmax) a.T2[lane * nmax + j] = (lane < n && j < n && j >= lane) ? x[j] : 0.0;
    }
  }

  // Line 8: R = R2 R_s (upper times upper).  Consecutive threads take
  // consecutive j (R_s row reads are contiguous, R2 reads are broadcasts); four
  // partial sums per entry.
  for (int e = tid; e < n * n; e += kCholThreads) {
    const int j = e % n, i = e / n;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (i <= j) {
      for (int k0 = i; k0 <= j; k0 += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = k0 + u;
          if (k <= j) acc[u] = __builtin_fma(G[i * kCholLdg + k], Rs_l[k * kCholLdg + j], acc[u]);
        }
      }
    }
    a.R[i + (int64_t)j * a.ldr] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  }
}

}  // namespace rpq

// The n x n steps between the passes (Algorithm Preconditioned Cholesky-QR,
// lines 4-5 and 8): fixed-order reduction of the per-workgroup partial Gram
// matrices, Cholesky G1 = R2^T R2, and R = R2 R_s.
#pragma once

#include "device_common.h"

namespace rpq {

constexpr int kReduceThreads = 256;
constexpr int kReduceChunk = 32;  // partials summed per thread in the first level
constexpr int kCholThreads = 1024;
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
  const int p1 = min(P, p0 + kReduceChunk);
  double acc = 0.0;
  for (int p = p0; p < p1; ++p) acc = acc + partials[(int64_t)p * E + e];
  partial2[(int64_t)blockIdx.y * E + e] = acc;
}

struct CholArgs {
  const double* partial2;  // [G2][E]
  int32_t G2, E, NB;       // number of second-level partials, doubles per Gram, 16-blocks
  int32_t n, nmax;
  const double* Rs;     // R_s, n x n column-major
  double* tri2;         // out: packed R2 for the row solves (see Tri)
  double* R;            // out: n x n, ld ldr
  int64_t ldr;
  int32_t* info;
  double* G1_out;       // optional n x n, ld n (upper triangle)
  double* R2_out;       // optional n x n, ld n
};

// One workgroup.  Right-looking Cholesky on the LDS copy of G1: at step k the
// pivot row is scaled by 1/sqrt(G(k,k)) and the trailing upper triangle gets
// G(i,j) -= R(k,i) R(k,j).  Non-positive or non-finite pivot -> ECHOL(k).
__global__ __launch_bounds__(kCholThreads) void k_cholesky(CholArgs a) {
  __shared__ double G[kCholMaxN * kCholLdg];
  if (a.info[0] != 0) return;
  const int n = a.n, tid = threadIdx.x;

  // Assemble G1 from the second-level partials (ascending g).
  for (int e = tid; e < a.E; e += kCholThreads) {
    const int tile = e >> 8, w = e & 255;
    int bi = 0, rem = tile;
    while (rem >= a.NB - bi) {
      rem -= a.NB - bi;
      ++bi;
    }
    const int bj = bi + rem;
    const int i = 16 * bi + (w >> 4), j = 16 * bj + (w & 15);
    if (i <= j && j < n) {
      double acc = 0.0;
      for (int g = 0; g < a.G2; ++g) acc = acc + a.partial2[(int64_t)g * a.E + e];
      G[i * kCholLdg + j] = acc;
    }
  }
  __syncthreads();
  if (a.G1_out) {
    for (int e = tid; e < n * n; e += kCholThreads) {
      const int i = e % n, j = e / n;
      a.G1_out[e] = (i <= j) ? G[i * kCholLdg + j] : 0.0;
    }
  }
  __syncthreads();

  int bad = -1;
  for (int k = 0; k < n; ++k) {
    const double d = G[k * kCholLdg + k];
    if (!(d > 0.0) || !__builtin_isfinite(d)) {
      bad = k;
      break;
    }
    const double rkk = __builtin_sqrt(d);
    __syncthreads();  // everyone has read G(k,k)
    for (int j = k + tid; j < n; j += kCholThreads)
      G[k * kCholLdg + j] = (j == k) ? rkk : G[k * kCholLdg + j] / rkk;
    __syncthreads();
    const int w = n - k - 1;
    for (int e = tid; e < w * w; e += kCholThreads) {
      const int i = k + 1 + e / w, j = k + 1 + e % w;
      if (i <= j) G[i * kCholLdg + j] = __builtin_fma(-G[k * kCholLdg + i], G[k * kCholLdg + j], G[i * kCholLdg + j]);
    }
    __syncthreads();
  }
  if (bad >= 0) {
    if (tid == 0) {
      a.info[0] = 2;
      a.info[1] = bad;
    }
    return;
  }

  // R2 for pass B (packed, identity padding) and the optional copy.
  const int nmax = a.nmax;
  for (int e = tid; e < nmax * nmax; e += kCholThreads) {
    const int k = e / nmax, j = e - k * nmax;
    if (j < k) continue;
    double v;
    if (k < n && j < n)
      v = (j == k) ? 1.0 / G[k * kCholLdg + k] : G[k * kCholLdg + j];
    else
      v = (j == k) ? 1.0 : 0.0;
    a.tri2[tri_row_start(k, nmax) + (j - k)] = v;
  }
  if (a.R2_out) {
    for (int e = tid; e < n * n; e += kCholThreads) {
      const int i = e % n, j = e / n;
      a.R2_out[e] = (i <= j) ? G[i * kCholLdg + j] : 0.0;
    }
  }

  // Line 8: R = R2 R_s (upper times upper).
  for (int e = tid; e < n * n; e += kCholThreads) {
    const int i = e % n, j = e / n;
    double acc = 0.0;
    if (i <= j)
      for (int k = i; k <= j; ++k) acc = __builtin_fma(G[i * kCholLdg + k], a.Rs[k + (int64_t)j * n], acc);
    a.R[i + (int64_t)j * a.ldr] = acc;
  }
}

}  // namespace rpq

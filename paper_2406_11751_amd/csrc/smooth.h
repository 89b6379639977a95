// Smoothed sample (Algorithm rpCholesky-QR line 2 with F = F_T D: the remark
// after Theorem t_prob lets F_T be a Walsh-Hadamard transform and D a diagonal
// of independent random signs).  A is taken as padded with zero rows to
// M = 2^p >= m, its row i moved to position pi(i) by a fixed bit-scrambling
// permutation (scramble) and multiplied by D_i; only the s sampled rows of the
// Hadamard transform of that are formed:
//   A_s(r, j) = T(r, j) * (1 / sqrt(s)),
//   T(r, j)   = sum_{i < m} D_i (-1)^popcount(idx_r AND pi(i)) A(i, j),
// idx_r uniform on [0, M).  (Without the permutation, rows k and k' of the
// transform agree when k = k' mod 2^q and A lives in its first 2^q rows, and
// the sample of such a coherent matrix is singular.)  Every term is an exact
// signed copy of A(i, j), and the order of the sum is fixed (rows in chunks of
// smooth_chunk_rows(m); an fma chain in ascending i within a chunk; chunk sums
// added in ascending order), so the sample is reproducible to the bit.
//
// k_smooth_partials: workgroup (chunk, column block cb, row-block group) forms
//   the chunk sums of 16 columns for up to 32 blocks of 16 sampled rows on
//   MFMA: the A operand is the sign S(r, i) (computed per lane), the B operand
//   A(i, 16 cb + ..) staged in LDS 32 rows at a time; v_mfma_f64_16x16x4f64
//   adds its four products in ascending i as an fma chain onto the
//   accumulator, so each output is the chunk's fma chain in ascending i.
// k_smooth_finish: T = chunk sums added in ascending order, A_s = T / sqrt(s).
#pragma once

#include "sketch.h"

namespace rpq {

constexpr uint64_t kSignSalt = 0x5851f42d4c957f2dull;
constexpr int64_t kSmoothBlock = 4096;
constexpr int kSmoothRows = 32;    // rows staged in LDS per step
constexpr int kSmoothTPW = 8;      // 16-row output blocks per wave
constexpr int kSmoothThreads = 256;

__host__ __device__ inline int64_t smooth_padded_rows(int64_t m) {
  int64_t M = 1;
  while (M < m) M <<= 1;
  return M;
}

__host__ __device__ inline int64_t smooth_chunk_rows(int64_t m) {
  const int64_t blocks = (m + kSmoothBlock - 1) / kSmoothBlock;
  int64_t g = (blocks + 255) / 256;
  return (g < 1 ? 1 : g) * kSmoothBlock;
}

// pi(i) on [0, M), M = 2^p: multiply by an odd constant, xorshift by
// h = max(1, p/2), multiply, xorshift, all mod M (each step a bijection).
__host__ __device__ inline uint64_t scramble(uint64_t i, int64_t M) {
  const uint64_t mask = (uint64_t)M - 1u;
  int p = 0;
  while (((int64_t)1 << p) < M) ++p;
  const int h = p / 2 > 1 ? p / 2 : 1;
  uint64_t x = (i * 0x9e3779b97f4a7c15ull) & mask;
  x ^= x >> h;
  x = (x * 0xbf58476d1ce4e5b9ull) & mask;
  x ^= x >> h;
  return x;
}

// Random sign D_i: bit 63 of SplitMix64 output i seeded with seed XOR kSignSalt.
__device__ __forceinline__ double rademacher(uint64_t seed, int64_t i) {
  return (splitmix64_at(seed ^ kSignSalt, (uint64_t)i) >> 63) ? -1.0 : 1.0;
}

struct SmoothArgs {
  int64_t m;
  int32_t n, s;
  uint64_t seed;
  int64_t M, chunk;      // padded rows, rows per chunk
  int32_t nchunks;
  double scale;          // 1 / sqrt(s), correctly rounded on the host
  const double* A;
  int64_t lda;
  double* partials;      // [nchunks][n][s]
  double* As;            // out: s x n, ld s
  int64_t* idx_out;      // optional
  double* As_out;        // optional
};

__global__ __launch_bounds__(kSmoothThreads) void k_smooth_partials(SmoothArgs a) {
  __shared__ double xs[kSmoothRows][16 + 1];
  __shared__ double ds[kSmoothRows];
  __shared__ uint64_t ps[kSmoothRows];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  const int chunk = blockIdx.x, cb = blockIdx.y;
  const int rb0 = (blockIdx.z * kPassWaves + wave) * kSmoothTPW;  // first 16-row block of this wave
  const int64_t i0 = (int64_t)chunk * a.chunk;
  const int64_t i1 = i0 + a.chunk < a.m ? i0 + a.chunk : a.m;
  // sampled index of output row 16 rb + i16 for each of the wave's blocks
  uint64_t idx[kSmoothTPW];
#pragma unroll
  for (int t = 0; t < kSmoothTPW; ++t) {
    const int r = 16 * (rb0 + t) + i16;
    idx[t] = (r < a.s) ? (uint64_t)sample_index(a.seed, (uint64_t)r, (uint64_t)a.M) : 0;
  }
  d4 acc[kSmoothTPW];
#pragma unroll
  for (int t = 0; t < kSmoothTPW; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t r0 = i0; r0 < i1; r0 += kSmoothRows) {
    __syncthreads();
    // stage rows r0 .. r0+31 of columns 16 cb .. 16 cb + 15 (zero past m or n) and their signs
    for (int e = threadIdx.x; e < kSmoothRows * 16; e += kSmoothThreads) {
      const int rr = e % kSmoothRows, cc = e / kSmoothRows;
      const int64_t row = r0 + rr;
      const int col = 16 * cb + cc;
      xs[rr][cc] = (row < i1 && col < a.n) ? a.A[row + (int64_t)col * a.lda] : 0.0;
    }
    if (threadIdx.x < kSmoothRows) {
      const int64_t row = r0 + threadIdx.x;
      ds[threadIdx.x] = (row < i1) ? rademacher(a.seed, row) : 0.0;
      ps[threadIdx.x] = scramble((uint64_t)row, a.M);
    }
    __syncthreads();
#pragma unroll
    for (int kc = 0; kc < kSmoothRows / 4; ++kc) {
      const int kr = 4 * kc + g4;
      const uint64_t pi = ps[kr];
      const double b = xs[kr][i16];       // B(k, j) = A(i, 16 cb + j)
      const double d = ds[kr];
#pragma unroll
      for (int t = 0; t < kSmoothTPW; ++t) {
        // A(r, k) = D_i (-1)^popcount(idx_r AND pi(i)); zero past m (d = 0)
        const double sg = (__builtin_popcountll(idx[t] & pi) & 1) ? -d : d;
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(sg, b, acc[t], 0, 0, 0);
      }
    }
  }
  // result (r, j) of a block: lane j + 16 (r mod 4), register r / 4
  double* out = a.partials + (int64_t)chunk * a.n * a.s;
#pragma unroll
  for (int t = 0; t < kSmoothTPW; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * (rb0 + t) + g4 + 4 * v, j = 16 * cb + i16;
      if (r < a.s && j < a.n) out[(int64_t)j * a.s + r] = acc[t][v];
    }
}

__global__ __launch_bounds__(kSmoothThreads) void k_smooth_finish(SmoothArgs a) {
  const int64_t e = (int64_t)blockIdx.x * kSmoothThreads + threadIdx.x;
  const int64_t total = (int64_t)a.s * a.n;
  if (e >= total) return;
  double T = a.partials[e];
  for (int c = 1; c < a.nchunks; ++c) T = T + a.partials[(int64_t)c * total + e];
  const double v = T * a.scale;
  a.As[e] = v;
  if (a.As_out) a.As_out[e] = v;
  if (a.idx_out && e < a.s) a.idx_out[e] = sample_index(a.seed, (uint64_t)e, (uint64_t)a.M);
}

}  // namespace rpq

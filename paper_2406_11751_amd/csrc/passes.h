// The two streaming passes over A (Algorithm Preconditioned Cholesky-QR,
// lines 2, 4 and 6), FP64.
//
// Layout: one lane per row.  A wave takes a panel of 64 consecutive rows; for
// each column j the 64 lanes load 64 consecutive doubles of column-major A
// (one 512-byte coalesced load).  The row then lives in NMAX registers.
//
// pass A: A1 row = A row * R_s^{-1} (trsm_row), then the wave adds the panel's
//         contribution A1_p^T A1_p to its Gram accumulator: the panel is
//         transposed through LDS and contracted over rows with
//         v_mfma_f64_16x16x4f64 on the upper 16x16 block tiles.  At the end the
//         four waves of a workgroup are summed in fixed order into one partial
//         Gram per workgroup (upper block tiles, 256 doubles each).
// pass B: recomputes the same A1 row with the same trsm_row code (so the bits
//         equal those whose Gram was formed), solves with R2 and writes Q.
//
// The packed triangles (R_s, R2) are read through the scalar memory path (see
// trsm_row).  A workgroup's waves take panel groups in lock step (every wave
// runs the same number of iterations; rows past m are masked), so the barriers
// inside trsm_row are reached by all of them.
#pragma once

#include "device_common.h"

namespace rpq {

constexpr int kPassThreads = 256;
constexpr int kPassWaves = kPassThreads / kWave;
constexpr int kTriGroup = 16;  // triangle values per pipelined group in trsm_row
constexpr int kTriSync = 8;    // groups between workgroup barriers in trsm_row

template <int NMAX>
struct GramShape {
  static constexpr int NB = (NMAX + 15) / 16;    // 16-wide column blocks
  static constexpr int NT = NB * (NB + 1) / 2;    // upper block tiles
  static constexpr int E = NT * 256;              // doubles per partial Gram
};

template <int NMAX>
__device__ __forceinline__ void load_row(double (&t)[NMAX], const double* __restrict__ arow, int64_t lda,
                                         int n, bool valid) {
#pragma unroll
  for (int j = 0; j < NMAX; ++j) t[j] = (valid && j < n) ? arow[(int64_t)j * lda] : 0.0;
}

struct PassAArgs {
  int64_t m;
  int32_t n;
  const double* A;
  int64_t lda;
  const double* tri_s;  // packed R_s (see Tri)
  double* partials;     // [gridDim.x][E]
  const int32_t* info;
  double* A1;           // optional m x n, ld m
};

// Final cross-wave sum: each wave stored its tiles in LDS red[wave][E].
template <int E>
__device__ __forceinline__ void sum_waves_to_partial(const double* red, double* __restrict__ out) {
  for (int e = threadIdx.x; e < E; e += kPassThreads) {
    double v = red[e];
#pragma unroll
    for (int w = 1; w < kPassWaves; ++w) v = v + red[w * E + e];
    out[(int64_t)blockIdx.x * E + e] = v;
  }
}

template <int NMAX>
__device__ __forceinline__ void store_a1(const PassAArgs& a, const double (&t)[NMAX], int64_t r, bool valid) {
  if (a.A1 && valid) {
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
      if (j < a.n) a.A1[r + (int64_t)j * a.m] = t[j];
  }
}

// pass A (NMAX a multiple of 16, <= 64).
// LDS per wave: a half panel (32 rows) of A1, row stride NMAX+1 doubles.
template <int NMAX>
__global__ __launch_bounds__(kPassThreads, 2) void k_passA_mfma(PassAArgs a) {
  static_assert(NMAX % 16 == 0 && NMAX <= 64, "MFMA Gram tiles");
  constexpr int NB = GramShape<NMAX>::NB, NT = GramShape<NMAX>::NT, E = GramShape<NMAX>::E;
  constexpr int LDX = NMAX + 1;
  constexpr int XS = 32 * LDX;  // doubles per wave
  constexpr int LDS_D = (kPassWaves * XS > kPassWaves * E) ? kPassWaves * XS : kPassWaves * E;
  __shared__ double lds[LDS_D];
  if (a.info[0] != 0) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  double* xs = lds + wave * XS;
  const int64_t panels = (a.m + kWave - 1) / kWave;
  d4 acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
  const int half_row = lane & 31;
  const int rq = lane >> 4, cq = lane & 15;  // MFMA operand position
  const int64_t pgroups = (panels + kPassWaves - 1) / kPassWaves;
  for (int64_t pg = blockIdx.x; pg < pgroups; pg += gridDim.x) {
    const int64_t r = (pg * kPassWaves + wave) * kWave + lane;
    const bool valid = r < a.m;
    double t[NMAX];
    load_row<NMAX>(t, a.A + r, a.lda, a.n, valid);
    pin_values(t);
    trsm_row<NMAX, kTriGroup, kTriSync>(t, opaque(as_const(a.tri_s)));
    pin_values(t);
    if (!valid) {
#pragma unroll
      for (int j = 0; j < NMAX; ++j) t[j] = 0.0;
    }
    store_a1<NMAX>(a, t, r, valid);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      wave_lds_fence();
      if ((lane >> 5) == h) {
#pragma unroll
        for (int j = 0; j < NMAX; ++j) xs[half_row * LDX + j] = t[j];
      }
      wave_lds_fence();
#pragma unroll
      for (int q = 0; q < 8; ++q) {  // 4-row chunks of the half panel
        double v[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) v[b] = xs[(4 * q + rq) * LDX + 16 * b + cq];
        int tt = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi)
#pragma unroll
          for (int bj = bi; bj < NB; ++bj) {
            acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[bi], v[bj], acc[tt], 0, 0, 0);
            ++tt;
          }
      }
    }
  }
  __syncthreads();
  // D(i, j) of a 16x16 f64 MFMA tile sits in lane j + 16*(i%4), register i/4.
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = (lane >> 4) + 4 * v, j = lane & 15;
      lds[wave * E + q * 256 + i * 16 + j] = acc[q][v];
    }
  __syncthreads();
  sum_waves_to_partial<E>(lds, a.partials);
}

struct PassBArgs {
  int64_t m;
  int32_t n;
  const double* A;
  int64_t lda;
  const double* tri_s;  // packed R_s
  const double* tri_2;  // packed R2
  double* Q;
  int64_t ldq;
  const int32_t* info;
};

template <int NMAX>
__global__ __launch_bounds__(kPassThreads) void k_passB(PassBArgs a) {
  if (a.info[0] != 0) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int64_t panels = (a.m + kWave - 1) / kWave;
  const int64_t pgroups = (panels + kPassWaves - 1) / kPassWaves;
  for (int64_t pg = blockIdx.x; pg < pgroups; pg += gridDim.x) {
    const int64_t r = (pg * kPassWaves + wave) * kWave + lane;
    const bool valid = r < a.m;
    double t[NMAX];
    load_row<NMAX>(t, a.A + r, a.lda, a.n, valid);
    pin_values(t);
    trsm_row<NMAX, kTriGroup, kTriSync>(t, opaque(as_const(a.tri_s)));
    trsm_row<NMAX, kTriGroup, kTriSync>(t, opaque(as_const(a.tri_2)));
    pin_values(t);
    if (valid) {
      double* qrow = a.Q + r;
#pragma unroll
      for (int j = 0; j < NMAX; ++j)
        if (j < a.n) qrow[(int64_t)j * a.ldq] = t[j];
    }
  }
}

}  // namespace rpq

// Streaming passes for 64 < n <= 128 (Algorithm Preconditioned Cholesky-QR,
// lines 2, 4 and 6).  A row of 128 doubles does not fit a lane's registers
// next to the Gram accumulators, so the row solve runs in two halves of 64
// columns, the Gram matrix is a separate pass over the stored A1, and pass B
// keeps R2^{-1} in LDS:
//   k_passW:  A1(:, 0:64)   = A(:, 0:64) R11^{-1}, then
//             A1(:, 64:128) = (A(:, 64:128) - A1(:, 0:64) R12) R22^{-1}
//             with the rank-64 update on MFMA (see passW_body); the fma
//             order per element is that of the 128-wide row solve (ascending
//             k), so A1 is the same to the bit.
//   k_gramW:  per-workgroup partial Gram matrices of A1 (36 upper 16x16 tiles),
//             32-row blocks staged in LDS, tiles split over the four waves.
//   k_passB128: Q = A1 R2^{-1} in place, R2^{-1} (128 x 128) in LDS.
// The triangle operands for nmax = 128 are R11 and R22 packed (see Tri) and R12
// row-major, in that order (written by sketch_finish).
#pragma once

#include "passes.h"

namespace rpq {

constexpr int kWH = 64;                      // half width
constexpr int kWideTri = kWH * (kWH + 1) / 2;  // packed 64-triangle
constexpr int kWideNB = 8, kWideNT = kWideNB * (kWideNB + 1) / 2, kWideE = kWideNT * 256;

// Stores columns 0 .. ncols-1 of this lane's half row at W + r0 (ld ldw).
__device__ __forceinline__ void store_half(double* W, int64_t ldw, const double (&t)[kWH], int64_t r0, int lane,
                                           bool valid, int ncols) {
  asm volatile("" : "+s"(ncols), "+s"(ldw));
  double* base = W + r0;
  if (valid) {
#pragma unroll
    for (int j = 0; j < kWH; ++j)
      if (j < ncols) (base + (int64_t)j * ldw)[lane] = t[j];
  }
}

// Row solve of the 128-column class, one 64-row panel per wave:
//   A1(:, 0:64)   = A(:, 0:64) R11^{-1}                         (lane per row)
//   A1(:, 64:128) = (A(:, 64:128) - A1(:, 0:64) R12) R22^{-1}
// The rank-64 update runs on MFMA.  For each 16-row block rb and 16-column
// block cb, in the transposed form
//   D'(col, row) = A(row, 64 + col) + sum_k R12(k, col) (-A1(row, k)),
// the accumulator starts from the A tile and each v_mfma_f64_16x16x4f64 adds
// four products of ascending k as an fma chain (which is how it rounds), so
// every entry receives exactly the fmas of the 128-wide row solve in the same
// order and A1 is the same to the bit.  R12 comes from LDS (row stride 66: the
// four lane rows hit distinct banks) and the A tiles straight from memory in
// the operand layout (four 128-byte column segments per load).
//
// Layouts: "row" layout, lane l holds row l of the panel, register set s
// (s = 0..3) holding columns 16 cb + 4 v + s at index 4 cb + v; "operand"
// layout, lane l holds in set rb row 16 rb + l % 16 at columns
// 16 cb + 4 v + l / 16.  The two are block transposes of each other over
// (lane row l / 16, register set), done by permlane32_swap between sets s and
// s + 2 and then permlane16_swap between sets s and s + 1, in both directions.
// So the solved left half goes to the operand layout (where set rb holds the
// MFMA B operands -A1(row, 4 c + l / 16) of block rb at index c), each block's
// products replace its operands in the same registers, and the result comes
// back to the row layout for the R22 solve.
constexpr int kR12Ld = kWH + 2;

__device__ __forceinline__ void swap32(double& x, double& y) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false,
                                                   false);
  x = __hiloint2double((int)hi[0], (int)lo[0]);
  y = __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ void swap16(double& x, double& y) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(x), (unsigned)__double2loint(y), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(x), (unsigned)__double2hiint(y), false,
                                                   false);
  x = __hiloint2double((int)hi[0], (int)lo[0]);
  y = __hiloint2double((int)hi[1], (int)lo[1]);
}
// Block transpose between the row and operand layouts (its own inverse).
__device__ __forceinline__ void transpose_sets(double (&vals)[4][16]) {
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    swap32(vals[0][e], vals[2][e]);
    swap32(vals[1][e], vals[3][e]);
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    swap16(vals[0][e], vals[1][e]);
    swap16(vals[2][e], vals[3][e]);
  }
}

__device__ __forceinline__ void passW_body(const PassAArgs& a, int bid, int nblk) {
  __shared__ double r12s[kWH * kR12Ld];
  if (a.info[0] != 0) return;
  // -R12 in LDS: the update A(:, 64:) - A1(:, :64) R12 takes fma(-r, x, acc),
  // which rounds as fma(r, -x, acc), with no negation of an MFMA operand
  for (int e = threadIdx.x; e < kWH * kWH; e += kPassThreads)
    r12s[(e / kWH) * kR12Ld + e % kWH] = -a.tri_s[2 * kWideTri + e];
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int64_t panels = (a.m + kWave - 1) / kWave;
  const int64_t pgroups = (panels + kPassWaves - 1) / kPassWaves;
  const int ncols = a.n - kWH;
  for (int64_t pg = bid; pg < pgroups; pg += nblk) {
    const int64_t r0 = (pg * kPassWaves + wave) * kWave;
    const bool valid = r0 + lane < a.m;
    double vals[4][16];
    {
      double t[kWH];
      load_row<kWH>(t, a.A, r0, a.lda, kWH, lane, valid);
      pin_values(t);
      trsm_row<kWH, kTriGroup, kTriSync>(t, opaque(as_const(a.tri_s)));
      pin_values(t);
      if (!valid) {
#pragma unroll
        for (int j = 0; j < kWH; ++j) t[j] = 0.0;
      }
      store_half(a.W, a.ldw, t, r0, lane, valid, kWH);
#pragma unroll
      for (int col = 0; col < kWH; ++col) vals[col & 3][4 * (col >> 4) + ((col >> 2) & 3)] = t[col];
    }
    transpose_sets(vals);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int64_t row = r0 + 16 * rb + i16;
      const bool rvalid = row < a.m;
      int nc = ncols;
      int64_t lda = a.lda;
      asm volatile("" : "+s"(nc), "+s"(lda));
      d4 acc[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = 16 * cb + 4 * v + g;
          acc[cb][v] = (rvalid && col < nc) ? a.A[row + (int64_t)(kWH + col) * lda] : 0.0;
        }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int c = 0; c < 16; ++c)
          acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(r12s[(4 * c + g) * kR12Ld + 16 * cb + i16], vals[rb][c],
                                                         acc[cb], 0, 0, 0);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) vals[rb][4 * cb + v] = acc[cb][v];
    }
    transpose_sets(vals);
    double t[kWH];
#pragma unroll
    for (int col = 0; col < kWH; ++col) t[col] = vals[col & 3][4 * (col >> 4) + ((col >> 2) & 3)];
    pin_values(t);
    trsm_row<kWH, kTriGroup, kTriSync>(t, opaque(as_const(a.tri_s + kWideTri)));
    pin_values(t);
    store_half(a.W + (int64_t)kWH * a.ldw, a.ldw, t, r0, lane, valid, ncols);
  }
}

__global__ __launch_bounds__(kPassThreads, 2) void k_passW(PassAArgs a) { passW_body(a, blockIdx.x, gridDim.x); }

// Upper 16x16 block tiles of the 128-column Gram, wave w taking tiles w, w+4, ...
struct WideTiles {
  int bi[kWideNT], bj[kWideNT];
  constexpr WideTiles() : bi(), bj() {
    int t = 0;
    for (int i = 0; i < kWideNB; ++i)
      for (int j = i; j < kWideNB; ++j) {
        bi[t] = i;
        bj[t] = j;
        ++t;
      }
  }
};

constexpr int kGramRows = 32;
constexpr int kGramLd = 2 * kWH + 1;

// Tiles W, W + 4, ... of one 4-row chunk (operand rows of the LDS block at
// xq): the tile set of each wave is fixed at compile time, so every operand and
// accumulator index is static.
template <int W>
__device__ __forceinline__ void gram_chunk(d4 (&acc)[kWideNT / kPassWaves], const double* xq, int cq) {
  constexpr WideTiles map{};
  constexpr int MT = kWideNT / kPassWaves;
  double v[kWideNB];
#pragma unroll
  for (int b = 0; b < kWideNB; ++b) v[b] = xq[16 * b + cq];
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[map.bi[W + kPassWaves * i]], v[map.bj[W + kPassWaves * i]],
                                                  acc[i], 0, 0, 0);
  }
}

// Partial Gram of the m x n matrix a.W (n <= 128) over the workgroup's 32-row
// blocks, written to a.partials[bid][tile * 256 + i * 16 + j].  Wave W owns
// tiles W, W + 4, ...; each wave runs its own instance of the block loop (same
// barriers), so that its accumulators keep one register assignment.
template <int W>
__device__ __forceinline__ void gram_loop(const PassAArgs& a, int bid, int nblk, double* xs) {
  constexpr int MT = kWideNT / kPassWaves;  // tiles per wave
  const int lane = threadIdx.x & (kWave - 1);
  const int rq = lane >> 4, cq = lane & 15;
  d4 acc[MT];
#pragma unroll
  for (int i = 0; i < MT; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  // The next block's values are loaded into registers while the current block
  // is contracted from LDS.
  constexpr int U = kGramRows * 2 * kWH / kPassThreads;
  const int64_t blocks = (a.m + kGramRows - 1) / kGramRows;
  double nx[U];
  // Row blocks are taken last first: k_passW wrote A1 in ascending row order,
  // so its last rows are still in the memory-side cache, and the first rows,
  // read last here, are then in the cache for k_passB128, which reads forward.
  auto fetch = [&](int64_t blk) __attribute__((always_inline)) {
    const int64_t r0 = (blk < blocks ? blocks - 1 - blk : 0) * kGramRows;
    int n = a.n;
    asm volatile("" : "+s"(n));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = threadIdx.x + u * kPassThreads;
      const int r = e % kGramRows, c = e / kGramRows;
      nx[u] = (blk < blocks && r0 + r < a.m && c < n) ? a.W[r0 + r + (int64_t)c * a.ldw] : 0.0;
    }
  };
  fetch(bid);
  for (int64_t blk = bid; blk < blocks; blk += nblk) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = threadIdx.x + u * kPassThreads;
      xs[(e % kGramRows) * kGramLd + e / kGramRows] = nx[u];
    }
    __syncthreads();
    fetch(blk + nblk);
#pragma unroll
    for (int q = 0; q < kGramRows / 4; ++q) gram_chunk<W>(acc, xs + (4 * q + rq) * kGramLd, cq);
  }
  // Result element (i, j) of a tile sits in lane j + 16 (i mod 4), register i / 4.
#pragma unroll
  for (int i = 0; i < MT; ++i) {
    const int tile = W + kPassWaves * i;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      a.partials[(int64_t)bid * kWideE + tile * 256 + ((lane >> 4) + 4 * v) * 16 + (lane & 15)] = acc[i][v];
  }
}

__device__ __forceinline__ void gramW_body(const PassAArgs& a, int bid, int nblk) {
  __shared__ double xs[kGramRows * kGramLd];
  if (a.info[0] != 0) return;
  switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
    case 0: gram_loop<0>(a, bid, nblk, xs); break;
    case 1: gram_loop<1>(a, bid, nblk, xs); break;
    case 2: gram_loop<2>(a, bid, nblk, xs); break;
    default: gram_loop<3>(a, bid, nblk, xs); break;
  }
}

__global__ __launch_bounds__(kPassThreads) void k_gramW(PassAArgs a) { gramW_body(a, blockIdx.x, gridDim.x); }

// Q = A1 R2^{-1} in place for nmax = 128 (see k_passB), with R2^{-1} in LDS
// (128 KB: one workgroup of eight waves per CU).  Wave w of workgroup b takes
// the 16-row blocks b * 8 + w, stepping by nblk * 8.
constexpr int kPassB128Threads = 512;
constexpr int kPassB128Waves = kPassB128Threads / kWave;

__device__ __forceinline__ void passB128_body(const PassBArgs& a, int bid, int nblk) {
  constexpr int NM = 2 * kWH, NB = NM / 16, NKC = NM / 4;
  __shared__ double Tl[NM * NM];
  if (a.info[0] != 0) return;
#pragma unroll
  for (int u = 0; u < NM * NM / kPassB128Threads; ++u) {
    const int e = threadIdx.x + u * kPassB128Threads;
    Tl[e] = a.T2[e];
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  const int64_t blocks = (a.m + 15) / 16;
  const int64_t nw = (int64_t)nblk * kPassB128Waves;
  for (int64_t blk = (int64_t)bid * kPassB128Waves + wave; blk < blocks; blk += nw) {
    const int64_t row = blk * 16 + i16;
    const bool rvalid = row < a.m;
    double x[NKC];
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      const int col = 4 * kc + g4;
      x[kc] = (rvalid && col < a.n) ? a.Q[row + (int64_t)col * a.ldq] : 0.0;
    }
    // A operand T(4 kc + l / 16, 16 cb + l % 16), B operand A1(row, 4 kc + l / 16):
    // block cb of the product is Q(rows, 16 cb ..)^T, element (c, r) in lane
    // r + 16 (c mod 4), register c / 4.  T is upper triangular, so chunk kc
    // contributes to column blocks cb >= kc / 4 only.
    // The LDS operands of chunk kc + 1 are read while chunk kc multiplies (the
    // scheduling barriers keep the compiler from hoisting all 144 reads).
    d4 acc[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
    const double* trow = Tl + g4 * NM + i16;
    double tc[NB], tn[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) tc[cb] = trow[16 * cb];
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      __builtin_amdgcn_sched_barrier(0);
      if (kc + 1 < NKC) {
#pragma unroll
        for (int cb = (kc + 1) / 4; cb < NB; ++cb) tn[cb] = trow[4 * (kc + 1) * NM + 16 * cb];
      }
#pragma unroll
      for (int cb = kc / 4; cb < NB; ++cb)
        acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(tc[cb], x[kc], acc[cb], 0, 0, 0);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) tc[cb] = tn[cb];
    }
    if (rvalid) {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int col = 16 * cb + g4 + 4 * v;
          if (col < a.n) a.Q[row + (int64_t)col * a.ldq] = acc[cb][v];
        }
    }
  }
}

__global__ __launch_bounds__(kPassB128Threads) void k_passB128(PassBArgs a) {
  passB128_body(a, blockIdx.x, gridDim.x);
}

}  // namespace rpq

// Streaming passes for 64 < n <= 128 (Algorithm Preconditioned Cholesky-QR,
// lines 2, 4 and 6).  A row of 128 doubles does not fit a lane's registers
// next to the Gram accumulators, so the row solve runs in two halves of 64
// columns, the Gram matrix is a separate pass over the stored A1, and pass B
// keeps R2^{-1} in LDS:
//   k_passW<0>: A1(:, 0:64)   = A(:, 0:64) R11^{-1}              (row solve)
//   k_passW<1>: A1(:, 64:128) = (A(:, 64:128) - A1(:, 0:64) R12) R22^{-1}
//             A1(:, 0:64) is re-read one column (512 bytes per wave) at a time,
//             eight columns ahead; the fma order per element is that of the
//             128-wide row solve (ascending k), so A1 is the same to the bit.
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

// Rank-64 update of a half row: for k = 0..63, t_j = fma(-x_k, B(k, j), t_j),
// j = 0..63, with x_k = X[k * ldx + lane] (this lane's row of column k; X is
// the wave's uniform row base) loaded D columns ahead and B streamed row by row
// through the scalar path in groups of G (as in trsm_row).
template <int G, int SYNC, typename P>
__device__ __forceinline__ void update_row64(double (&t)[kWH], P B, const double* X, int64_t ldx, int lane,
                                             bool valid) {
  constexpr int S = kWH * kWH, NG = S / G, D = 8;
  static_assert(kWH % G == 0, "a group never spans two rows of B");
  // Column k's address is formed when its load is issued (a uniform base plus
  // the lane offset), not hoisted into 64 per-lane pointers.
  auto xload = [&](int k) -> double {
    int64_t off = (int64_t)k * ldx;
    asm volatile("" : "+s"(off));
    return valid ? (X + off)[lane] : 0.0;
  };
  double xr[D];
#pragma unroll
  for (int d = 0; d < D; ++d) xr[d] = xload(d);
  double cur[G], nxt[G];
#pragma unroll
  for (int i = 0; i < G; ++i) cur[i] = B[i];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int p = (g + 1) * G + i;
      nxt[i] = (p < S) ? B[p] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int p = g * G + i;
      const int k = p / kWH, j = p % kWH;
      t[j] = __builtin_fma(-xr[k % D], cur[i], t[j]);
      if (j == kWH - 1 && k + D < kWH) xr[k % D] = xload(k + D);
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (SYNC > 0) {
      if ((g + 1) % SYNC == 0) __builtin_amdgcn_s_barrier();
    }
#pragma unroll
    for (int i = 0; i < G; ++i) cur[i] = nxt[i];
  }
}

// The same update with B (row-major 64 x 64) in LDS: B arrives as wave-uniform
// 16-byte LDS reads (every lane reads the same address) in groups of eight
// values, RING groups in flight; LDS reads of a wave return in issue order, so
// the wait for a group leaves the later groups outstanding.  The fma order per
// element is that of update_row64.
template <int RING>
__device__ __forceinline__ void update_row64_lds(double (&t)[kWH], const double* Bl, const double* X, int64_t ldx,
                                                 int lane, bool valid) {
  constexpr int G = 8, NG = kWH * kWH / G, D = 8;
  static_assert(kWH % G == 0 && NG >= RING, "groups");
  auto xload = [&](int k) -> double {
    int64_t off = (int64_t)k * ldx;
    asm volatile("" : "+s"(off));
    return valid ? (X + off)[lane] : 0.0;
  };
  double xr[D];
#pragma unroll
  for (int d = 0; d < D; ++d) xr[d] = xload(d);
  double buf[RING][G];
#pragma unroll
  for (int r = 0; r < RING; ++r)
#pragma unroll
    for (int i = 0; i < G; ++i) buf[r][i] = Bl[r * G + i];
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int slot = g % RING;
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int p = g * G + i;
      const int k = p / kWH, j = p % kWH;
      t[j] = __builtin_fma(-xr[k % D], buf[slot][i], t[j]);
      if (j == kWH - 1 && k + D < kWH) xr[k % D] = xload(k + D);
    }
    // The group's results are pinned here and the memory clobber keeps the LDS
    // reads of later groups below this point: otherwise the optimizer sinks the
    // fmas and hoists the reads, and all 4096 values of B are live at once.
#pragma unroll
    for (int i = 0; i < G; ++i) asm volatile("" : "+v"(t[(g * G + i) % kWH]));
    asm volatile("" ::: "memory");
    if (g + RING < NG) {
#pragma unroll
      for (int i = 0; i < G; ++i) buf[slot][i] = Bl[(g + RING) * G + i];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

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

// HALF 0: first 64 columns; HALF 1: the remaining n - 64 columns.
template <int HALF>
__device__ __forceinline__ void passW_body(const PassAArgs& a, int bid, int nblk) {
  __shared__ __attribute__((aligned(16))) double r12s[HALF == 1 ? kWH * kWH : 2];
  if (a.info[0] != 0) return;
  if constexpr (HALF == 1) {
    for (int e = threadIdx.x; e < kWH * kWH; e += kPassThreads) r12s[e] = a.tri_s[2 * kWideTri + e];
    __syncthreads();
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int64_t panels = (a.m + kWave - 1) / kWave;
  const int64_t pgroups = (panels + kPassWaves - 1) / kPassWaves;
  const int ncols = HALF == 0 ? kWH : a.n - kWH;
  for (int64_t pg = bid; pg < pgroups; pg += nblk) {
    const int64_t r0 = (pg * kPassWaves + wave) * kWave;
    const bool valid = r0 + lane < a.m;
    double t[kWH];
    load_row<kWH>(t, a.A + (int64_t)HALF * kWH * a.lda, r0, a.lda, ncols, lane, valid);
    pin_values(t);
    if constexpr (HALF == 1) {
      // A per-lane (all equal) base: the LDS reads then take their offsets as
      // immediates instead of one address register each.
      int z = 0;
      asm volatile("" : "+v"(z));
      update_row64_lds<4>(t, static_cast<const double*>(r12s) + 2 * z, a.W + r0, a.ldw, lane, valid);
      pin_values(t);
      trsm_row<kWH, kTriGroup, kTriSync>(t, opaque(as_const(a.tri_s + kWideTri)));
    } else {
      trsm_row<kWH, kTriGroup, kTriSync>(t, opaque(as_const(a.tri_s)));
    }
    pin_values(t);
    store_half(a.W + (int64_t)HALF * kWH * a.ldw, a.ldw, t, r0, lane, valid, ncols);
  }
}

template <int HALF>
__global__ __launch_bounds__(kPassThreads, 2) void k_passW(PassAArgs a) {
  passW_body<HALF>(a, blockIdx.x, gridDim.x);
}

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
  auto fetch = [&](int64_t blk) __attribute__((always_inline)) {
    const int64_t r0 = blk * kGramRows;
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

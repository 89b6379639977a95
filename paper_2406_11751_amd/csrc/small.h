// The n x n steps between the passes (Algorithm Preconditioned Cholesky-QR,
// lines 4-5 and 8): fixed-order reduction of the per-workgroup partial Gram
// matrices, Cholesky G1 = R2^T R2, and R = R2 R_s.
#pragma once

#include "device_common.h"

namespace rpq {

constexpr int kReduceThreads = 256;
constexpr int kReduceChunk = 64;  // partials summed per thread in the first level
constexpr int kMaxPartial2 = 8;   // second-level partials (first-level chunks) at most
constexpr int kCholThreads = 1024;
constexpr int kCholMaxN = 64;

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
  int32_t fail_code;    // info code for a failed pivot (ECHOL, or ECHOL2 in a second pass)
  double* Gg;           // nmax > 128: G1, then R2, nmax x (nmax + 1) row-major (workspace)
};

// Blocked Cholesky G1 = R2^T R2 with R2^{-1} and R = R2 R_s, one workgroup of
// sixteen waves (the block products of a step are spread over all of them, and
// each thread has few Gram partial loads), NMAX/16 column blocks of 16.  The
// matrices are row-major with a padded row stride (placement below).  Per
// block kb:
//   (a) wave 0 factors the 16x16 diagonal block and inverts it in the same
//       sweep: lanes 0-15 hold the columns of the block, lanes 16-31 the rows of
//       the identity; step k scales register k by 1/R(k,k) (lane k gets R(k,k))
//       and broadcasts R(k,i), i > k, by readlane; one fma per register then
//       updates both the trailing columns and the inverse rows;
//   (b) panel R(kb, j) = R(kb,kb)^{-T} G(kb, j), one MFMA block product per j;
//   (c) trailing update G(i, j) -= R(kb,i)^T R(kb,j) on MFMA.
// The off-diagonal blocks of R2^{-1} follow by block back substitution
// T(i,j) = -T(i,i) sum_{i<l<=j} R2(i,l) T(l,j), by increasing j - i, and
// R = R2 R_s is a sum of MFMA block products.  Diagonal pivots use the
// hardware reciprocal square root refined by Newton steps.
// A non-positive or non-finite pivot gives ECHOL at its column.

// v_mfma_f64_16x16x4f64 operand and result positions within a 16x16 block:
//   A(i, kk): lane l holds i = l%16, kk = l/16;  B(kk, j): kk = l/16, j = l%16;
//   D(i, j):  lane l register v holds i = 4v + l/16, j = l%16.
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Operands of a 16x16 block at (r0, c0) of a row-major matrix M with row stride ld.
// A operand, chunk c.
__device__ __forceinline__ double opA(const double* M, int ld, int r0, int c0, int c, int lane) {
  return M[(r0 + (lane & 15)) * ld + c0 + 4 * c + (lane >> 4)];
}
// A operand, chunk c, of the transpose of the block.
__device__ __forceinline__ double opAT(const double* M, int ld, int r0, int c0, int c, int lane) {
  return M[(r0 + 4 * c + (lane >> 4)) * ld + c0 + (lane & 15)];
}
// B operand, chunk c.
__device__ __forceinline__ double opB(const double* M, int ld, int r0, int c0, int c, int lane) {
  return M[(r0 + 4 * c + (lane >> 4)) * ld + c0 + (lane & 15)];
}
__device__ __forceinline__ d4 load_d(const double* M, int ld, int r0, int c0, int lane) {
  d4 x;
#pragma unroll
  for (int v = 0; v < 4; ++v) x[v] = M[(r0 + 4 * v + (lane >> 4)) * ld + c0 + (lane & 15)];
  return x;
}
__device__ __forceinline__ void store_d(double* M, int ld, int r0, int c0, int lane, d4 x) {
#pragma unroll
  for (int v = 0; v < 4; ++v) M[(r0 + 4 * v + (lane >> 4)) * ld + c0 + (lane & 15)] = x[v];
}

// NMAX <= 64: G, R2^{-1} and R_s all staged in LDS.  NMAX = 128: only G (then
// R2) fits in LDS; R2^{-1} is built directly in the T2 output (global memory,
// row-major, visible to the workgroup after each barrier) and R_s is read from
// its column-major workspace copy.  NMAX > 128: G as well lives in global
// memory (the workspace copy a.Gg), with the same operations in the same order.
template <int NMAX>
__device__ __forceinline__ void cholesky_body(const CholArgs& a) {
  constexpr int NB = NMAX / 16;
  constexpr int NT = NB * (NB + 1) / 2;
  constexpr int E = NT * 256;
  constexpr bool WIDE = NMAX > kCholMaxN;
  constexpr bool GLOBAL_G = NMAX > 2 * kCholMaxN;
  constexpr int LD = NMAX + 1;               // row stride of G
  constexpr int TLD = WIDE ? NMAX : LD;      // row stride of R2^{-1}
  constexpr int PER = (E + kCholThreads - 1) / kCholThreads;  // Gram entries per thread
  constexpr int PCH_MAX = WIDE ? 5 : 10;                      // registers: PCH x kMaxPartial2 loads
  constexpr int PCH = PER < PCH_MAX ? PER : PCH_MAX;          // entries per assembly round
  static_assert(NMAX % 16 == 0 && (NMAX <= kCholMaxN || NMAX % (2 * kCholMaxN) == 0), "block size");
  __shared__ double Gsl[GLOBAL_G ? 1 : NMAX * LD];  // G1, then R2 (upper)
  __shared__ double Tsl[WIDE ? 1 : NMAX * LD];    // R2^{-1} (upper), NMAX <= 64
  __shared__ double Rsl[WIDE ? 1 : NMAX * LD];    // R_s, NMAX <= 64
  __shared__ int bad_s;
  if (a.info[0] != 0) return;
  double* Ts = WIDE ? a.T2 : Tsl;
  double* Gs = GLOBAL_G ? a.Gg : Gsl;
  const int n = a.n, tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid >> 6;
  if (tid == 0) bad_s = -1;

  // Assemble G1 (upper; identity beyond n) from the second-level partials:
  // every load of a round first, then the sums in ascending partial index.
  // Zero the lower triangles so that diagonal-block products see triangular
  // operands.
  for (int e = tid; e < NMAX * NMAX; e += kCholThreads) {
    const int i = e / NMAX, j = e % NMAX;
    if (WIDE) Ts[i * TLD + j] = 0.0;
    if (i > j) Gs[i * LD + j] = 0.0;
  }
  // R_s is column-major: consecutive threads take consecutive rows i of a
  // column.  The loads are unconditional (clamped in bounds) and are issued
  // before the partial Gram loads below, so that both sets are in flight
  // together; they are placed in LDS after the assembly.
  constexpr int U = WIDE ? 1 : (NMAX * NMAX + kCholThreads - 1) / kCholThreads;
  double rv[U];
  if constexpr (!WIDE) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid + u * kCholThreads;
      const int i = min(e % NMAX, n - 1), j = min(e / NMAX, n - 1);
      rv[u] = a.Rs[i + j * n];
    }
  }
  for (int u0 = 0; u0 < PER; u0 += PCH) {
    double acc[PCH];
#pragma unroll
    for (int u = 0; u < PCH; ++u) acc[u] = 0.0;
    for (int g0 = 0; g0 < a.G2; g0 += kMaxPartial2) {
      double v[PCH][kMaxPartial2];
#pragma unroll
      for (int u = 0; u < PCH; ++u) {
        const int e = tid + (u0 + u) * kCholThreads;
#pragma unroll
        for (int g = 0; g < kMaxPartial2; ++g)
          v[u][g] = (e < E && g0 + g < a.G2) ? a.partial2[(int64_t)(g0 + g) * E + e] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < PCH; ++u) {
        double t = (g0 == 0) ? v[u][0] : acc[u] + v[u][0];
#pragma unroll
        for (int g = 1; g < kMaxPartial2; ++g)
          if (g0 + g < a.G2) t = t + v[u][g];
        acc[u] = t;
      }
    }
#pragma unroll
    for (int u = 0; u < PCH; ++u) {
      const int e = tid + (u0 + u) * kCholThreads;
      if (u0 + u < PER && e < E) {
        const int tile = e >> 8, w = e & 255;
        int bi = 0, rem = tile;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (rem >= NB - bi) {
            rem -= NB - bi;
            ++bi;
          }
        const int bj = bi + rem;
        const int i = 16 * bi + (w >> 4), j = 16 * bj + (w & 15);
        if (i <= j) Gs[i * LD + j] = (j < n) ? acc[u] : (i == j ? 1.0 : 0.0);
      }
    }
  }
  if constexpr (!WIDE) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = tid + u * kCholThreads;
      if (e >= NMAX * NMAX) break;
      const int i = e % NMAX, j = e / NMAX;
      Rsl[i * LD + j] = (i <= j && j < n) ? rv[u] : 0.0;
      Tsl[i * LD + j] = 0.0;
    }
  }
  __syncthreads();
  if (a.G1_out) {
    for (int e = tid; e < n * n; e += kCholThreads) {
      const int i = e % n, j = e / n;
      a.G1_out[e] = (i <= j) ? Gs[i * LD + j] : 0.0;
    }
  }

  // The block loops run as loops (not unrolled): the kernel executes once per
  // factorization, so its instruction stream is fetched cold and straight-line
  // code costs more than the loop overhead.
#pragma unroll 1
  for (int kb = 0; kb < NB; ++kb) {
    const int base = 16 * kb;
    // (a) diagonal block: factor (lanes 0-15) and invert (lanes 16-31).
    if (wave == 0) {
      double g[16];
#pragma unroll
      for (int r = 0; r < 16; ++r)
        g[r] = (lane < 16) ? Gs[(base + r) * LD + base + lane] : (lane - 16 == r ? 1.0 : 0.0);
      // Branch-free: a failed pivot only records its index (the first one);
      // the values computed after it are never used.
      int bad = -1;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const double d = readlane_d(g[k], k);
        if (bad < 0 && (!(d > 0.0) || !__builtin_isfinite(d))) bad = base + k;
        // Coupled Newton iteration for sqrt(d) and 1/sqrt(d) from the hardware
        // estimate (two steps), then a residual correction.
        const double y0 = __builtin_amdgcn_rsq(d);
        double gq = d * y0, hq = 0.5 * y0;
#pragma unroll
        for (int it = 0; it < 2; ++it) {
          const double rr = __builtin_fma(-hq, gq, 0.5);
          gq = __builtin_fma(gq, rr, gq);
          hq = __builtin_fma(hq, rr, hq);
        }
        const double rkk = __builtin_fma(__builtin_fma(-gq, gq, d), hq, gq);  // R(k,k)
        const double y = 2.0 * hq;                                           // 1 / R(k,k)
        g[k] = (lane == k) ? rkk : g[k] * y;
#pragma unroll
        for (int i = k + 1; i < 16; ++i) g[i] = __builtin_fma(-readlane_d(g[k], i), g[k], g[i]);
      }
      if (lane < 16) {
#pragma unroll
        for (int r = 0; r < 16; ++r) Gs[(base + r) * LD + base + lane] = (r <= lane) ? g[r] : 0.0;
      } else if (lane < 32) {
#pragma unroll
        for (int c = 0; c < 16; ++c) Ts[(base + lane - 16) * TLD + base + c] = (c >= lane - 16) ? g[c] : 0.0;
      }
      if (lane == 0 && bad >= 0 && bad < n) bad_s = bad;
    }
    __syncthreads();
    if (bad_s >= 0) {
      if (tid == 0) {
        a.info[0] = a.fail_code;
        a.info[1] = bad_s;
      }
      return;
    }
    if (kb + 1 < NB) {
      // (b) panel: R(kb, bj) = T(kb,kb)^T G(kb, bj).
      for (int pw = wave; pw < NB - 1 - kb; pw += kCholThreads / kWave) {
        const int c0 = base + 16 + 16 * pw;
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc = mfma16(opAT(Ts, TLD, base, base, c, lane), opB(Gs, LD, base, c0, c, lane), acc);
        store_d(Gs, LD, base, c0, lane, acc);
      }
      __syncthreads();
      // (c) trailing update of the blocks (bi, bj), kb < bi <= bj; tile q of
      // the trailing triangle (row by row) goes to wave q mod 4.
      const int mt = NB - 1 - kb;
#pragma unroll 1
      for (int q = wave; q < mt * (mt + 1) / 2; q += kCholThreads / kWave) {
        int bi = kb + 1, rem = q;
        while (rem >= NB - bi) {
          rem -= NB - bi;
          ++bi;
        }
        const int bj = bi + rem;
        d4 acc = load_d(Gs, LD, 16 * bi, 16 * bj, lane);
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc = mfma16(-opAT(Gs, LD, base, 16 * bi, c, lane), opB(Gs, LD, base, 16 * bj, c, lane), acc);
        store_d(Gs, LD, 16 * bi, 16 * bj, lane, acc);
      }
      __syncthreads();
    }
  }

  // Off-diagonal blocks of T = R2^{-1}, by increasing distance from the diagonal.
#pragma unroll 1
  for (int dist = 1; dist < NB; ++dist) {
    for (int bi = wave; bi + dist < NB; bi += kCholThreads / kWave) {
      const int bj = bi + dist;
      d4 p = {0.0, 0.0, 0.0, 0.0};
      for (int l = bi + 1; l <= bj; ++l)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          p = mfma16(opA(Gs, LD, 16 * bi, 16 * l, c, lane), opB(Ts, TLD, 16 * l, 16 * bj, c, lane), p);
      d4 t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int c = 0; c < 4; ++c) t = mfma16(-opA(Ts, TLD, 16 * bi, 16 * bi, c, lane), p[c], t);
      store_d(Ts, TLD, 16 * bi, 16 * bj, lane, t);
    }
    __syncthreads();
  }

  if (a.R2_out) {
    for (int e = tid; e < n * n; e += kCholThreads) {
      const int i = e % n, j = e / n;
      a.R2_out[e] = (i <= j) ? Gs[i * LD + j] : 0.0;
    }
  }
  // T2 for pass B: NMAX x NMAX row-major, zero outside the n x n upper triangle.
  if constexpr (!WIDE) {
    for (int e = tid; e < NMAX * NMAX; e += kCholThreads) {
      const int i = e / NMAX, j = e % NMAX;
      a.T2[e] = (j >= i && j < n) ? Tsl[i * LD + j] : 0.0;
    }
  } else {
    // Beyond n, R2 is the identity, so its inverse holds exact zeros there
    // except for the unit diagonal, cleared here.
    if (tid >= n && tid < NMAX) a.T2[tid * NMAX + tid] = 0.0;
  }
  // Line 8: R = R2 R_s, upper block tiles on MFMA; blocks below the diagonal are zero.
  {
#pragma unroll 1
    for (int q = wave; q < NT; q += kCholThreads / kWave) {
      int bi = 0, rem = q;
      while (rem >= NB - bi) {
        rem -= NB - bi;
        ++bi;
      }
      const int bj = bi + rem;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int l = bi; l <= bj; ++l)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          double b;
          if constexpr (WIDE) {
            const int r = 16 * l + 4 * c + (lane >> 4), cc = 16 * bj + (lane & 15);
            b = (r < n && cc < n) ? a.Rs[r + (int64_t)cc * n] : 0.0;
          } else {
            b = opB(Rsl, LD, 16 * l, 16 * bj, c, lane);
          }
          acc = mfma16(opA(Gs, LD, 16 * bi, 16 * l, c, lane), b, acc);
        }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * bi + 4 * v + (lane >> 4), j = 16 * bj + (lane & 15);
        if (i < n && j < n) a.R[i + (int64_t)j * a.ldr] = acc[v];
      }
    }
    for (int e = tid; e < n * n; e += kCholThreads) {
      const int i = e % n, j = e / n;
      if (i / 16 > j / 16) a.R[i + (int64_t)j * a.ldr] = 0.0;
    }
  }
}

// Row-solve operands (write_solve_operands, or write_solve_operands_big for
// nmax > 128 with the full matrix in `full`) of the n x n upper triangular U
// (column-major, ld n), for the substitution form of line 6 with U = R2.
__global__ __launch_bounds__(kCholThreads) void k_solve_operands(const double* U, int n, int nmax, double* tri,
                                                                 double* full, const int32_t* info) {
  if (info[0] != 0) return;
  auto u = [U, n](int k, int j) __attribute__((always_inline)) -> double { return U[k + (int64_t)j * n]; };
  if (nmax > 2 * kCholMaxN)
    write_solve_operands_big(tri, full, n, nmax, u);
  else
    write_solve_operands(tri, n, nmax, u);
}

template <int NMAX>
__global__ __launch_bounds__(kCholThreads, 1) void k_cholesky(CholArgs a) {
  cholesky_body<NMAX>(a);
}

}  // namespace rpq

// The two streaming passes over A (Algorithm Preconditioned Cholesky-QR,
// lines 2, 4 and 6), FP64.
//
// Layout: one lane per row.  A wave takes a panel of 64 consecutive rows; for
// each column j the 64 lanes load 64 consecutive doubles of column-major A
// (one 512-byte coalesced load).  The row then lives in NMAX registers.
//
// pass A: A1 row = A row * R_s^{-1} (trsm_row), stored into the Q buffer, and
//         the wave adds the panel's contribution A1_p^T A1_p to its Gram
//         accumulator: the panel is transposed through LDS and contracted over
//         rows with v_mfma_f64_16x16x4f64 on the upper 16x16 block tiles.  At
//         the end the four waves of a workgroup are summed in fixed order into
//         one partial Gram per workgroup (upper block tiles, 256 doubles each).
// pass B: Q = A1 R2^{-1}, in place in the Q buffer, on MFMA (see k_passB).
//         Reading back the stored A1 means the solve uses exactly the bits whose
//         Gram was formed.
//
// The packed triangle R_s is read through the scalar memory path (see
// trsm_row).  A workgroup's waves take panel groups in lock step (every wave
// runs the same number of iterations; rows past m are masked), so the barriers
// inside trsm_row are reached by all of them.
#pragma once

#include "device_common.h"

namespace rpq {

constexpr int kPassThreads = 256;
constexpr int kPassWaves = kPassThreads / kWave;
constexpr int kTriGroup = 32;  // triangle values per pipelined group in trsm_row
constexpr int kTriSync = 4;    // groups between workgroup barriers in trsm_row

template <int NMAX>
struct GramShape {
  static constexpr int NB = (NMAX + 15) / 16;    // 16-wide column blocks
  static constexpr int NT = NB * (NB + 1) / 2;    // upper block tiles
  static constexpr int E = NT * 256;              // doubles per partial Gram
};

// Row `lane` of the panel starting at row r0: the column base pointers are
// wave-uniform (scalar registers), the lane adds its offset.  n and lda are
// made opaque per call so that the column guards and column offsets are
// recomputed per panel instead of being hoisted into NMAX live scalar pairs.
template <int NMAX>
__device__ __forceinline__ void load_row(double (&t)[NMAX], const double* __restrict__ A, int64_t r0, int64_t lda,
                                         int n, int lane, bool valid) {
  asm volatile("" : "+s"(n), "+s"(lda));
  const double* base = A + r0;
#pragma unroll
  for (int j = 0; j < NMAX; ++j) t[j] = (valid && j < n) ? (base + (int64_t)j * lda)[lane] : 0.0;
}

// The binary32 copy of A1 (RPCHOLQR_A1_FP32) inside the Q buffer: rows
// 64b .. 64b+63 of column j occupy the first 256 bytes (two full 128-byte
// lines) of the same rows of Q, so a 64-row block of Q overwrites only its own
// rows' copy.
constexpr int kA1fRows = 64;
__device__ __forceinline__ float* a1f_ptr(double* Q, int64_t ldq, int64_t r, int64_t j) {
  return reinterpret_cast<float*>(Q + (r & ~(int64_t)(kA1fRows - 1)) + j * ldq) + (r & (kA1fRows - 1));
}

struct PassAArgs {
  int64_t m;
  int32_t n;
  const double* A;
  int64_t lda;
  const double* tri_s;  // packed R_s (see Tri)
  double* partials;     // [gridDim.x][E]
  const int32_t* info;
  double* W;            // A1 out (the Q buffer), m x n, ld ldw
  int64_t ldw;
};

// Final cross-wave sum: each wave stored its tiles in LDS red[wave][E].
template <int E>
__device__ __forceinline__ void sum_waves_to_partial(const double* red, double* __restrict__ out, int bid) {
  for (int e = threadIdx.x; e < E; e += kPassThreads) {
    double v = red[e];
#pragma unroll
    for (int w = 1; w < kPassWaves; ++w) v = v + red[w * E + e];
    out[(int64_t)bid * E + e] = v;
  }
}

template <int NMAX, bool F32A1 = false>
__device__ __forceinline__ void store_a1(const PassAArgs& a, const double (&t)[NMAX], int64_t r0, int lane,
                                         bool valid) {
  int n = a.n;
  int64_t ldw = a.ldw;
  asm volatile("" : "+s"(n), "+s"(ldw));
  if (valid) {
    if constexpr (F32A1) {
      // r0 is a multiple of 64: the wave's rows are one block of the copy
      float* base = reinterpret_cast<float*>(a.W + r0) + lane;
#pragma unroll
      for (int j = 0; j < NMAX; ++j)
        if (j < n) base[2 * (int64_t)j * ldw] = (float)t[j];
    } else {
      double* base = a.W + r0;
#pragma unroll
      for (int j = 0; j < NMAX; ++j)
        if (j < n) (base + (int64_t)j * ldw)[lane] = t[j];
    }
  }
}

// pass A (NMAX a multiple of 16, <= 64).
// MODE kSolveGram: A1 = A R_s^{-1} (stored in W) and its Gram partial.
// MODE kGramOnly:  the Gram partial of A itself (used for Q1 in the second
//                  Cholesky-QR pass of the refined precisions).
// GP: arithmetic of the Gram contraction: FP64 (v_mfma_f64_16x16x4f64); FP32
//     (A1 rounded to float, v_mfma_f32_16x16x4f32, FP32 accumulation); or BF16x2
//     (A1 rounded to float and split into bfloat16 hi + lo, G ~ hi^T hi +
//     hi^T lo + lo^T hi on v_mfma_f32_16x16x16bf16_1k, FP32 accumulation).
// LDS per wave: a half panel (32 rows) of A1, row stride NMAX+1 elements.
// MODE kSolveOnly: A1 = A U^{-1} stored in W, no Gram (the substitution form of
//                  line 6, Q = A1 R2^{-1}, run in place with A = W).
constexpr int kSolveGram = 0, kGramOnly = 1, kSolveOnly = 2;
constexpr int kBfLdr = 36;  // bf16 elements per column in the BF16x2 staging (32 rows + pad)

// bfloat16 of a float, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
constexpr int kGramF64 = 0, kGramF32 = 1, kGramBF16x2 = 2;

// F32A1: A1 is rounded to binary32, stored as such (a1f_ptr), and the Gram is
// formed from the rounded values.
template <int NMAX, int MODE = kSolveGram, int GP = kGramF64, bool F32A1 = false>
__device__ __forceinline__ void passA_body(const PassAArgs& a, int bid, int nblk) {
  static_assert(!F32A1 || (MODE == kSolveGram && GP == kGramF64), "binary32 A1 with the FP64 Gram");
  static_assert(NMAX % 16 == 0 && NMAX <= 64, "MFMA Gram tiles");
  constexpr int NB = GramShape<NMAX>::NB, NT = GramShape<NMAX>::NT, E = GramShape<NMAX>::E;
  constexpr int LDX = NMAX + 1;
  constexpr int XS = 32 * LDX;  // doubles per wave
  constexpr int LDS_D = (kPassWaves * XS > kPassWaves * E) ? kPassWaves * XS : kPassWaves * E;
  using Acc = std::conditional_t<GP == kGramF64, d4, f4>;
  static_assert(GP != kGramBF16x2 || 2 * NMAX * kBfLdr * 2 <= XS * 8, "bf16 staging fits the half-panel buffer");
  __shared__ double lds[LDS_D];
  if (a.info[0] != 0) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  double* xs = lds + wave * XS;
  const int64_t panels = (a.m + kWave - 1) / kWave;
  Acc acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = Acc{0, 0, 0, 0};
  const int half_row = lane & 31;
  const int rq = lane >> 4, cq = lane & 15;  // MFMA operand position
  const int64_t pgroups = (panels + kPassWaves - 1) / kPassWaves;
  for (int64_t pg = bid; pg < pgroups; pg += nblk) {
    const int64_t r0 = (pg * kPassWaves + wave) * kWave;
    const bool valid = r0 + lane < a.m;
    double t[NMAX];
    load_row<NMAX>(t, a.A, r0, a.lda, a.n, lane, valid);
    pin_values(t);
    if constexpr (MODE == kSolveGram || MODE == kSolveOnly) {
      trsm_row<NMAX, kTriGroup, kTriSync>(t, opaque(as_const(a.tri_s)));
      pin_values(t);
      if (!valid) {
#pragma unroll
        for (int j = 0; j < NMAX; ++j) t[j] = 0.0;
      }
      if constexpr (F32A1) {
#pragma unroll
        for (int j = 0; j < NMAX; ++j) t[j] = (double)(float)t[j];
      }
      store_a1<NMAX, F32A1>(a, t, r0, lane, valid);
    }
    if constexpr (MODE == kSolveOnly) continue;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if constexpr (GP == kGramF64) {
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
      } else if constexpr (GP == kGramBF16x2) {
        // Half panel column-major in LDS, hi and lo planes, element (r, c) at
        // c * kBfLdr + r: a lane's four consecutive rows of a column are one
        // 8-byte read, and 16 columns apart land in distinct banks.
        uint16_t* xh = reinterpret_cast<uint16_t*>(xs);
        uint16_t* xl = xh + NMAX * kBfLdr;
        wave_lds_fence();
        if ((lane >> 5) == h) {
#pragma unroll
          for (int j = 0; j < NMAX; ++j) {
            const float f = (float)t[j];
            const uint16_t hi = bf16_rne(f);
            xh[j * kBfLdr + half_row] = hi;
            xl[j * kBfLdr + half_row] = bf16_rne(f - bf16_to_float(hi));
          }
        }
        wave_lds_fence();
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {  // 16-row chunks of the half panel
          s4 vh[NB], vl[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const int off = (16 * b + cq) * kBfLdr + 16 * kk + 4 * rq;
            vh[b] = *reinterpret_cast<const s4*>(xh + off);
            vl[b] = *reinterpret_cast<const s4*>(xl + off);
          }
          int tt = 0;
#pragma unroll
          for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int bj = bi; bj < NB; ++bj) {
              acc[tt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(vh[bi], vh[bj], acc[tt], 0, 0, 0);
              acc[tt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(vh[bi], vl[bj], acc[tt], 0, 0, 0);
              acc[tt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(vl[bi], vh[bj], acc[tt], 0, 0, 0);
              ++tt;
            }
        }
      } else {
        float* xf = reinterpret_cast<float*>(xs);
        wave_lds_fence();
        if ((lane >> 5) == h) {
#pragma unroll
          for (int j = 0; j < NMAX; ++j) xf[half_row * LDX + j] = (float)t[j];
        }
        wave_lds_fence();
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          float v[NB];
#pragma unroll
          for (int b = 0; b < NB; ++b) v[b] = xf[(4 * q + rq) * LDX + 16 * b + cq];
          int tt = 0;
#pragma unroll
          for (int bi = 0; bi < NB; ++bi)
#pragma unroll
            for (int bj = bi; bj < NB; ++bj) {
              acc[tt] = __builtin_amdgcn_mfma_f32_16x16x4f32(v[bi], v[bj], acc[tt], 0, 0, 0);
              ++tt;
            }
        }
      }
    }
  }
  if constexpr (MODE == kSolveOnly) return;
  __syncthreads();
  // Result element (i, j) of a 16x16 tile sits in lane j + 16 (i mod 4), register
  // i / 4 for the FP64 MFMA, and in lane j + 16 (i / 4), register i mod 4 for FP32.
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = (GP == kGramF64) ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v, j = lane & 15;
      lds[wave * E + q * 256 + i * 16 + j] = (double)acc[q][v];
    }
  __syncthreads();
  sum_waves_to_partial<E>(lds, a.partials, bid);
}

template <int NMAX, int MODE = kSolveGram, int GP = kGramF64, bool F32A1 = false>
__global__ __launch_bounds__(kPassThreads, 2) void k_passA_mfma(PassAArgs a) {
  passA_body<NMAX, MODE, GP, F32A1>(a, blockIdx.x, gridDim.x);
}

struct PassBArgs {
  int64_t m;
  int32_t n;
  const double* T2;     // R2^{-1}, NMAX x NMAX row-major, zero outside the n x n upper triangle
  double* Q;            // holds A1 on entry, Q on exit
  int64_t ldq;
  const int32_t* info;
};

constexpr int kPassBThreads = 256;

// pass B: Q = A1 R2^{-1} with the explicit inverse T2 (R2 is well conditioned:
// kappa(R2) = kappa(A1)), one 16-row block at a time, formed transposed,
// Q^T = T2^T A1^T, on v_mfma_f64_16x16x4f64:
//   operand A (i, kk) = T2(4 kc + kk, 16 cb + i): lane l holds T2(4 kc + l/16, 16 cb + l%16),
//                       the same for every block, so it stays in registers;
//   operand B (kk, j) = A1(r0 + j, 4 kc + kk):   lane l loads A1(r0 + l%16, 4 kc + l/16),
//                       four 128-byte column segments per load;
//   result D (i, j) = Q(r0 + j, 16 cb + i) in lane j + 16 (i%4), register i/4,
//                       stored as four 128-byte column segments per store.
// All loads of a block are issued before its stores, so the update is in place.
template <int NMAX>
__device__ __forceinline__ void passB_body(const PassBArgs& a, int bid, int nblk) {
  static_assert(NMAX % 16 == 0 && NMAX <= 64, "MFMA tiles");
  constexpr int NB = NMAX / 16, NKC = NMAX / 4;
  constexpr int NOPS = NKC * NB - 2 * NB * (NB - 1);  // (kc, cb) pairs with cb >= kc / 4
  if (a.info[0] != 0) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  double t2[NOPS];
  {
    int o = 0;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
      for (int cb = kc / 4; cb < NB; ++cb) t2[o++] = a.T2[(4 * kc + g4) * NMAX + 16 * cb + i16];
  }
  const int64_t blocks = (a.m + 15) / 16;
  const int64_t nw = (int64_t)nblk * (kPassBThreads / kWave);
  for (int64_t it = (int64_t)bid * (kPassBThreads / kWave) + wave; it < blocks; it += nw) {
    // Last row blocks first: pass A wrote A1 in ascending row order, so its
    // last rows are the ones still in the memory-side cache.
    const int64_t blk = blocks - 1 - it;
    const int64_t row = blk * 16 + i16;
    const bool rvalid = row < a.m;
    double x[NKC];
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) {
      const int col = 4 * kc + g4;
      x[kc] = (rvalid && col < a.n) ? a.Q[row + (int64_t)col * a.ldq] : 0.0;
    }
    d4 acc[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
    int o = 0;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
      for (int cb = kc / 4; cb < NB; ++cb) {
        acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(t2[o], x[kc], acc[cb], 0, 0, 0);
        ++o;
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

// pass B reading the binary32 copy of A1 (a1f_ptr), widened exactly: as
// passB_body, but a wave takes a whole 64-row block of the copy (four 16-row
// blocks) and loads all of it before storing any of its rows of Q.
template <int NMAX>
__device__ __forceinline__ void passB_f32_body(const PassBArgs& a, int bid, int nblk) {
  static_assert(NMAX % 16 == 0 && NMAX <= 64, "MFMA tiles");
  constexpr int NB = NMAX / 16, NKC = NMAX / 4, SB = kA1fRows / 16;
  constexpr int NOPS = NKC * NB - 2 * NB * (NB - 1);
  if (a.info[0] != 0) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int i16 = lane & 15, g4 = lane >> 4;
  double t2[NOPS];
  {
    int o = 0;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
      for (int cb = kc / 4; cb < NB; ++cb) t2[o++] = a.T2[(4 * kc + g4) * NMAX + 16 * cb + i16];
  }
  const int64_t blocks = (a.m + kA1fRows - 1) / kA1fRows;
  const int64_t nw = (int64_t)nblk * (kPassBThreads / kWave);
  for (int64_t it = (int64_t)bid * (kPassBThreads / kWave) + wave; it < blocks; it += nw) {
    const int64_t r0 = (blocks - 1 - it) * kA1fRows;  // last blocks first, as in passB_body
    const float* src = reinterpret_cast<const float*>(a.Q + r0);
    float x[SB][NKC];
#pragma unroll
    for (int sb = 0; sb < SB; ++sb)
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc) {
        const int col = 4 * kc + g4;
        const int64_t row = r0 + 16 * sb + i16;
        x[sb][kc] = (row < a.m && col < a.n) ? src[2 * (int64_t)col * a.ldq + 16 * sb + i16] : 0.0f;
      }
    // Every load of the block has returned before the first store of the
    // block is issued (the stores overwrite the copy they read).
#pragma unroll
    for (int sb = 0; sb < SB; ++sb)
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc) asm volatile("" : "+v"(x[sb][kc])::"memory");
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      const int64_t row = r0 + 16 * sb + i16;
      d4 acc[NB];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) acc[cb] = d4{0.0, 0.0, 0.0, 0.0};
      int o = 0;
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
        for (int cb = kc / 4; cb < NB; ++cb) {
          acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(t2[o], (double)x[sb][kc], acc[cb], 0, 0, 0);
          ++o;
        }
      if (row < a.m) {
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
}

template <int NMAX, bool F32A1 = false>
__global__ __launch_bounds__(kPassBThreads) void k_passB(PassBArgs a) {
  if constexpr (F32A1)
    passB_f32_body<NMAX>(a, blockIdx.x, gridDim.x);
  else
    passB_body<NMAX>(a, blockIdx.x, gridDim.x);
}

// The binary32 copy of A1 widened into a caller's m x n column-major buffer
// (debug output).
__global__ void k_export_a1f(const double* Q, int64_t ldq, int64_t m, int32_t n, double* out, int64_t ldo) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (r < m && j < n) out[r + j * ldo] = (double)*a1f_ptr(const_cast<double*>(Q), ldq, r, j);
}

}  // namespace rpq

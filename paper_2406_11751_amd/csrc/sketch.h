// Sampling, scaled gather and Householder QR of the sample (Algorithm
// rpCholesky-QR, lines 2-3).
//
// k_gather (many workgroups): idx_r = SplitMix64 index r, A_s = sqrt(m/s) A(idx, :)
// into the workspace (s x n, ld s).  Spreading the s*n random reads over the
// whole chip matters: one workgroup cannot keep enough of them in flight.
//
// k_sketch_qr (one workgroup of 16 waves): Householder QR of A_s, R only.
// Column j lives in the 16-lane row q = j / 16 of wave j mod 16; lane l16 of
// that row holds sample rows r = l16 + 16t.  Each element is touched by one
// thread only; the Householder vector, tau and R go through LDS.
//
// Every dot product over rows r >= k uses one fixed order: lane l16 accumulates
// its rows in ascending r with fma, then the 16 partials are combined by an
// XOR butterfly (h = 1, 2, 4, 8), whose result equals the pairwise tree
// p_i += p_{i+h} and is identical in all 16 lanes.  With beta = -sign(alpha) nu,
// d = 1/(alpha - beta), v = (1, y_1 d, ...), tau = (beta - alpha)/beta and the
// update w_r = fma(-tau (v.w), v_r, w_r), this fixes every rounding of R_s.
#pragma once

#include <type_traits>
#include <utility>

#include "device_common.h"

namespace rpq {

// Calls f(integral_constant<int, i>) for i = 0..N-1 (compile-time loop).
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr int kSketchWaves = 16;
constexpr int kSketchThreads = kSketchWaves * kWave;
constexpr int kSketchMaxN = 64;  // 16 waves x 4 rows of 16 lanes; R_s staged in LDS as 64 x 65
constexpr int kGatherThreads = 256;

struct SketchArgs {
  int64_t m;
  int32_t n, s;
  uint64_t seed;
  double scale;  // sqrt(m/s), correctly rounded on the host
  const double* A;
  int64_t lda;
  double* As;     // workspace: scaled sample, s x n, ld s (the generic QR works on it in place)
  double* tri;    // out: packed R_s for the row solves (see Tri), nmax rows
  double* Rs;     // out: R_s, n x n column-major (ld n)
  int32_t nmax;
  int32_t* info;  // {code, index}
  int64_t* idx_out;  // optional
  double* As_out;    // optional, s x n, ld s
  double* Rs_out;    // optional, n x n, ld n
};

// Line 2: one thread per sample entry.
__device__ __forceinline__ void gather_body(const SketchArgs& a, int64_t bid) {
  const int64_t e = bid * kGatherThreads + threadIdx.x;
  const int64_t total = (int64_t)a.s * a.n;
  if (e >= total) return;
  const int r = (int)(e % a.s), j = (int)(e / a.s);
  const int64_t ir = sample_index(a.seed, (uint64_t)r, (uint64_t)a.m);
  const double v = a.scale * a.A[ir + (int64_t)j * a.lda];
  a.As[e] = v;
  if (a.As_out) a.As_out[e] = v;
  if (a.idx_out && j == 0) a.idx_out[r] = ir;
}

__global__ __launch_bounds__(kGatherThreads) void k_gather(SketchArgs a) { gather_body(a, blockIdx.x); }

// XOR butterfly over the 16 lanes of a row (all lanes active):
// h = 1, 2 by quad permutation, h = 4 by half-row mirror, h = 8 by row mirror.
__device__ __forceinline__ double row16_sum(double p) {
  p = p + dpp_d<0xB1>(p);   // quad_perm [1,0,3,2]
  p = p + dpp_d<0x4E>(p);   // quad_perm [2,3,0,1]
  p = p + dpp_d<0x141>(p);  // row_half_mirror
  p = p + dpp_d<0x140>(p);  // row_mirror
  return p;
}

// Sign-normalize R_s (negate rows with a negative diagonal; exact) and write
// the triangle operands of the row solves (write_solve_operands), the
// column-major copy and the optional output.  Rl holds R row-major with row
// stride LDR.
// With NORMALIZE false (a caller-supplied preconditioner, Algorithm
// Preconditioned Cholesky-QR) R is used as given.
template <int LDR, bool NORMALIZE = true>
__device__ __forceinline__ void sketch_finish(const SketchArgs& a, const double* Rl) {
  const int n = a.n, nmax = a.nmax;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e % n, j = e / n;
    double v = 0.0;
    if (i <= j) {
      v = Rl[i * LDR + j];
      if (NORMALIZE && Rl[i * LDR + i] < 0.0) v = -v;
    }
    a.Rs[e] = v;
    if (a.Rs_out) a.Rs_out[e] = v;
  }
  // element (k, j) of the sign-normalized R
  write_solve_operands(a.tri, n, nmax, [&](int k, int j) __attribute__((always_inline)) -> double {
    const double rkk = Rl[k * LDR + k];
    const double v = Rl[k * LDR + j];
    return (NORMALIZE && rkk < 0.0) ? -v : v;
  });
}

__device__ __forceinline__ void sketch_status(const SketchArgs& a, int bad_k) {
  if (threadIdx.x == 0) {
    a.info[0] = bad_k >= 0 ? 1 : 0;
    a.info[1] = bad_k;
  }
}

// Line 3 with the sample in registers: RPT rows per lane (s <= 16 RPT), n <= 64.
// Wave w owns columns 4w .. 4w+3, one per 16-lane group; lane l16 of a group
// holds rows l16 + 16 t in slot t.  One barrier per Householder step: during
// step k every wave applies reflector k to its columns that are not final yet,
// and the wave owning column k+1 then forms reflector k+1 from the freshly
// updated column into the other LDS buffer.
//
// WIDE (64 < n <= 128): the group also owns column j + 64.  Phase 1 runs steps
// 0..63 on columns 0..63 and keeps each reflector v_k in place of sample column
// k (no longer needed) and tau_k in LDS; phase 2 applies reflectors 0..63 to
// columns 64..127, each group its own column with no barriers; phase 3 runs
// steps 64..127 on columns 64..127.  Every column receives the same reflectors
// in the same order with the same arithmetic as in the unblocked sweep, so R is
// the same to the bit.
template <int RPT, bool WIDE = false>
__device__ __forceinline__ void sketch_qr_body(const SketchArgs& a) {
  constexpr int MAXN = WIDE ? 2 * kSketchMaxN : kSketchMaxN, LDR = MAXN + 1;
  static_assert(!WIDE || RPT >= 8, "rows 64..127 need slots 4..7");
  __shared__ double vbuf[2][16 * RPT];
  __shared__ double tau_s[2];
  __shared__ double tau_all[WIDE ? kSketchMaxN : 1];
  __shared__ double Rl[MAXN * LDR];
  // bad[k & 1] = k when reflector k has a zero or non-finite norm.  Written by
  // the wave forming reflector k during step k-1, read by all after the barrier
  // that ends step k-1: never read and written in the same step.
  __shared__ int bad[2];

  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int l16 = lane & 15, q = lane >> 4;
  const int j = 4 * wave + q;  // my column: each wave owns four consecutive columns
  const int n = a.n, s = a.s;
  int jc = j;  // the column currently in W (j, then j + 64 when WIDE)

  for (int e = threadIdx.x; e < MAXN * LDR; e += kSketchThreads) Rl[e] = 0.0;
  if (threadIdx.x < 2) bad[threadIdx.x] = -1;
  double W[RPT];
  auto load_column = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int r = l16 + 16 * t;
      W[t] = (jc < n && r < s) ? a.As[r + (int64_t)jc * s] : 0.0;
    }
  };
  load_column();
  __syncthreads();

  // Reflector k from my column (this wave owns column k, in lane group k mod 4;
  // row k of it sits in lane k mod 16 of that group, slot KB = k / 16).
  auto reflector = [&](auto kb, int k) __attribute__((always_inline)) {
    constexpr int KB = decltype(kb)::value;
    const int buf = k & 1;
    double p = 0.0;
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int r = l16 + 16 * t;
      const double x = (r >= k) ? W[t] : 0.0;
      p = __builtin_fma(x, x, p);
    }
    // Row k of column k sits in lane k mod 16 of the owner's group k mod 4.
    const int owner_lane = 16 * (k & 3) + (k & 15);
    const double nu2 = readlane_d(row16_sum(p), owner_lane);
    const double alpha = readlane_d(W[KB], owner_lane);
    if (nu2 == 0.0 || !__builtin_isfinite(nu2)) {
      if (lane == 0) bad[buf] = k;
      return;
    }
    const double nu = __builtin_sqrt(nu2);
    const double beta = (alpha >= 0.0) ? -nu : nu;
    const double d = 1.0 / (alpha - beta);
    const double tau = (beta - alpha) / beta;
    if (q == (k & 3)) {
      // Every slot is written (zero outside rows k .. s-1), so that the
      // reflector's readers need no row mask.  In the 128-column kernel the
      // lane's index is made opaque so that slot t is an immediate offset
      // from one LDS address: per-slot addresses hoisted out of the step loop
      // spill there, and their reloads would sit on the step's critical path.
      // (An opaque pointer instead would lose its address space and turn the
      // LDS stores into flat ones.)
      if constexpr (WIDE) {
        int li = l16 + 16 * RPT * buf;
        asm volatile("" : "+v"(li));
        double* vb = &vbuf[0][0];
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
          const int r = l16 + 16 * t;
          vb[li + 16 * t] = (r >= k && r < s) ? ((r == k) ? 1.0 : W[t] * d) : 0.0;
        }
      } else {
#pragma unroll
        for (int t = 0; t < RPT; ++t) {
          const int r = l16 + 16 * t;
          vbuf[buf][r] = (r >= k && r < s) ? ((r == k) ? 1.0 : W[t] * d) : 0.0;
        }
      }
    }
    if (lane == 0) {
      tau_s[buf] = tau;
      if (WIDE && k < kSketchMaxN) tau_all[k] = tau;
      Rl[k * LDR + k] = beta;
    }
  };

  // Reflector k applied to my column.  Rows r < k enter the dot product and
  // the update with a zero Householder entry: they add exact zeros and are
  // left unchanged (those rows of the column are already final in R).
  auto apply = [&](auto kb, int k) __attribute__((always_inline)) {
    constexpr int KB = decltype(kb)::value;
    const int buf = k & 1;
    const double tau = tau_s[buf];
    double vk[RPT];
#pragma unroll
    for (int t = 0; t < RPT; ++t) vk[t] = vbuf[buf][l16 + 16 * t];  // zero outside rows k .. s-1
    double p = 0.0;
#pragma unroll
    for (int t = 0; t < RPT; ++t) p = __builtin_fma(vk[t], W[t], p);
    const double tt = tau * row16_sum(p);
#pragma unroll
    for (int t = 0; t < RPT; ++t) W[t] = __builtin_fma(-tt, vk[t], W[t]);
    if (l16 == (k & 15) && jc > k && jc < n) Rl[k * LDR + jc] = W[KB];
  };

  // The first failed reflector ends the sweep: every wave reads bad[k & 1] at
  // the top of step k (stable there, see bad) and so stops at the same step;
  // `stopped` then skips the remaining 16-step blocks, whose first step would
  // otherwise look at the other bad slot and go on with a stale reflector.
  bool stopped = false;
  // Steps 16 KB0 .. 16 KB0 + 63 of the sweep (the columns of W are jc).
  auto sweep = [&](auto kb0) __attribute__((always_inline)) {
    constexpr int KB0 = decltype(kb0)::value;
    if (wave == 0) reflector(std::integral_constant<int, KB0>{}, 16 * KB0);
    __syncthreads();
    static_for<4>([&](auto kbI) __attribute__((always_inline)) {
      constexpr int KB = KB0 + decltype(kbI)::value;
      if (stopped) return;
      for (int kk = 0; kk < 16; ++kk) {
        const int k = 16 * KB + kk;
        if (k >= n) break;
        if (bad[k & 1] >= 0) {
          stopped = true;
          break;
        }
        // Columns jc <= k are final (reflector k would only add exact zeros to
        // them); waves whose four columns are all final idle until the barrier.
        if (jc > k && jc < n) apply(std::integral_constant<int, KB>{}, k);
        if constexpr (WIDE && KB0 == 0) {
          // Keep reflector k (in LDS since the last barrier) in place of sample
          // column k for phase 2: one value per thread.
          for (int r = threadIdx.x; r < s; r += kSketchThreads) a.As[r + (int64_t)k * s] = vbuf[k & 1][r];
        }
        if (k + 1 < n && wave == (((k + 1) & 63) >> 2)) {
          if (kk < 15)
            reflector(std::integral_constant<int, KB>{}, k + 1);
          else if constexpr (KB < KB0 + 3)
            reflector(std::integral_constant<int, KB + 1>{}, k + 1);
        }
        __syncthreads();
      }
    });
  };

  sweep(std::integral_constant<int, 0>{});
  if constexpr (WIDE) {
    if (n > kSketchMaxN && bad[0] < 0 && bad[1] < 0) {
      // Phase 2: reflectors 0..63 (kept in sample columns 0..63) on column j + 64.
      jc = j + kSketchMaxN;
      load_column();
      static_for<4>([&](auto kbI) __attribute__((always_inline)) {
        constexpr int KB = decltype(kbI)::value;
        for (int kk = 0; kk < 16; ++kk) {
          const int k = 16 * KB + kk;
          const double tau = tau_all[k];
          double vk[RPT];
#pragma unroll
          for (int t = 0; t < RPT; ++t) {
            const int r = l16 + 16 * t;
            vk[t] = (r >= k && r < s) ? a.As[r + (int64_t)k * s] : 0.0;
          }
          double p = 0.0;
#pragma unroll
          for (int t = 0; t < RPT; ++t) p = __builtin_fma(vk[t], W[t], p);
          const double tt = tau * row16_sum(p);
#pragma unroll
          for (int t = 0; t < RPT; ++t) W[t] = __builtin_fma(-tt, vk[t], W[t]);
          if (l16 == (k & 15) && jc < n) Rl[k * LDR + jc] = W[KB];
        }
      });
      __syncthreads();
      // Phase 3: steps 64..127.
      sweep(std::integral_constant<int, 4>{});
    }
  }
  const int bad_k = bad[0] >= 0 ? bad[0] : bad[1];
  sketch_status(a, bad_k);
  if (bad_k >= 0) return;
  sketch_finish<LDR>(a, Rl);
}

// Line 3 for large s or n > 64: the same layout and operation order, with the
// sample kept in global memory (a.As, worked on in place) and the Householder
// vector in dynamic LDS (2 s doubles).  n <= MAXN; each 16-lane group owns
// MAXN / 64 columns, 4 w + q + 64 c for c = 0, 1, ...
template <int MAXN>
__device__ __forceinline__ void sketch_qr_generic_body(const SketchArgs& a) {
  constexpr int NS = MAXN / 64, LDR = MAXN + 1;
  extern __shared__ double vdyn[];  // [2][s]
  __shared__ double tau_s[2];
  __shared__ double Rl[MAXN * LDR];
  __shared__ int bad[2];  // as in k_sketch_qr

  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int l16 = lane & 15, q = lane >> 4;
  const int n = a.n, s = a.s;

  for (int e = threadIdx.x; e < MAXN * LDR; e += kSketchThreads) Rl[e] = 0.0;
  if (threadIdx.x < 2) bad[threadIdx.x] = -1;
  __syncthreads();

  for (int k = -1; k < n; ++k) {
    if (k >= 0 && bad[k & 1] >= 0) break;
    if (k >= 0) {
      const int buf = k & 1;
      const double* vb = vdyn + (size_t)buf * s;
      const double tau = tau_s[buf];
#pragma unroll
      for (int c = 0; c < NS; ++c) {
        const int j = 4 * wave + q + 64 * c;
        if (j > k && j < n) {  // columns j <= k are final
          double* W = a.As + (int64_t)j * s;
          double p = 0.0;
          for (int r = l16; r < s; r += 16) {
            const double v = (r >= k) ? vb[r] : 0.0;
            p = __builtin_fma(v, W[r], p);
          }
          const double tt = tau * row16_sum(p);
          for (int r = l16; r < s; r += 16)
            if (r >= k) W[r] = __builtin_fma(-tt, vb[r], W[r]);
          if (l16 == (k & 15)) Rl[k * LDR + j] = W[k];
        }
      }
    }
    const int k1 = k + 1;
    if (k1 < n && wave == ((k1 & 63) >> 2)) {
      // Column k1 is slot k1 / 64 of lane group k1 mod 4 of this wave; its row k1
      // is in lane k1 mod 16 of that group.
      const int j1 = 4 * wave + q + 64 * (k1 >> 6);
      const bool mine1 = j1 < n;
      const double* W = a.As + (int64_t)(mine1 ? j1 : 0) * s;
      double p = 0.0;
      for (int r = l16; r < s; r += 16) {
        const double x = (r >= k1 && mine1) ? W[r] : 0.0;
        p = __builtin_fma(x, x, p);
      }
      const int owner_lane = 16 * (k1 & 3) + (k1 & 15);
      const double nu2 = readlane_d(row16_sum(p), owner_lane);
      const double alpha = readlane_d(lane == owner_lane ? W[k1] : 0.0, owner_lane);
      if (nu2 == 0.0 || !__builtin_isfinite(nu2)) {
        if (lane == 0) bad[k1 & 1] = k1;
      } else {
        const double nu = __builtin_sqrt(nu2);
        const double beta = (alpha >= 0.0) ? -nu : nu;
        const double d = 1.0 / (alpha - beta);
        const double tau = (beta - alpha) / beta;
        double* vb = vdyn + (size_t)(k1 & 1) * s;
        if (q == (k1 & 3))
          for (int r = l16; r < s; r += 16)
            if (r >= k1) vb[r] = (r == k1) ? 1.0 : W[r] * d;
        if (lane == 0) {
          tau_s[k1 & 1] = tau;
          Rl[k1 * LDR + k1] = beta;
        }
      }
    }
    __syncthreads();
  }
  const int bad_k = bad[0] >= 0 ? bad[0] : bad[1];
  sketch_status(a, bad_k);
  if (bad_k >= 0) return;
  sketch_finish<LDR>(a, Rl);
}

// Algorithm Preconditioned Cholesky-QR with a caller-supplied R_s (n x n
// upper triangular, column-major, ld a.lda, at a.A): one workgroup writes the
// numerical status (none yet) and the operands the sketch QR would have
// written, from R_s as given.
template <int MAXN>
__global__ __launch_bounds__(kSketchThreads) void k_precond_setup(SketchArgs a) {
  constexpr int LDR = MAXN + 1;
  __shared__ double Rl[MAXN * LDR];
  const int n = a.n;
  for (int e = threadIdx.x; e < MAXN * LDR; e += kSketchThreads) {
    const int i = e / LDR, j = e - i * LDR;
    Rl[e] = (i < n && j < n && i <= j) ? a.A[i + (int64_t)j * a.lda] : 0.0;
  }
  __syncthreads();
  sketch_status(a, -1);
  sketch_finish<LDR, false>(a, Rl);
}

template <int RPT>
__global__ __launch_bounds__(kSketchThreads) void k_sketch_qr(SketchArgs a) {
  sketch_qr_body<RPT>(a);
}

template <int RPT>
__global__ __launch_bounds__(kSketchThreads) void k_sketch_qr_wide(SketchArgs a) {
  sketch_qr_body<RPT, true>(a);
}

template <int MAXN>
__global__ __launch_bounds__(kSketchThreads) void k_sketch_qr_generic(SketchArgs a) {
  sketch_qr_generic_body<MAXN>(a);
}

}  // namespace rpq

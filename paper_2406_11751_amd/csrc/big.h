// Kernels for 128 < n <= 1024 (Algorithm rpCholesky-QR lines 2-3 and Algorithm
// Preconditioned Cholesky-QR lines 2, 4 and 6), FP64.  Column counts are
// padded to nmax, a multiple of 128 (identity beyond n in every triangle).
//
// Sketch QR (line 3), in panels of 32 (or 16) columns with the arithmetic of
// the unblocked sweep, so that R_s is the same to the bit:
//   k_sketch_panel:  one workgroup runs Householder steps c0 .. c0+pw-1 on the
//                    panel's columns (each 16-lane group one column in
//                    registers, one barrier per step), keeps reflector v_k in
//                    place of sample column k (zero above row k) and tau_k, and
//                    records R(k, j) for the panel's columns;
//   k_sketch_trail:  many workgroups apply reflectors c0 .. c0+pw-1, one by one
//                    and in order, to every later column (a 16-lane group per
//                    column, the reflector staged in LDS), recording R(k, j).
//   Every column thus receives reflectors 0, 1, ... in order, each as the same
//   CR16 dot product and fma update as in the unblocked sweep.
//   k_big_finish:    sign-normalizes R (or takes a caller's R_s as given) and
//                    writes the row-solve operands (write_solve_operands_big).
// Line 2 (A1 = A R_s^{-1}), k_trsm_panel, one launch per 64-column panel P:
//   the accumulator of each 16 x 16 tile starts from A and receives, on MFMA,
//   -A1(:, k) R_s(k, :) for k = 0 .. 64P - 1 in ascending order (the earlier
//   panels of A1 are read back from memory); then the panel's diagonal block is
//   solved row by row (trsm_row).  Each entry gets the fmas of the full row
//   solve in the same order, so A1 is the same to the bit.
// Line 4 (Gram), k_gram_big: 128 x 128 output groups x row splits on MFMA.
// Line 6 (Q = A1 R2^{-1}), k_passB_big: product with the explicit inverse on
//   MFMA, in place; or, with a caller's preconditioner, k_trsm_panel with R2.
#pragma once

#include "passes.h"
#include "sketch.h"
#include "wide.h"

namespace rpq {

constexpr int kBigMaxN = 1024;
constexpr int kBigBlock = 128;                 // nmax is a multiple of this
// Sketch panel width: one 16-lane group per panel column, 32 columns (512
// threads), or 16 (256 threads, 512 registers per lane) when the sample
// column takes 64 or more registers per lane.
template <int RPT>
constexpr int panel_width() { return RPT >= 64 ? 16 : 32; }
constexpr int kTrailThreads = 256;             // 16 trailing columns per workgroup
constexpr int kBigTri = kWH * (kWH + 1) / 2;   // packed 64-triangle

struct BigSketchArgs {
  int32_t n, s;
  int32_t c0;      // first column of the panel
  int32_t pw;      // panel width (panel_width<RPT>())
  double* As;      // s x n, ld s: sample; column k holds reflector v_k once formed
  double* tau;     // [n]
  double* Rg;      // n x n row-major: R of the sample as formed (before sign normalization)
  int32_t* info;
};

// W[t] for a run-time slot t without dynamic register indexing.
template <int RPT>
__device__ __forceinline__ double slot_value(const double (&W)[RPT], int t) {
  double v = 0.0;
#pragma unroll
  for (int u = 0; u < RPT; ++u) v = (u == t) ? W[u] : v;
  return v;
}

// Keeps the compiler from carrying LDS values across this point (they are
// read again after it), so that a reflector of RPT slots is not held in
// registers next to the column.
__device__ __forceinline__ void lds_reload_point() { asm volatile("" ::: "memory"); }

// Sum over t of v(t) W[t] as one fma chain in ascending t, v(t) = vb[16 t] in
// LDS, and the update W[t] -= tt v(t).  The reflector is read in chunks of
// kVChunk slots, each chunk issued before the products of the previous one
// (the scheduling barriers keep that order: left to itself the compiler puts
// each LDS read right before its fma and waits for it there).
constexpr int kVChunk = 8;
template <int RPT>
__device__ __forceinline__ double lds_dot(const double* vb, const double (&W)[RPT], double p = 0.0) {
  static_assert(RPT % kVChunk == 0, "chunks");
  double v[2][kVChunk];
#pragma unroll
  for (int u = 0; u < kVChunk; ++u) v[0][u] = vb[16 * u];
#pragma unroll
  for (int c = 0; c < RPT / kVChunk; ++c) {
    if (c + 1 < RPT / kVChunk) {
#pragma unroll
      for (int u = 0; u < kVChunk; ++u) v[(c + 1) & 1][u] = vb[16 * (kVChunk * (c + 1) + u)];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kVChunk; ++u) p = __builtin_fma(v[c & 1][u], W[kVChunk * c + u], p);
    __builtin_amdgcn_sched_barrier(0);
  }
  return p;
}
// The same with one chunk in flight at a time (its reads, then its products):
// fewer registers, for the kernels that have none to spare.
template <int RPT>
__device__ __forceinline__ double lds_dot1(const double* vb, const double (&W)[RPT], double p) {
  static_assert(RPT % kVChunk == 0, "chunks");
#pragma unroll
  for (int c = 0; c < RPT / kVChunk; ++c) {
    double v[kVChunk];
#pragma unroll
    for (int u = 0; u < kVChunk; ++u) v[u] = vb[16 * (kVChunk * c + u)];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kVChunk; ++u) p = __builtin_fma(v[u], W[kVChunk * c + u], p);
    __builtin_amdgcn_sched_barrier(0);
  }
  return p;
}
template <int RPT>
__device__ __forceinline__ void lds_update1(const double* vb, double tt, double (&W)[RPT]) {
#pragma unroll
  for (int c = 0; c < RPT / kVChunk; ++c) {
    double v[kVChunk];
#pragma unroll
    for (int u = 0; u < kVChunk; ++u) v[u] = vb[16 * (kVChunk * c + u)];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kVChunk; ++u) W[kVChunk * c + u] = __builtin_fma(-tt, v[u], W[kVChunk * c + u]);
    __builtin_amdgcn_sched_barrier(0);
  }
}
template <int RPT>
__device__ __forceinline__ void lds_update(const double* vb, double tt, double (&W)[RPT]) {
  double v[2][kVChunk];
#pragma unroll
  for (int u = 0; u < kVChunk; ++u) v[0][u] = vb[16 * u];
#pragma unroll
  for (int c = 0; c < RPT / kVChunk; ++c) {
    if (c + 1 < RPT / kVChunk) {
#pragma unroll
      for (int u = 0; u < kVChunk; ++u) v[(c + 1) & 1][u] = vb[16 * (kVChunk * (c + 1) + u)];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < kVChunk; ++u) W[kVChunk * c + u] = __builtin_fma(-tt, v[c & 1][u], W[kVChunk * c + u]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int RPT>
__global__ __launch_bounds__(16 * panel_width<RPT>()) void k_sketch_panel(BigSketchArgs a) {
  constexpr int PW = panel_width<RPT>(), NT = 16 * PW;
  __shared__ double vbuf[2][16 * RPT];
  __shared__ double tau_s[2];
  // bad[k & 1] = k when reflector k has a zero or non-finite norm (written in
  // step k-1 by the wave forming reflector k, read by all after its barrier).
  __shared__ int bad[2];
  const int n = a.n, s = a.s, c0 = a.c0;
  if (c0 > 0 && a.info[0] != 0) return;  // an earlier panel failed
  if (c0 == 0 && threadIdx.x == 0) {
    a.info[0] = 0;
    a.info[1] = -1;
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int l16 = lane & 15, q = lane >> 4;
  const int j = c0 + 4 * wave + q;  // my column
  const int kend = min(c0 + PW, n);
  double W[RPT];
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int r = l16 + 16 * t;
    W[t] = (j < n && r < s) ? a.As[r + (int64_t)j * s] : 0.0;
  }
  if (threadIdx.x < 2) bad[threadIdx.x] = -1;
  __syncthreads();

  // Reflector k from column k, run by the whole wave owning it (group qk).
  auto reflector = [&](int k) __attribute__((always_inline)) {
    const int buf = k & 1, qk = (k - c0) & 3;
    double p = 0.0;
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int r = l16 + 16 * t;
      const double x = (r >= k) ? W[t] : 0.0;
      p = __builtin_fma(x, x, p);
    }
    const int owner_lane = 16 * qk + (k & 15);
    const double nu2 = readlane_d(row16_sum(p), owner_lane);
    const double alpha = readlane_d(slot_value(W, k >> 4), owner_lane);
    if (nu2 == 0.0 || !__builtin_isfinite(nu2)) {
      if (lane == 0) bad[buf] = k;
      return;
    }
    const double nu = __builtin_sqrt(nu2);
    const double beta = (alpha >= 0.0) ? -nu : nu;
    const double d = 1.0 / (alpha - beta);
    const double tau = (beta - alpha) / beta;
    if (q == qk) {
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const int r = l16 + 16 * t;
        vbuf[buf][r] = (r >= k && r < s) ? ((r == k) ? 1.0 : W[t] * d) : 0.0;
      }
    }
    if (lane == 0) {
      tau_s[buf] = tau;
      a.tau[k] = tau;
      a.Rg[(int64_t)k * n + k] = beta;
    }
  };

  // Reflector k applied to my column (rows above k meet zeros of v_k).
  auto apply = [&](int k) __attribute__((always_inline)) {
    const int buf = k & 1;
    const double tau = tau_s[buf];
    const double tt = tau * row16_sum(lds_dot<RPT>(&vbuf[buf][l16], W));
    lds_reload_point();
    lds_update<RPT>(&vbuf[buf][l16], tt, W);
    if (l16 == (k & 15)) a.Rg[(int64_t)k * n + j] = slot_value(W, k >> 4);
  };

  if (wave == 0) reflector(c0);
  __syncthreads();
  for (int k = c0; k < kend; ++k) {
    if (bad[k & 1] >= 0) break;
    // Reflector k (in LDS since the last barrier) replaces sample column k,
    // where the trailing-column kernel reads it: one value per thread.
    for (int r = threadIdx.x; r < s; r += NT) a.As[r + (int64_t)k * s] = vbuf[k & 1][r];
    if (j > k && j < kend) apply(k);
    if (k + 1 < kend && wave == ((k + 1 - c0) >> 2)) reflector(k + 1);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int b = bad[0] >= 0 ? bad[0] : bad[1];
    if (b >= 0) {
      a.info[0] = 1;  // ESKETCH
      a.info[1] = b;
    }
  }
}

// Reflectors c0 .. kend-1 applied to the columns after the panel.
template <int RPT>
__global__ __launch_bounds__(kTrailThreads) void k_sketch_trail(BigSketchArgs a) {
  constexpr int VPT = (16 * RPT + kTrailThreads - 1) / kTrailThreads;  // staged values per thread
  __shared__ double vbuf[2][16 * RPT];
  if (a.info[0] != 0) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int l16 = lane & 15, q = lane >> 4;
  const int n = a.n, s = a.s, c0 = a.c0;
  const int kend = min(c0 + a.pw, n);
  const int j = kend + 16 * (int)blockIdx.x + 4 * wave + q;
  double W[RPT];
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int r = l16 + 16 * t;
    W[t] = (j < n && r < s) ? a.As[r + (int64_t)j * s] : 0.0;
  }
  double nv[VPT];
  auto fetch = [&](int k) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int e = threadIdx.x + u * kTrailThreads;
      nv[u] = (k < kend && e < s) ? a.As[e + (int64_t)k * s] : 0.0;
    }
  };
  auto put = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int e = threadIdx.x + u * kTrailThreads;
      if (e < 16 * RPT) vbuf[buf][e] = nv[u];
    }
  };
  fetch(c0);
  put(0);
  __syncthreads();
  for (int k = c0; k < kend; ++k) {
    const int buf = (k - c0) & 1;
    fetch(k + 1);
    const double tau = a.tau[k];
    const double tt = tau * row16_sum(lds_dot<RPT>(&vbuf[buf][l16], W));
    lds_reload_point();
    lds_update<RPT>(&vbuf[buf][l16], tt, W);
    if (j < n && l16 == (k & 15)) a.Rg[(int64_t)k * n + j] = slot_value(W, k >> 4);
    put(buf ^ 1);  // read in step k+1, after the barrier; last read in step k-1
    __syncthreads();
  }
  if (j < n) {
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int r = l16 + 16 * t;
      if (r < s) a.As[r + (int64_t)j * s] = W[t];
    }
  }
}

// Streaming sketch for samples beyond 96 rows per lane (s > 1536): the same
// steps with the same arithmetic, but the sample columns stay in the sample
// buffer (global memory, updated in place) and every pass over a column streams
// it, 16 rows per load, lane l16 taking rows l16, l16 + 16, ... in order.  The
// reflector is staged in LDS.  Panels are kGmPW columns wide.
constexpr int kGmPW = 16;
constexpr int kGmThreads = 16 * kGmPW;
constexpr int kGmMaxRows = 8192;            // LDS: two staged reflectors
constexpr int kGmUnroll = 16;               // rows per lane and chunk of a streamed pass

// The lane's rows r = l16 + 16 t, t < T, are streamed in chunks of kGmUnroll,
// the next chunk's loads issued before the current chunk is used.  Rows at or
// past s read as zero.
template <typename F>
__device__ __forceinline__ void gm_stream(const double* x, int l16, int T, int s, F&& body) {
  double cur[kGmUnroll], nxt[kGmUnroll];
  auto load = [&](int t0, double (&dst)[kGmUnroll]) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < kGmUnroll; ++u) {
      const int r = l16 + 16 * (t0 + u);
      dst[u] = (t0 + u < T && r < s) ? x[r] : 0.0;
    }
  };
  load(0, cur);
  for (int t0 = 0; t0 < T; t0 += kGmUnroll) {
    load(t0 + kGmUnroll, nxt);
#pragma unroll
    for (int u = 0; u < kGmUnroll; ++u) body(t0 + u, cur[u]);
#pragma unroll
    for (int u = 0; u < kGmUnroll; ++u) cur[u] = nxt[u];
  }
}

// fma chain of v(r) * x(r) over the lane's rows in ascending order (v zero at
// and past s).
__device__ __forceinline__ double gm_dot(const double* __restrict__ v, const double* x, int l16, int T, int s) {
  double p = 0.0;
  gm_stream(x, l16, T, s, [&](int t, double xv) __attribute__((always_inline)) {
    if (t < T) p = __builtin_fma(v[l16 + 16 * t], xv, p);
  });
  return p;
}

// x(r) = fma(-tt, v(r), x(r)) over the lane's rows below s; the new values of
// rows r0 and r1 are returned in k0 / k1 by the lanes holding them.
__device__ __forceinline__ void gm_update(const double* __restrict__ v, double* x, double tt, int l16, int T, int s,
                                          int r0, int r1, double& k0, double& k1) {
  gm_stream(x, l16, T, s, [&](int t, double xv) __attribute__((always_inline)) {
    const int r = l16 + 16 * t;
    if (t < T && r < s) {
      const double w = __builtin_fma(-tt, v[r], xv);
      x[r] = w;
      if (r == r0) k0 = w;
      if (r == r1) k1 = w;
    }
  });
}

__global__ __launch_bounds__(kGmThreads) void k_sketch_panel_gm(BigSketchArgs a) {
  __shared__ double vbuf[2][kGmMaxRows];
  __shared__ double tau_s[2];
  __shared__ int bad[2];
  const int n = a.n, s = a.s, c0 = a.c0;
  if (c0 > 0 && a.info[0] != 0) return;  // an earlier panel failed
  if (c0 == 0 && threadIdx.x == 0) {
    a.info[0] = 0;
    a.info[1] = -1;
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int l16 = lane & 15, q = lane >> 4;
  const int j = c0 + 4 * wave + q;  // my column
  const int kend = min(c0 + kGmPW, n);
  const int T = (s + 15) / 16;
  double* col = a.As + (int64_t)(j < n ? j : 0) * s;
  for (int e = threadIdx.x; e < 2 * kGmMaxRows; e += kGmThreads) (&vbuf[0][0])[e] = 0.0;
  if (threadIdx.x < 2) bad[threadIdx.x] = -1;
  // alpha: row k of the owner column after its last update, kept by the lane
  // holding it (for the first panel column, read below)
  double diag = 0.0;
  __syncthreads();

  // Reflector k from my column (k == j), run by my 16-lane group.
  auto reflector = [&](int k) __attribute__((always_inline)) {
    const int buf = k & 1;
    double p = 0.0;
    gm_stream(col, l16, T, s, [&](int t, double xv) __attribute__((always_inline)) {
      const double x = (l16 + 16 * t >= k) ? xv : 0.0;
      if (t < T) p = __builtin_fma(x, x, p);
    });
    const int owner_lane = 16 * q + (k & 15);
    const double nu2 = readlane_d(row16_sum(p), owner_lane);
    const double alpha = readlane_d(diag, owner_lane);
    if (nu2 == 0.0 || !__builtin_isfinite(nu2)) {
      if (l16 == 0) bad[buf] = k;
      return;
    }
    const double nu = __builtin_sqrt(nu2);
    const double beta = (alpha >= 0.0) ? -nu : nu;
    const double d = 1.0 / (alpha - beta);
    const double tau = (beta - alpha) / beta;
    gm_stream(col, l16, T, s, [&](int t, double xv) __attribute__((always_inline)) {
      const int r = l16 + 16 * t;
      if (t < T && r < s) vbuf[buf][r] = (r >= k) ? ((r == k) ? 1.0 : xv * d) : 0.0;
    });
    if (l16 == 0) {
      tau_s[buf] = tau;
      a.tau[k] = tau;
      a.Rg[(int64_t)k * n + k] = beta;
    }
  };

  if (j == c0) {
    diag = col[c0];  // row c0 of column c0 (c0 < n <= s)
    reflector(c0);
  }
  __syncthreads();
  for (int k = c0; k < kend; ++k) {
    if (bad[k & 1] >= 0) break;
    const int buf = k & 1;
    // Reflector k replaces sample column k, where the trailing-column kernel reads it.
    for (int r = threadIdx.x; r < s; r += kGmThreads) a.As[r + (int64_t)k * s] = vbuf[buf][r];
    if (j > k && j < kend) {
      const double tt = tau_s[buf] * row16_sum(gm_dot(vbuf[buf], col, l16, T, s));
      double w = 0.0;
      gm_update(vbuf[buf], col, tt, l16, T, s, k, k + 1, w, diag);
      if (l16 == (k & 15)) a.Rg[(int64_t)k * n + j] = w;
      if (j == k + 1) reflector(k + 1);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int b = bad[0] >= 0 ? bad[0] : bad[1];
    if (b >= 0) {
      a.info[0] = 1;  // ESKETCH
      a.info[1] = b;
    }
  }
}

// Reflectors c0 .. kend-1 applied to the columns after the panel, one 16-lane
// group per column, the reflector staged in LDS (double buffered).
__global__ __launch_bounds__(kGmThreads) void k_sketch_trail_gm(BigSketchArgs a) {
  __shared__ double vbuf[2][kGmMaxRows];
  if (a.info[0] != 0) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int l16 = lane & 15, q = lane >> 4;
  const int n = a.n, s = a.s, c0 = a.c0;
  const int kend = min(c0 + a.pw, n);
  const int j = kend + kGmPW * (int)blockIdx.x + 4 * wave + q;
  const int T = (s + 15) / 16;
  double* col = a.As + (int64_t)(j < n ? j : 0) * s;
  auto stage = [&](int k, int buf) __attribute__((always_inline)) {
    for (int e = threadIdx.x; e < 16 * T; e += kGmThreads) vbuf[buf][e] = (e < s) ? a.As[e + (int64_t)k * s] : 0.0;
  };
  stage(c0, 0);
  __syncthreads();
  for (int k = c0; k < kend; ++k) {
    const int buf = (k - c0) & 1;
    if (k + 1 < kend) stage(k + 1, buf ^ 1);  // buffer buf ^ 1 was last read in step k - 1
    if (j < n) {
      const double tt = a.tau[k] * row16_sum(gm_dot(vbuf[buf], col, l16, T, s));
      double w = 0.0, unused = 0.0;
      gm_update(vbuf[buf], col, tt, l16, T, s, k, -1, w, unused);
      if (l16 == (k & 15)) a.Rg[(int64_t)k * n + j] = w;
    }
    __syncthreads();
  }
}

// Register form of the streaming sketch for 1536 < s <= 16 * 4 * 96: one wave
// per column.  Lane (g, p) = (lane / 16, lane % 16) holds rows p + 16 t for
// t = g L .. g L + L - 1 in W[0 .. L-1] (T = ceil(s / 16) <= 4 L), so the CR16
// partial p, an fma chain over t = 0, 1, ..., is run by lane row 0 over its L
// values, handed to row 1 (same p), and so on; row 3 ends with the 16 partials
// and the same butterfly as elsewhere.  The reflector is staged in LDS.
// Columns (waves) per panel: 8, or 4 (one wave per SIMD, so that the L = 96
// column of 192 registers does not spill) for the largest samples.
template <int L>
constexpr int w_pw() { return L >= 96 ? 4 : 8; }

template <int L>
constexpr int w_rows() { return 16 * 4 * L; }

// x from lane - 16 (the next lane row's predecessor); lanes 0..15 get lane 48..63's.
__device__ __forceinline__ double from_row_above(double x, int lane) {
  const int src = ((lane + 48) & 63) << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(src, __double2loint(x));
  const int hi = __builtin_amdgcn_ds_bpermute(src, __double2hiint(x));
  return __hiloint2double(hi, lo);
}

// The CR16 dot product of the wave's column with term(i) (an fma chain per
// partial in ascending row, the four lane rows in turn), butterflied and
// broadcast to the whole wave.
template <int L, typename F>
__device__ __forceinline__ double w_chain(int lane, F&& term) {
  const int g = lane >> 4;
  double acc = 0.0;
#pragma unroll
  for (int gg = 0; gg < 4; ++gg) {
    if (g == gg) {
#pragma unroll
      for (int i = 0; i < L; ++i) acc = term(i, acc);
    }
    if (gg < 3) {
      const double up = from_row_above(acc, lane);
      if (g == gg + 1) acc = up;
    }
  }
  return readlane_d(row16_sum(acc), 48);
}

template <int L>
__device__ __forceinline__ void w_load(double (&W)[L], const double* col, int lane, int s, bool have) {
  const int g = lane >> 4, p = lane & 15;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int r = p + 16 * (g * L + i);
    W[i] = (have && r < s) ? col[r] : 0.0;
  }
}

// Apply reflector v (LDS, zero outside rows k .. s-1) with tau to the column:
// returns the new values of rows k0 and k1 to the lanes holding them.
template <int L>
__device__ __forceinline__ void w_apply(double (&W)[L], const double* v, double tau, int lane, int k0, int k1,
                                        double& keep0, double& keep1) {
  const int g = lane >> 4, p = lane & 15;
  // this lane's slots of v: v(p + 16 (g L + i)) at vb[16 i]; the chain of each
  // lane row reads them a chunk at a time (lds_dot1)
  const double* vb = v + p + 16 * g * L;
  double acc = 0.0;
#pragma unroll
  for (int gg = 0; gg < 4; ++gg) {
    if (g == gg) acc = lds_dot1<L>(vb, W, acc);
    if (gg < 3) {
      const double up = from_row_above(acc, lane);
      if (g == gg + 1) acc = up;
    }
  }
  const double tt = tau * readlane_d(row16_sum(acc), 48);
  lds_update1<L>(vb, tt, W);
#pragma unroll
  for (int i = 0; i < L; ++i) {
    const int r = p + 16 * (g * L + i);
    keep0 = (r == k0) ? W[i] : keep0;
    keep1 = (r == k1) ? W[i] : keep1;
  }
}

template <int L>
__global__ __launch_bounds__(kWave * w_pw<L>()) void k_sketch_panel_w(BigSketchArgs a) {
  constexpr int kWPW = w_pw<L>(), kWThreads = kWave * kWPW;
  __shared__ double vbuf[2][w_rows<L>()];
  __shared__ double tau_s[2];
  __shared__ int bad[2];
  const int n = a.n, s = a.s, c0 = a.c0;
  if (c0 > 0 && a.info[0] != 0) return;  // an earlier panel failed
  if (c0 == 0 && threadIdx.x == 0) {
    a.info[0] = 0;
    a.info[1] = -1;
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int g = lane >> 4, p = lane & 15;
  const int j = c0 + wave;  // my column
  const int kend = min(c0 + kWPW, n);
  double W[L];
  w_load<L>(W, a.As + (int64_t)(j < n ? j : 0) * s, lane, s, j < n);
  for (int e = threadIdx.x; e < 2 * w_rows<L>(); e += kWThreads) (&vbuf[0][0])[e] = 0.0;
  if (threadIdx.x < 2) bad[threadIdx.x] = -1;
  __syncthreads();

  // Reflector k from my column (j == k); alpha = row k of it.
  auto reflector = [&](int k, double alpha) __attribute__((always_inline)) {
    const int buf = k & 1;
    const double nu2 = w_chain<L>(lane, [&](int i, double acc) __attribute__((always_inline)) {
      const double x = (p + 16 * (g * L + i) >= k) ? W[i] : 0.0;
      return __builtin_fma(x, x, acc);
    });
    if (nu2 == 0.0 || !__builtin_isfinite(nu2)) {
      if (lane == 0) bad[buf] = k;
      return;
    }
    const double nu = __builtin_sqrt(nu2);
    const double beta = (alpha >= 0.0) ? -nu : nu;
    const double d = 1.0 / (alpha - beta);
    const double tau = (beta - alpha) / beta;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const int r = p + 16 * (g * L + i);
      if (r < s) vbuf[buf][r] = (r >= k) ? ((r == k) ? 1.0 : W[i] * d) : 0.0;
    }
    if (lane == 0) {
      tau_s[buf] = tau;
      a.tau[k] = tau;
      a.Rg[(int64_t)k * n + k] = beta;
    }
  };

  if (wave == 0) reflector(c0, a.As[c0 + (int64_t)c0 * s]);  // row c0 of column c0 (c0 < n <= s)
  __syncthreads();
  for (int k = c0; k < kend; ++k) {
    if (bad[k & 1] >= 0) break;
    const int buf = k & 1;
    // Reflector k replaces sample column k, where the trailing-column kernel reads it.
    for (int r = threadIdx.x; r < s; r += kWThreads) a.As[r + (int64_t)k * s] = vbuf[buf][r];
    if (j > k && j < kend) {
      double rk = 0.0, rk1 = 0.0;
      w_apply<L>(W, vbuf[buf], tau_s[buf], lane, k, k + 1, rk, rk1);
      const int holder = 16 * ((k >> 4) / L) + (k & 15);
      if (lane == holder) a.Rg[(int64_t)k * n + j] = rk;
      if (j == k + 1) reflector(k + 1, readlane_d(rk1, 16 * (((k + 1) >> 4) / L) + ((k + 1) & 15)));
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int b = bad[0] >= 0 ? bad[0] : bad[1];
    if (b >= 0) {
      a.info[0] = 1;  // ESKETCH
      a.info[1] = b;
    }
  }
}

// Reflectors c0 .. kend-1 applied to the columns after the panel, one wave per
// column, each reflector staged in LDS (double buffered).
template <int L>
__global__ __launch_bounds__(kWave * w_pw<L>()) void k_sketch_trail_w(BigSketchArgs a) {
  constexpr int kWPW = w_pw<L>(), kWThreads = kWave * kWPW;
  __shared__ double vbuf[2][w_rows<L>()];
  if (a.info[0] != 0) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int n = a.n, s = a.s, c0 = a.c0;
  const int kend = min(c0 + a.pw, n);
  const int j = kend + kWPW * (int)blockIdx.x + wave;
  double* col = a.As + (int64_t)(j < n ? j : 0) * s;
  double W[L];
  w_load<L>(W, col, lane, s, j < n);
  auto stage = [&](int k, int buf) __attribute__((always_inline)) {
    for (int e = threadIdx.x; e < w_rows<L>(); e += kWThreads) vbuf[buf][e] = (e < s) ? a.As[e + (int64_t)k * s] : 0.0;
  };
  stage(c0, 0);
  __syncthreads();
  for (int k = c0; k < kend; ++k) {
    const int buf = (k - c0) & 1;
    if (k + 1 < kend) stage(k + 1, buf ^ 1);  // buffer buf ^ 1 was last read in step k - 1
    if (j < n) {
      double rk = 0.0, unused = 0.0;
      w_apply<L>(W, vbuf[buf], a.tau[k], lane, k, -1, rk, unused);
      if (lane == 16 * ((k >> 4) / L) + (k & 15)) a.Rg[(int64_t)k * n + j] = rk;
    }
    __syncthreads();
  }
  if (j < n) {
    const int g = lane >> 4, p = lane & 15;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const int r = p + 16 * (g * L + i);
      if (r < s) col[r] = W[i];
    }
  }
}

struct BigFinishArgs {
  int32_t n, nmax;
  const double* Rg;        // element (k, j) at Rg[k * rs_k + j * rs_j]
  int64_t rs_k, rs_j;
  int32_t normalize;       // negate rows with a negative diagonal (the sketch's R)
  int32_t init_info;       // first kernel of the call: write info = OK
  double* Rs;              // out: n x n column-major
  double* Rs_out;          // optional copy
  double* tri;             // out: packed diagonal 64-blocks
  double* full;            // out: nmax x nmax row-major
  int32_t* info;
};

__global__ __launch_bounds__(1024) void k_big_finish(BigFinishArgs a) {
  if (a.init_info) {
    if (threadIdx.x == 0) {
      a.info[0] = 0;
      a.info[1] = -1;
    }
  } else if (a.info[0] != 0) {
    return;
  }
  const int n = a.n;
  auto rn = [&](int k, int j) -> double {
    const double v = a.Rg[k * a.rs_k + j * a.rs_j];
    return (a.normalize && a.Rg[k * a.rs_k + k * a.rs_j] < 0.0) ? -v : v;
  };
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e % n, j = e / n;
    const double v = (i <= j) ? rn(i, j) : 0.0;
    a.Rs[e] = v;
    if (a.Rs_out) a.Rs_out[e] = v;
  }
  write_solve_operands_big(a.tri, a.full, n, a.nmax, rn);
}

// Line 2 for column panel P (columns 64P .. 64P+63).  With W == A it runs in
// place (the solve Q = A1 R2^{-1}): a panel reads its own columns of A and
// the earlier panels of the result only.
struct BigTrsmArgs {
  int64_t m;
  int32_t n, nmax, P;
  const double* A;
  int64_t lda;
  double* W;
  int64_t ldw;
  const double* tri;   // packed diagonal 64-blocks of U
  const double* full;  // U row-major nmax x nmax
  const int32_t* info;
};

// The update loop keeps the B operands of the next kDepth k-chunks (over the
// block boundary) in flight while a chunk is multiplied; two waves per SIMD
// (the register budget of that) hide the rest of the latency.
constexpr int kDepth = 2;

__global__ __launch_bounds__(kPassThreads, 2) void k_trsm_panel(BigTrsmArgs a) {
  constexpr int RPT = kWH * kWH / kPassThreads;  // U block values per thread
  __shared__ double rq[2][kWH * kR12Ld];  // U(64Q .., 64P ..) blocks, double buffered
  if (a.info[0] != 0) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
  const int i16 = lane & 15, g = lane >> 4;
  const int P = a.P, c0 = kWH * P;
  const int ncols = min(kWH, a.n - c0);
  const int nit = 16 * P;  // k-chunks of the update
  const int64_t panels = (a.m + kWave - 1) / kWave;
  const int64_t pgroups = (panels + kPassWaves - 1) / kPassWaves;
  // -U(64 Qb .., 64 P ..) into LDS buffer buf.  The negation is taken here, once
  // per element, rather than on the MFMA operand each time it is read
  // (fma(-u, b, acc) is the update -A1(:, k) U(k, :) and rounds as
  // fma(u, -b, acc)).
  auto load_u = [&](int Qb, int buf) __attribute__((always_inline)) {
    const double* src = a.full + (int64_t)(kWH * Qb) * a.nmax + c0;
#pragma unroll 4
    for (int u = 0; u < RPT; ++u) {
      const int e = threadIdx.x + u * kPassThreads;
      rq[buf][(e / kWH) * kR12Ld + e % kWH] = -src[(int64_t)(e / kWH) * a.nmax + e % kWH];
    }
  };
  for (int64_t pg = blockIdx.x; pg < pgroups; pg += gridDim.x) {
    const int64_t r0 = (pg * kPassWaves + wave) * kWave;
    const bool valid = r0 + lane < a.m;
    // A1(rows, k-chunk it) for the four row blocks.  The loads are
    // unconditional (a conditional load would make the compiler wait for the
    // ones in flight): rows past m are read at row m - 1 and only reach rows
    // that are never stored; chunks past the update (it >= nit, prefetched at
    // the end) are read at clamped columns and never used.
    auto fetch_b = [&](int it, double (&dst)[4]) __attribute__((always_inline)) {
      const int col = min(4 * it + g, a.n - 1);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const int64_t row = min(r0 + 16 * rb + i16, a.m - 1);
        dst[rb] = a.W[row + (int64_t)col * a.ldw];
      }
    };
    double ring[kDepth][4];
#pragma unroll
    for (int d = 0; d < kDepth; ++d) fetch_b(d, ring[d]);
    d4 acc[4][4];
    {
      int nc = ncols;
      int64_t lda = a.lda;
      asm volatile("" : "+s"(nc), "+s"(lda));
      const double* Ap = a.A + (int64_t)c0 * lda;
      // unconditional loads as above: columns past the panel's last (nc) only
      // reach solve columns past it, which are never stored (U is the
      // identity beyond n)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        const int64_t row = min(r0 + 16 * rb + i16, a.m - 1);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int col = min(16 * cb + 4 * v + g, nc - 1);
            acc[rb][cb][v] = Ap[row + (int64_t)col * lda];
          }
      }
    }
    __syncthreads();  // the previous panel group's readers of rq are done
    if (P > 0) load_u(0, 0);
    __syncthreads();
    for (int Qb = 0; Qb < P; ++Qb) {
      const int buf = Qb & 1;
      // buffer buf ^ 1 was last read in block Qb - 1, before the last barrier
      if (Qb + 1 < P) load_u(Qb + 1, buf ^ 1);
      const double* uq = &rq[buf][g * kR12Ld + i16];
#pragma unroll
      for (int kc = 0; kc < 16; ++kc) {
        double b[4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) b[rb] = ring[kc % kDepth][rb];
        fetch_b(16 * Qb + kc + kDepth, ring[kc % kDepth]);
        // the chunk's four -U operands read together (one LDS wait, not four);
        // the wave takes issue priority over the other wave of its SIMD for the
        // products, which that wave's loads then overlap
        __builtin_amdgcn_s_setprio(1);
        double u[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) u[cb] = uq[4 * kc * kR12Ld + 16 * cb];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
          for (int rb = 0; rb < 4; ++rb)
            acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(u[cb], b[rb], acc[rb][cb], 0, 0, 0);
        __builtin_amdgcn_s_setprio(0);
      }
      __syncthreads();
    }
    double vals[4][16];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) vals[rb][4 * cb + v] = acc[rb][cb][v];
    transpose_sets(vals);
    double t[kWH];
#pragma unroll
    for (int col = 0; col < kWH; ++col) t[col] = vals[col & 3][4 * (col >> 4) + ((col >> 2) & 3)];
    pin_values(t);
    trsm_row<kWH, kTriGroup, kTriSync>(t, opaque(as_const(a.tri + (int64_t)P * kBigTri)));
    pin_values(t);
    store_half(a.W + (int64_t)c0 * a.ldw, a.ldw, t, r0, lane, valid, ncols);
  }
}

// Line 4: partial Gram matrices of X (m x n, n <= nmax).  Workgroup b takes
// output group gi = b mod ngroups, a pair (I, J), I <= J, of 128-column blocks
// (the 64 upper 16 x 16 tiles of G(I, J), or the 36 upper ones when I == J),
// and row split b / ngroups: 32-row blocks split, split + nsplit, ...  The two
// column strips of a block are staged in LDS; wave w owns tile rows {2w, 2w+1}
// (or {w, 7-w} when I == J).  Partial `split` holds every upper tile of the
// Gram matrix in the order the Cholesky kernel reads (row-major over the upper
// 16 x 16 block triangle).
struct BigGramArgs {
  int64_t m;
  int32_t n, nmax, ngroups, nsplit;
  const double* X;
  int64_t ldx;
  double* partials;
  int64_t E;
  const int32_t* info;
};

constexpr int kGRows = 32;
constexpr int kXcds = 8;  // accelerator complex dies of the device, each with its own L2
constexpr int kGLd = 2 * kBigBlock + 1;  // LDS row stride of the staged strips (odd: the transposing stores of 32 rows hit distinct banks)

// Group kinds: kGramOff, the pair I < J of 128-column blocks (G(I, J), 64
// tiles); kGramDiag, one diagonal block (G(I, I), 36 upper tiles); kGramDiag2,
// two diagonal blocks I and J = I + 1 (72 tiles, about the work of an
// off-diagonal group, so that the groups of one row split go through the rows
// at the same pace and share them in L2).  Wave WV takes tile rows
// {2 WV, 2 WV + 1} of G(I, J), or rows {WV, 7 - WV} of each diagonal block.
constexpr int kGramOff = 0, kGramDiag = 1, kGramDiag2 = 2;

template <int MODE, int WV>
__device__ __forceinline__ void gram_big_tiles(const BigGramArgs& a, int I, int J, int split, double* xs) {
  constexpr int NSET = MODE == kGramDiag2 ? 2 : 1;
  constexpr int NTS = MODE == kGramOff ? 16 : 9;  // tiles per set
  constexpr int NTW = NSET * NTS;                  // tiles of this wave
  // tile rows of this wave in a set and the first tile column of each
  constexpr int B0 = MODE == kGramOff ? 2 * WV : WV, B1 = MODE == kGramOff ? 2 * WV + 1 : 7 - WV;
  constexpr int C0 = MODE == kGramOff ? 0 : B0, C1 = MODE == kGramOff ? 0 : B1;
  static_assert((8 - C0) + (8 - C1) == NTS, "tile count");
  const int lane = threadIdx.x & (kWave - 1);
  const int rq = lane >> 4, cq = lane & 15;
  d4 acc[NTW];
#pragma unroll
  for (int i = 0; i < NTW; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  constexpr int STRIP = MODE == kGramDiag ? kBigBlock : 2 * kBigBlock;
  constexpr int U = kGRows * STRIP / kPassThreads;  // staged values per thread
  const int64_t blocks = (a.m + kGRows - 1) / kGRows;
  const int nsplit = a.nsplit;
  double nx[U];
  auto fetch = [&](int64_t blk) __attribute__((always_inline)) {
    const int64_t r0 = (blk < blocks ? blk : 0) * kGRows;
    int n = a.n;
    asm volatile("" : "+s"(n));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = threadIdx.x + u * kPassThreads;
      const int r = e % kGRows, c = e / kGRows;
      const int col = (c < kBigBlock) ? kBigBlock * I + c : kBigBlock * J + c - kBigBlock;
      nx[u] = (blk < blocks && r0 + r < a.m && col < n) ? a.X[r0 + r + (int64_t)col * a.ldx] : 0.0;
    }
  };
  fetch(split);
  for (int64_t blk = split; blk < blocks; blk += nsplit) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = threadIdx.x + u * kPassThreads;
      xs[(e % kGRows) * kGLd + e / kGRows] = nx[u];
    }
    __syncthreads();
    fetch(blk + nsplit);
#pragma unroll
    for (int qq = 0; qq < kGRows / 4; ++qq) {
      const double* xr = xs + (4 * qq + rq) * kGLd;
#pragma unroll
      for (int set = 0; set < NSET; ++set) {
        // A operand rows from the first strip of the set, B operand columns
        // from the second (the same strip for a diagonal block)
        const int aoff = set * kBigBlock;
        const int boff = MODE == kGramOff ? kBigBlock : set * kBigBlock;
        const double a0 = xr[aoff + 16 * B0 + cq], a1 = xr[aoff + 16 * B1 + cq];
        double bv[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) bv[c] = xr[boff + 16 * c + cq];
        int tt = set * NTS;
#pragma unroll
        for (int c = C0; c < 8; ++c) {
          acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bv[c], acc[tt], 0, 0, 0);
          ++tt;
        }
#pragma unroll
        for (int c = C1; c < 8; ++c) {
          acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv[c], acc[tt], 0, 0, 0);
          ++tt;
        }
      }
    }
  }
  // Result element (i, j) of a tile sits in lane j + 16 (i mod 4), register i / 4.
  const int NB = a.nmax / 16;
  double* out = a.partials + (int64_t)split * a.E;
  int tt = 0;
#pragma unroll
  for (int set = 0; set < NSET; ++set) {
    const int RI = set == 0 ? I : J;                              // block row of the set
    const int RJ = MODE == kGramOff ? J : (set == 0 ? I : J);    // block column
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int bi = 8 * RI + (h == 0 ? B0 : B1);
#pragma unroll
      for (int c = (h == 0 ? C0 : C1); c < 8; ++c) {
        const int bj = 8 * RJ + c;
        const int tile = bi * NB - bi * (bi - 1) / 2 + (bj - bi);
#pragma unroll
        for (int v = 0; v < 4; ++v) out[(int64_t)tile * 256 + ((lane >> 4) + 4 * v) * 16 + (lane & 15)] = acc[tt][v];
        ++tt;
      }
    }
  }
}

__global__ __launch_bounds__(kPassThreads) void k_gram_big(BigGramArgs a) {
  __shared__ double xs[kGRows * kGLd];
  if (a.info[0] != 0) return;
  // Workgroups are dispatched to the 8 XCDs round robin (XCD = blockIdx mod 8),
  // each XCD with its own L2.  When nsplit is a multiple of 8, the ngroups
  // workgroups of one row split are given consecutive dispatch slots of one
  // XCD, so that they read the same rows of A1 through the same L2.
  int gi, split;
  if (a.nsplit % kXcds == 0) {
    const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
    split = xcd + kXcds * (slot / a.ngroups);
    gi = slot % a.ngroups;
  } else {
    gi = blockIdx.x % a.ngroups;
    split = blockIdx.x / a.ngroups;
  }
  // Group gi: the off-diagonal pairs I < J first (row by row), then the
  // diagonal blocks two at a time, the last alone when their number is odd.
  const int NG = a.nmax / kBigBlock;
  const int noff = NG * (NG - 1) / 2;
  int mode, I, J;
  if (gi < noff) {
    mode = kGramOff;
    I = 0;
    int rem = gi;
    while (rem >= NG - 1 - I) {
      rem -= NG - 1 - I;
      ++I;
    }
    J = I + 1 + rem;
  } else {
    I = 2 * (gi - noff);
    J = I + 1;
    mode = J < NG ? kGramDiag2 : kGramDiag;
    if (mode == kGramDiag) J = I;
  }
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#define RPQ_GRAM_WAVES(M)                                       \
  switch (wv) {                                                 \
    case 0: gram_big_tiles<M, 0>(a, I, J, split, xs); break;    \
    case 1: gram_big_tiles<M, 1>(a, I, J, split, xs); break;    \
    case 2: gram_big_tiles<M, 2>(a, I, J, split, xs); break;    \
    default: gram_big_tiles<M, 3>(a, I, J, split, xs); break;   \
  }
  if (mode == kGramOff) {
    RPQ_GRAM_WAVES(kGramOff)
  } else if (mode == kGramDiag2) {
    RPQ_GRAM_WAVES(kGramDiag2)
  } else {
    RPQ_GRAM_WAVES(kGramDiag)
  }
#undef RPQ_GRAM_WAVES
}

// Line 6: Q = A1 R2^{-1} with the explicit inverse T2 (nmax x nmax row-major,
// zero outside the n x n upper triangle), in place over A1.  One workgroup of
// eight waves per CU (two per SIMD) takes 16 * passb_rows rows at a time;
// wave w owns 16-column blocks in snake order (passb_block) for all row
// blocks, with at most 64 accumulators per lane.  The contraction runs in
// stages of passb_chunks 4-wide k-chunks.  Each wave loads its own operands
// straight into registers: its T2 blocks from L2 through a buffer descriptor
// (each T2 element is used by one wave per row group, so staging it in LDS
// would only add a barrier per stage) and the rows' A1, into a ring of
// passb_depth stages, each slot refilled right after its products, so a
// load has passb_depth - 1 stages of products to arrive.  The stage loop
// runs over this workgroup's row groups back to back (the ring crosses from
// one group into the next) and is unrolled by the ring depth, so that every
// slot is a fixed set of registers.  The only barrier is at the end of a row
// group: all waves read every column of the rows, so the results are stored
// over A1 only after it.  MFMA layout as in k_passB: A operand T2(4 kc + l/16,
// 16 cb + l%16), B operand A1(row l%16, 4 kc + l/16), result Q(row l%16,
// 16 cb + 4 v + l/16) in register v.  Each accumulator receives its
// k-chunks in ascending order, so Q is the same to the bit for any shape.
// Row blocks per iteration: 64 accumulators per lane at most (48 rows at
// nmax = 512, where 64 rows would leave too few registers for the stages in
// flight); 4-wide k-chunks per stage: two up to 512 columns, else one; ring
// depth: as many stages as fit the 256 registers of a lane without spilling.
constexpr int kPassBBigWaves = 8;
template <int NMAX>
constexpr int passb_rows() { return NMAX == 512 ? 3 : 2048 / NMAX < 4 ? 2048 / NMAX : 4; }
template <int NMAX>
constexpr int passb_chunks() { return NMAX > 512 ? 1 : 2; }
template <int NMAX>
constexpr int passb_depth() { return NMAX == 1024 ? 2 : (NMAX == 384 || NMAX == 512 || NMAX == 896) ? 4 : 5; }

// Column block i of wave w, in snake order (w, 2W - 1 - w, 2W + w, ...): block
// cb carries 4 (cb + 1) k-chunks of the triangle, so every wave gets the same
// total when the blocks per wave are even.
template <int WAVES>
__device__ __forceinline__ int passb_block(int wave, int i) {
  return WAVES * i + ((i & 1) ? WAVES - 1 - wave : wave);
}

template <int NMAX, int kBRows = passb_rows<NMAX>()>
__global__ __launch_bounds__(64 * kPassBBigWaves, 1) void k_passB_big(PassBArgs a) {
  constexpr int WAVES = kPassBBigWaves;
  constexpr int NB = NMAX / 16, PERW = NB / WAVES;
  constexpr int SK = passb_chunks<NMAX>();   // 4-wide k-chunks per stage
  constexpr int SR = 4 * SK;                 // T2 rows per stage
  constexpr int D = passb_depth<NMAX>();     // stages in flight
  static_assert(NB % WAVES == 0, "pass B shape");
  if (a.info[0] != 0) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i16 = lane & 15, g4 = lane >> 4;
  const int n = a.n;
  const int nstage = (n + SR - 1) / SR;
  const int64_t groups = (a.m + 16 * kBRows - 1) / (16 * kBRows);
  if ((int64_t)blockIdx.x >= groups) return;
  const int64_t my_groups = (groups - blockIdx.x + gridDim.x - 1) / gridDim.x;
  const int64_t nsteps = (my_groups * nstage + D - 1) / D * D;  // padded to whole rings
  const __amdgpu_buffer_rsrc_t t2r =
      __builtin_amdgcn_make_buffer_rsrc((void*)a.T2, (short)0, NMAX * NMAX * (int)sizeof(double), 0x00020000);
  const int t2_lane = (g4 * NMAX + i16) * (int)sizeof(double);
  constexpr int kT2Past = NMAX * NMAX * (int)sizeof(double);
  double U[D][SK][PERW];    // ring of stages: T2(4 kc + l/16, 16 cb + l%16) of the wave's blocks
  double B[D][SK][kBRows];  // and A1(row l%16, 4 kc + l/16) of the row blocks
  auto fetch = [&](int slot, int64_t grp, int st) __attribute__((always_inline)) {
    const int64_t rbase = grp * 16 * kBRows;
#pragma unroll
    for (int kk = 0; kk < SK; ++kk) {
      const int kc = SK * st + kk;
#pragma unroll
      for (int i = 0; i < PERW; ++i) {
        const int cb = passb_block<WAVES>(wave, i);
        const int off = cb >= (kc >> 2) ? (4 * kc * NMAX + 16 * cb) * (int)sizeof(double) : kT2Past;
        U[slot][kk][i] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(t2r, t2_lane, off, 0));
      }
      const int col = min(4 * kc + g4, n - 1);
#pragma unroll
      for (int rb = 0; rb < kBRows; ++rb) {
        const int64_t row = min(rbase + 16 * rb + i16, a.m - 1);
        B[slot][kk][rb] = a.Q[row + (int64_t)col * a.ldq];
      }
    }
  };
  // stage counters: (grp_c, st_c) consumed now, (grp_f, st_f) fetched now (D later)
  int64_t grp_c = blockIdx.x, grp_f = blockIdx.x;
  int st_c = 0, st_f = 0;
  auto advance = [&](int64_t& grp, int& st) __attribute__((always_inline)) {
    if (++st == nstage) {
      st = 0;
      grp += gridDim.x;
    }
  };
#pragma unroll
  for (int j = 0; j < D; ++j) {
    fetch(j, grp_f, st_f);
    advance(grp_f, st_f);
  }
  d4 acc[kBRows][PERW];
  for (int64_t g0 = 0; g0 < nsteps; g0 += D) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int st = st_c;
      if (st == 0) {
#pragma unroll
        for (int rb = 0; rb < kBRows; ++rb)
#pragma unroll
          for (int i = 0; i < PERW; ++i) acc[rb][i] = d4{0.0, 0.0, 0.0, 0.0};
      }
      __builtin_amdgcn_s_setprio(1);  // issue priority for the stage's products
      if (SR * (st + 1) > n) {  // the last stage: columns past n (clamped reads) are zero
#pragma unroll
        for (int kk = 0; kk < SK; ++kk)
#pragma unroll
          for (int rb = 0; rb < kBRows; ++rb)
            if (SR * st + 4 * kk + g4 >= n) B[j][kk][rb] = 0.0;
      }
#pragma unroll
      for (int kk = 0; kk < SK; ++kk) {
        const int kc = SK * st + kk;
#pragma unroll
        for (int i = 0; i < PERW; ++i) {
          const int cb = passb_block<WAVES>(wave, i);
          if (cb >= (kc >> 2)) {  // T2 is zero left of its diagonal (a wave-uniform test)
#pragma unroll
            for (int rb = 0; rb < kBRows; ++rb)
              acc[rb][i] = __builtin_amdgcn_mfma_f64_16x16x4f64(U[j][kk][i], B[j][kk][rb], acc[rb][i], 0, 0, 0);
          }
        }
      }
      __builtin_amdgcn_s_setprio(0);
      // the slot is free again: it takes the stage D - 1 stages after the next
      fetch(j, grp_f, st_f);
      advance(grp_f, st_f);
      if (st == nstage - 1) {
        // every wave has read all columns of these rows of A1 before any is overwritten
        __syncthreads();
        const int64_t rbase = grp_c * 16 * kBRows;
#pragma unroll
        for (int rb = 0; rb < kBRows; ++rb) {
          const int64_t row = rbase + 16 * rb + i16;
          if (row < a.m) {
#pragma unroll
            for (int i = 0; i < PERW; ++i)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int col = 16 * passb_block<WAVES>(wave, i) + 4 * v + g4;
                if (col < n) a.Q[row + (int64_t)col * a.ldq] = acc[rb][i][v];
              }
          }
        }
      }
      advance(grp_c, st_c);
    }
  }
}

}  // namespace rpq

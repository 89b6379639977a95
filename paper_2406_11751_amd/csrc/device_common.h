// Device helpers shared by the rpCholesky-QR kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rpq {

constexpr int kWave = 64;

// s_waitcnt immediates (gfx9 encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4,
// lgkmcnt 11:8; a field at its maximum does not wait).
constexpr int kWaitLgkm0 = 0xC07F;  // lgkmcnt(0) only

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) in counter form: output number
// r of the generator seeded with `seed` is mix64(seed + (r+1)*golden_gamma).
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t r) {
  uint64_t z = seed + (r + 1u) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Uniform index in [0, m): floor(z * m / 2^64) (multiply-high, Lemire 2019).
__device__ __forceinline__ int64_t sample_index(uint64_t seed, uint64_t r, uint64_t m) {
  return (int64_t)__umul64hi(splitmix64_at(seed, r), m);
}

// DPP move of a double (both halves with the same control; all lanes active).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// Keeps the compiler from moving LDS accesses of this wave across this point;
// LDS operations of one wave complete in issue order.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Packed triangle used by the row-wise solves: row k of an NMAX x NMAX upper
// triangular U is stored as [1/U(k,k), U(k,k+1), ..., U(k,NMAX-1)], rows back
// to back (NMAX(NMAX+1)/2 doubles).  Beyond n the triangle is the identity.
__host__ __device__ constexpr int tri_row_start(int k, int nmax) { return k * nmax - k * (k - 1) / 2; }

// Writes the operands of the row-wise solves with an upper triangular U of
// order n (element (k, j) given by u(k, j), identity beyond n), padded to nmax:
//   nmax <= 64: one packed triangle (below), nmax rows;
//   nmax = 128: the packed triangles of U11 = U(0:64, 0:64) and U22 =
//               U(64:128, 64:128), then U12 = U(0:64, 64:128) row-major 64 x 64
//               (nmax (nmax + 1) / 2 doubles in both cases).
// Every thread of the block takes part.
template <typename F>
__device__ __forceinline__ void write_solve_operands(double* dst, int n, int nmax, F&& u) {
  auto un = [&](int k, int j) __attribute__((always_inline)) -> double {
    return (k >= n || j >= n) ? ((j == k) ? 1.0 : 0.0) : u(k, j);
  };
  auto put_packed = [&](double* out, int k0, int w) __attribute__((always_inline)) {  // rows k0 .. k0+w-1, cols k0 ..
    for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
      const int k = e / w, j = e - k * w;
      if (j < k) continue;
      const double v = (j == k) ? 1.0 / un(k0 + k, k0 + k) : un(k0 + k, k0 + j);
      out[tri_row_start(k, w) + (j - k)] = v;
    }
  };
  if (nmax <= 64) {
    put_packed(dst, 0, nmax);
  } else {
    constexpr int H = 64;
    put_packed(dst, 0, H);
    put_packed(dst + H * (H + 1) / 2, H, H);
    double* u12 = dst + H * (H + 1);
    for (int e = threadIdx.x; e < H * H; e += blockDim.x) u12[e] = un(e / H, H + e % H);
  }
}

// Row-solve operands of an upper triangular U of order n > 128, padded to nmax
// (a multiple of 64; identity beyond n): the packed triangles of the 64 x 64
// diagonal blocks U(64p : 64p+64, 64p : 64p+64), p = 0 .. nmax/64 - 1, back to
// back in tri (64 * 65 / 2 doubles each), and all of U row-major nmax x nmax in
// full (zero below the diagonal), from which the off-diagonal blocks are read.
template <typename F>
__device__ __forceinline__ void write_solve_operands_big(double* tri, double* full, int n, int nmax, F&& u) {
  auto un = [&](int k, int j) __attribute__((always_inline)) -> double {
    return (k >= n || j >= n) ? ((j == k) ? 1.0 : 0.0) : u(k, j);
  };
  constexpr int H = 64, HT = H * (H + 1) / 2;
  for (int e = threadIdx.x; e < (nmax / H) * H * H; e += blockDim.x) {
    const int p = e / (H * H), k = (e / H) % H, j = e % H;
    if (j < k) continue;
    const int k0 = p * H;
    tri[p * HT + tri_row_start(k, H) + (j - k)] = (j == k) ? 1.0 / un(k0 + k, k0 + k) : un(k0 + k, k0 + j);
  }
  for (int e = threadIdx.x; e < nmax * nmax; e += blockDim.x) {
    const int k = e / nmax, j = e % nmax;
    full[e] = (j >= k) ? un(k, j) : 0.0;
  }
}

template <int NMAX>
struct Tri {
  static constexpr int size = NMAX * (NMAX + 1) / 2;
  int k[size], j[size];
  constexpr Tri() : k(), j() {
    int p = 0;
    for (int kk = 0; kk < NMAX; ++kk)
      for (int jj = kk; jj < NMAX; ++jj) {
        k[p] = kk;
        j[p] = jj;
        ++p;
      }
  }
};

// Row-wise triangular solve x U = t, in place on t, for the packed triangle
// `tri` (LDS or global):
//   for k = 0..NMAX-1:  x_k = t_k * (1/U(k,k));  t_j = fma(-x_k, U(k,j), t_j), j > k.
// Each t_j receives its fma updates in ascending k, so the result equals the
// substitution x_j = (t_j - sum_{k<j} x_k U(k,j)) * (1/U(j,j)) accumulated in
// that order.  Padding columns j >= n never feed a column below n.
// The triangle is consumed in groups of G values.  At the top of group g the
// wave waits for the values of group g (lgkmcnt(0): scalar loads return out of
// order, so no finer wait exists), then issues the loads of group g+1 and does
// the arithmetic of group g while they are in flight; a scheduling barrier
// closes each group, so at most 2G triangle values are live in registers.
// With SYNC > 0 the waves of the workgroup meet at a barrier every SYNC groups,
// so that they sweep the triangle together and its values are fetched into the
// scalar cache once per workgroup rather than once per wave (the caller must
// give every wave of the workgroup the same number of calls).
template <int NMAX, int G, int SYNC, typename P>
__device__ __forceinline__ void trsm_row(double (&t)[NMAX], P tri) {
  constexpr Tri<NMAX> map{};
  constexpr int S = Tri<NMAX>::size;
  constexpr int NG = (S + G - 1) / G;
  double cur[G], nxt[G];
#pragma unroll
  for (int i = 0; i < G; ++i) cur[i] = (i < S) ? tri[i] : 0.0;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int p = (g + 1) * G + i;
      nxt[i] = (p < S) ? tri[p] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int p = g * G + i;
      if (p < S) {
        const int k = map.k[p], j = map.j[p];
        if (j == k)
          t[k] = t[k] * cur[i];
        else
          t[j] = __builtin_fma(-t[k], cur[i], t[j]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (SYNC > 0) {
      if ((g + 1) % SYNC == 0) __builtin_amdgcn_s_barrier();
    }
#pragma unroll
    for (int i = 0; i < G; ++i) cur[i] = nxt[i];
  }
}

// Makes every value of t opaque at this point: the computation producing t
// completes here and is not sunk into later (conditional) uses.
template <int N>
__device__ __forceinline__ void pin_values(double (&t)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) asm volatile("" : "+v"(t[j]));
}

// Constant-address-space view of a device pointer.  Loads through it are
// eligible for the scalar memory path (s_load into SGPRs), which is how the
// row solves receive their wave-uniform triangle values: no vector-register or
// LDS bandwidth is spent on broadcasting them.  Only for memory that no kernel
// writes while the reading kernel runs.
typedef const __attribute__((address_space(4))) double* const_dptr;
__device__ __forceinline__ const_dptr as_const(const double* p) { return (const_dptr)p; }

__device__ __forceinline__ const_dptr opaque(const_dptr p) {
  int off = 0;
  asm volatile("" : "+s"(off));
  return p + off;
}

// Returns p unchanged, but opaque to the optimizer: loads through the result
// cannot be hoisted out of the enclosing loop.  Keeps the per-panel LDS reads
// of the triangles inside the panel loop instead of all 2x NMAX^2/2 values
// being hoisted into (spilled) registers.
template <typename T>
__device__ __forceinline__ const T* opaque(const T* p) {
  int off = 0;
  asm volatile("" : "+s"(off));
  return p + off;
}

}  // namespace rpq

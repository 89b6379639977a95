// Device helpers shared by the rpCholesky-QR kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpq {

constexpr int kWave = 64;

typedef double d4 __attribute__((ext_vector_type(4)));

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

// Fixed-order 64-lane sum: lane l holds partial p_l; for h = 32,16,...,1 the
// partials are combined as p_l + p_{l+h}.  Every lane returns p_0.
__device__ __forceinline__ double lane_tree_sum(double p) {
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1) p = p + __shfl_down(p, h, kWave);
  return __shfl(p, 0, kWave);
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
// The triangle is consumed in groups of G values; the loads of group g+1 are
// issued before the arithmetic of group g and a scheduling barrier closes each
// group, so at most 2G triangle values are live in registers.
template <int NMAX, int G>
__device__ __forceinline__ void trsm_row(double (&t)[NMAX], const double* tri) {
  constexpr Tri<NMAX> map{};
  constexpr int S = Tri<NMAX>::size;
  constexpr int NG = (S + G - 1) / G;
  double cur[G], nxt[G];
#pragma unroll
  for (int i = 0; i < G; ++i) cur[i] = (i < S) ? tri[i] : 0.0;
#pragma unroll
  for (int g = 0; g < NG; ++g) {
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
#pragma unroll
    for (int i = 0; i < G; ++i) cur[i] = nxt[i];
  }
}

// Copies a packed triangle into LDS (whole workgroup; caller synchronizes).
template <int NMAX>
__device__ __forceinline__ void stage_tri(double* dst, const double* src) {
  for (int e = threadIdx.x; e < Tri<NMAX>::size; e += blockDim.x) dst[e] = src[e];
}

// Makes every value of t opaque at this point: the computation producing t
// completes here and is not sunk into later (conditional) uses.
template <int N>
__device__ __forceinline__ void pin_values(double (&t)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) asm volatile("" : "+v"(t[j]));
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

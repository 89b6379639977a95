// Batched entry kernels: every launch covers all problems of one size class.
// A launch's blocks are described by an item table built when the plan is
// created (problem index, the block's index among that problem's blocks, and
// that problem's block count), so the single-problem kernel bodies run
// unchanged with per-problem arguments read from a device table.
#pragma once

#include "passes.h"
#include "sketch.h"
#include "small.h"
#include "wide.h"

namespace rpq {

struct BatchItem {
  int32_t problem, local, count;
};

// The argument tables are read from device memory, so the compiler cannot
// tell that their pointers address global memory and would go through flat
// instructions, which also count against the LDS counter and make it wait for
// each load before the next.  Each pointer field is therefore re-read from
// the table as a pointer to global memory.
template <typename T>
__device__ __forceinline__ T* global_field(T* const& field) {
  using G = __attribute__((address_space(1))) T*;
  return (T*)*static_cast<const G*>(static_cast<const void*>(&field));
}
__device__ __forceinline__ void to_global(SketchArgs& a, const SketchArgs& t) {
  a.A = global_field(t.A);
  a.As = global_field(t.As);
  a.tri = global_field(t.tri);
  a.Rs = global_field(t.Rs);
  a.idx_out = global_field(t.idx_out);
  a.As_out = global_field(t.As_out);
  a.Rs_out = global_field(t.Rs_out);
}
__device__ __forceinline__ void to_global(PassAArgs& a, const PassAArgs& t) {
  a.A = global_field(t.A);
  a.tri_s = global_field(t.tri_s);
  a.partials = global_field(t.partials);
  a.W = global_field(t.W);
}
__device__ __forceinline__ void to_global(PassBArgs& a, const PassBArgs& t) {
  a.T2 = global_field(t.T2);
  a.Q = global_field(t.Q);
}
__device__ __forceinline__ void to_global(CholArgs& a, const CholArgs& t) {
  a.partial2 = global_field(t.partial2);
  a.Rs = global_field(t.Rs);
  a.T2 = global_field(t.T2);
  a.R = global_field(t.R);
  a.G1_out = global_field(t.G1_out);
  a.R2_out = global_field(t.R2_out);
  a.Gg = global_field(t.Gg);
}

__global__ __launch_bounds__(kGatherThreads) void kb_gather(const SketchArgs* __restrict__ args,
                                                            const BatchItem* __restrict__ items) {
  const BatchItem it = items[blockIdx.x];
  SketchArgs a = args[it.problem];
  to_global(a, args[it.problem]);
  gather_body(a, it.local);
}

template <int RPT>
__global__ __launch_bounds__(kSketchThreads) void kb_sketch_qr(const SketchArgs* __restrict__ args,
                                                               const int32_t* __restrict__ probs, int32_t* info) {
  const int p = probs[blockIdx.x];
  SketchArgs a = args[p];
  a.info = info + 2 * p;
  to_global(a, args[p]);
  sketch_qr_body<RPT>(a);
}

template <int RPT>
__global__ __launch_bounds__(kSketchThreads) void kb_sketch_qr_wide(const SketchArgs* __restrict__ args,
                                                                    const int32_t* __restrict__ probs, int32_t* info) {
  const int p = probs[blockIdx.x];
  SketchArgs a = args[p];
  a.info = info + 2 * p;
  to_global(a, args[p]);
  sketch_qr_body<RPT, true>(a);
}

template <int MAXN>
__global__ __launch_bounds__(kSketchThreads) void kb_sketch_qr_generic(const SketchArgs* __restrict__ args,
                                                                       const int32_t* __restrict__ probs,
                                                                       int32_t* info) {
  const int p = probs[blockIdx.x];
  SketchArgs a = args[p];
  a.info = info + 2 * p;
  to_global(a, args[p]);
  sketch_qr_generic_body<MAXN>(a);
}

template <int NMAX>
__global__ __launch_bounds__(kPassThreads, 2) void kb_passA(const PassAArgs* __restrict__ args,
                                                           const BatchItem* __restrict__ items, int32_t* info) {
  const BatchItem it = items[blockIdx.x];
  PassAArgs a = args[it.problem];
  a.info = info + 2 * it.problem;
  to_global(a, args[it.problem]);
  passA_body<NMAX>(a, it.local, it.count);
}

template <int NMAX>
__global__ __launch_bounds__(kCholThreads, 1) void kb_cholesky(const CholArgs* __restrict__ args,
                                                              const int32_t* __restrict__ probs, int32_t* info) {
  const int p = probs[blockIdx.x];
  CholArgs a = args[p];
  a.info = info + 2 * p;
  to_global(a, args[p]);
  cholesky_body<NMAX>(a);
}

template <int NMAX>
__global__ __launch_bounds__(kPassBThreads) void kb_passB(const PassBArgs* __restrict__ args,
                                                          const BatchItem* __restrict__ items, int32_t* info) {
  const BatchItem it = items[blockIdx.x];
  PassBArgs a = args[it.problem];
  a.info = info + 2 * it.problem;
  to_global(a, args[it.problem]);
  passB_body<NMAX>(a, it.local, it.count);
}

__global__ __launch_bounds__(kPassThreads, 2) void kb_passW(const PassAArgs* __restrict__ args,
                                                           const BatchItem* __restrict__ items, int32_t* info) {
  const BatchItem it = items[blockIdx.x];
  PassAArgs a = args[it.problem];
  a.info = info + 2 * it.problem;
  to_global(a, args[it.problem]);
  passW_body(a, it.local, it.count);
}

__global__ __launch_bounds__(kPassThreads) void kb_gramW(const PassAArgs* __restrict__ args,
                                                        const BatchItem* __restrict__ items, int32_t* info) {
  const BatchItem it = items[blockIdx.x];
  PassAArgs a = args[it.problem];
  a.info = info + 2 * it.problem;
  to_global(a, args[it.problem]);
  gramW_body(a, it.local, it.count);
}

__global__ __launch_bounds__(kPassB128Threads) void kb_passB128(const PassBArgs* __restrict__ args,
                                                               const BatchItem* __restrict__ items, int32_t* info) {
  const BatchItem it = items[blockIdx.x];
  PassBArgs a = args[it.problem];
  a.info = info + 2 * it.problem;
  to_global(a, args[it.problem]);
  passB128_body(a, it.local, it.count);
}

}  // namespace rpq

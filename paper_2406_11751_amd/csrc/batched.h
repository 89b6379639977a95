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

__global__ __launch_bounds__(kGatherThreads) void kb_gather(const SketchArgs* __restrict__ args,
                                                            const BatchItem* __restrict__ items) {
  const BatchItem it = items[blockIdx.x];
  const SketchArgs a = args[it.problem];
  gather_body(a, it.local);
}

template <int RPT>
__global__ __launch_bounds__(kSketchThreads) void kb_sketch_qr(const SketchArgs* __restrict__ args,
                                                               const int32_t* __restrict__ probs, int32_t* info) {
  const int p = probs[blockIdx.x];
  SketchArgs a = args[p];
  a.info = info + 2 * p;
  sketch_qr_body<RPT>(a);
}

template <int RPT>
__global__ __launch_bounds__(kSketchThreads) void kb_sketch_qr_wide(const SketchArgs* __restrict__ args,
                                                                    const int32_t* __restrict__ probs, int32_t* info) {
  const int p = probs[blockIdx.x];
  SketchArgs a = args[p];
  a.info = info + 2 * p;
  sketch_qr_body<RPT, true>(a);
}

template <int MAXN>
__global__ __launch_bounds__(kSketchThreads) void kb_sketch_qr_generic(const SketchArgs* __restrict__ args,
                                                                       const int32_t* __restrict__ probs,
                                                                       int32_t* info) {
  const int p = probs[blockIdx.x];
  SketchArgs a = args[p];
  a.info = info + 2 * p;
  sketch_qr_generic_body<MAXN>(a);
}

template <int NMAX>
__global__ __launch_bounds__(kPassThreads, 2) void kb_passA(const PassAArgs* __restrict__ args,
                                                           const BatchItem* __restrict__ items, int32_t* info) {
  const BatchItem it = items[blockIdx.x];
  PassAArgs a = args[it.problem];
  a.info = info + 2 * it.problem;
  passA_body<NMAX>(a, it.local, it.count);
}

template <int NMAX>
__global__ __launch_bounds__(kCholThreads, 1) void kb_cholesky(const CholArgs* __restrict__ args,
                                                              const int32_t* __restrict__ probs, int32_t* info) {
  const int p = probs[blockIdx.x];
  CholArgs a = args[p];
  a.info = info + 2 * p;
  cholesky_body<NMAX>(a);
}

template <int NMAX>
__global__ __launch_bounds__(kPassBThreads) void kb_passB(const PassBArgs* __restrict__ args,
                                                          const BatchItem* __restrict__ items, int32_t* info) {
  const BatchItem it = items[blockIdx.x];
  PassBArgs a = args[it.problem];
  a.info = info + 2 * it.problem;
  passB_body<NMAX>(a, it.local, it.count);
}

__global__ __launch_bounds__(kPassThreads, 2) void kb_passW(const PassAArgs* __restrict__ args,
                                                           const BatchItem* __restrict__ items, int32_t* info) {
  const BatchItem it = items[blockIdx.x];
  PassAArgs a = args[it.problem];
  a.info = info + 2 * it.problem;
  passW_body(a, it.local, it.count);
}

__global__ __launch_bounds__(kPassThreads) void kb_gramW(const PassAArgs* __restrict__ args,
                                                        const BatchItem* __restrict__ items, int32_t* info) {
  const BatchItem it = items[blockIdx.x];
  PassAArgs a = args[it.problem];
  a.info = info + 2 * it.problem;
  gramW_body(a, it.local, it.count);
}

__global__ __launch_bounds__(kPassB128Threads) void kb_passB128(const PassBArgs* __restrict__ args,
                                                               const BatchItem* __restrict__ items, int32_t* info) {
  const BatchItem it = items[blockIdx.x];
  PassBArgs a = args[it.problem];
  a.info = info + 2 * it.problem;
  passB128_body(a, it.local, it.count);
}

}  // namespace rpq

// Host side of the rpCholesky-QR library: argument checks, workspace layout,
// kernel selection and the launch sequence behind the C ABI in rpcholqr.h.
#include "../../include/rpcholqr.h"

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "passes.h"
#include "sketch.h"
#include "small.h"

namespace {

using namespace rpq;

constexpr int kMaxN = 64;
constexpr int kMaxSketchRows = 1536;  // generic sketch kernel keeps 2*s doubles in LDS
constexpr int kPassAMaxBlocks = 512;
static_assert(kPassAMaxBlocks <= kReduceChunk * kMaxPartial2, "second-level partial count");
constexpr int kPassBMaxBlocks = 2048;
// The LDS-staged ping-pong pass A (k_passA_pp) is built and tested but not the
// default: on MI355X it measures slower than the register-load kernel.
constexpr bool kStagedPassA = false;

struct Plan {
  int nmax = 0, NB = 0, E = 0;
  int64_t panels = 0;
  int PA = 0, PB = 0, G2 = 0;
  int rpt = 0;  // sample rows per lane in the register sketch QR; 0 = generic kernel
  size_t off_tri = 0, off_tri2 = 0, off_Rs = 0, off_part = 0, off_part2 = 0, off_As = 0;
  size_t total = 0;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int pick_nmax(int64_t n) {
  if (n <= 16) return 16;
  if (n <= 32) return 32;
  if (n <= 48) return 48;
  return 64;
}

bool make_plan(int64_t m, int64_t n, int64_t s, Plan* p) {
  if (n < 1 || m < n || s < n || n > kMaxN) return false;
  p->nmax = pick_nmax(n);
  p->NB = (p->nmax + 15) / 16;
  p->E = p->NB * (p->NB + 1) / 2 * 256;
  p->panels = (m + kWave - 1) / kWave;
  const int64_t blocks = (p->panels + kPassWaves - 1) / kPassWaves;
  p->PA = (int)(blocks < kPassAMaxBlocks ? blocks : kPassAMaxBlocks);
  const int64_t bblocks = ((m + 15) / 16 + kPassBThreads / kWave - 1) / (kPassBThreads / kWave);
  p->PB = (int)(bblocks < kPassBMaxBlocks ? bblocks : kPassBMaxBlocks);
  p->G2 = (p->PA + kReduceChunk - 1) / kReduceChunk;  // <= kMaxPartial2 since PA <= 512
  const int64_t rows = (s + 15) / 16;
  p->rpt = rows <= 4 ? 4 : rows <= 8 ? 8 : rows <= 12 ? 12 : rows <= 16 ? 16 : rows <= 24 ? 24 : 0;
  if (p->rpt == 0 && s > kMaxSketchRows) return false;
  const size_t tri = (size_t)p->nmax * (p->nmax + 1) / 2 * sizeof(double);
  size_t off = 0;
  p->off_tri = off;
  off = align256(off + tri);
  p->off_tri2 = off;
  off = align256(off + (size_t)p->nmax * p->nmax * sizeof(double));
  p->off_Rs = off;
  off = align256(off + (size_t)n * n * sizeof(double));
  p->off_part = off;
  off = align256(off + (size_t)p->PA * p->E * sizeof(double));
  p->off_part2 = off;
  off = align256(off + (size_t)p->G2 * p->E * sizeof(double));
  p->off_As = off;
  off = align256(off + (size_t)s * n * sizeof(double));
  p->total = off;
  return true;
}

bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + bbytes && b0 < a0 + abytes;
}

size_t span_bytes(int64_t rows, int64_t cols, int64_t ld) {
  return ((size_t)ld * (size_t)(cols - 1) + (size_t)rows) * sizeof(double);
}

void launch_sketch(const Plan& p, const SketchArgs& a, hipStream_t st) {
  const dim3 blk(kSketchThreads);
  switch (p.rpt) {
    case 4: hipLaunchKernelGGL((k_sketch_qr<4>), dim3(1), blk, 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_sketch_qr<8>), dim3(1), blk, 0, st, a); break;
    case 12: hipLaunchKernelGGL((k_sketch_qr<12>), dim3(1), blk, 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_sketch_qr<16>), dim3(1), blk, 0, st, a); break;
    case 24: hipLaunchKernelGGL((k_sketch_qr<24>), dim3(1), blk, 0, st, a); break;
    default:
      hipLaunchKernelGGL(k_sketch_qr_generic, dim3(1), blk, 2 * (size_t)a.s * sizeof(double), st, a);
      break;
  }
}

// Compute units of the current device (cached per device).
int device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 0;
  if (dev < 64) {
    const int c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (dev < 64) cache[dev].store(cus, std::memory_order_relaxed);
  return cus;
}

// Pass A launch: the LDS-staged kernel when columns are 16-byte aligned, with
// one wave of work per SIMD slot the LDS allows; else the register kernel.
// Returns the number of workgroups launched (= Gram partials written), 0 on error.
template <int NMAX>
int launch_passes_A(const Plan& p, const PassAArgs& a, hipStream_t st) {
  const bool aligned = ((uintptr_t)a.A % 16 == 0) && (a.lda % 2 == 0);
  const int cus = kStagedPassA ? device_cus() : 0;
  if (kStagedPassA && aligned && cus > 0) {
    const int64_t pgroups = (p.panels + kPPWaves - 1) / kPPWaves;
    const int64_t slots = (int64_t)cus * PassAPP<NMAX>::OCC;
    int64_t grid = pgroups < slots ? pgroups : slots;
    if (grid > p.PA) grid = p.PA;
    hipLaunchKernelGGL((k_passA_pp<NMAX>), dim3((unsigned)grid), dim3(kPPThreads), 0, st, a);
    return (int)grid;
  }
  hipLaunchKernelGGL((k_passA_mfma<NMAX>), dim3(p.PA), dim3(kPassThreads), 0, st, a);
  return p.PA;
}

template <int NMAX>
void launch_pass_B(const Plan& p, const PassBArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_passB<NMAX>), dim3(p.PB), dim3(kPassBThreads), 0, st, a);
}

// Event timing (rpcholqr_timing_*): one set of NSTAGES+1 events per recorded call.
struct Timing {
  bool on = false;
  std::vector<std::array<hipEvent_t, RPCHOLQR_NSTAGES + 1>> sets;
  size_t used = 0;
};
Timing g_timing;

hipEvent_t* timing_slot() {
  if (!g_timing.on) return nullptr;
  if (g_timing.used == g_timing.sets.size()) {
    std::array<hipEvent_t, RPCHOLQR_NSTAGES + 1> ev{};
    for (auto& e : ev)
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_timing.sets.push_back(ev);
  }
  return g_timing.sets[g_timing.used++].data();
}

int32_t factor_impl(int64_t m, int64_t n, int64_t s, uint64_t seed, const double* A, int64_t lda,
                    double* Q, int64_t ldq, double* R, int64_t ldr, int32_t precision, void* ws,
                    size_t ws_bytes, rpcholqr_info* info, void* stream, int64_t* idx, double* As,
                    double* Rs, double* A1, double* G1, double* R2) {
  if (n < 1 || m < n || s < n || lda < m || ldq < m || ldr < n) return RPCHOLQR_EINVAL;
  if (!A || !Q || !R || !info) return RPCHOLQR_EINVAL;
  if (s > INT32_MAX) return RPCHOLQR_EUNSUPPORTED;
  if (precision != RPCHOLQR_FP64) return RPCHOLQR_EUNSUPPORTED;
  Plan p;
  if (!make_plan(m, n, s, &p)) return RPCHOLQR_EUNSUPPORTED;
  const size_t a_bytes = span_bytes(m, n, lda), q_bytes = span_bytes(m, n, ldq), r_bytes = span_bytes(n, n, ldr);
  if (overlaps(A, a_bytes, Q, q_bytes) || overlaps(A, a_bytes, R, r_bytes) || overlaps(Q, q_bytes, R, r_bytes))
    return RPCHOLQR_EINVAL;
  if (!ws || ws_bytes < p.total || ((uintptr_t)ws & 255)) return RPCHOLQR_EWORKSPACE;
  if (overlaps(ws, p.total, A, a_bytes) || overlaps(ws, p.total, Q, q_bytes) || overlaps(ws, p.total, R, r_bytes))
    return RPCHOLQR_EINVAL;

  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  double* tri = (double*)(base + p.off_tri);
  double* tri2 = (double*)(base + p.off_tri2);
  double* Rs_ws = (double*)(base + p.off_Rs);
  double* part = (double*)(base + p.off_part);
  double* part2 = (double*)(base + p.off_part2);
  int32_t* inf = (int32_t*)info;
  hipEvent_t* ev = timing_slot();
  int stage = 0;
  auto mark = [&]() {
    if (ev) (void)hipEventRecord(ev[stage++], st);
  };
  mark();

  // Lines 2-3: sample, gather, sketch QR.
  SketchArgs sa;
  sa.m = m;
  sa.n = (int32_t)n;
  sa.s = (int32_t)s;
  sa.seed = seed;
  sa.scale = std::sqrt((double)m / (double)s);
  sa.A = A;
  sa.lda = lda;
  sa.tri = tri;
  sa.Rs = Rs_ws;
  sa.nmax = p.nmax;
  sa.info = inf;
  sa.As = (double*)(base + p.off_As);
  sa.idx_out = idx;
  sa.As_out = As;
  sa.Rs_out = Rs;
  const int64_t gather_blocks = ((int64_t)s * n + kGatherThreads - 1) / kGatherThreads;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)gather_blocks), dim3(kGatherThreads), 0, st, sa);
  if (hipGetLastError() != hipSuccess) return RPCHOLQR_EHIP;
  launch_sketch(p, sa, st);
  if (hipGetLastError() != hipSuccess) return RPCHOLQR_EHIP;
  mark();

  // Lines 4 (A1 = A R_s^{-1}) and 5 (Gram partials).
  PassAArgs pa;
  pa.m = m;
  pa.n = (int32_t)n;
  pa.A = A;
  pa.lda = lda;
  pa.tri_s = tri;
  pa.partials = part;
  pa.info = inf;
  pa.W = Q;
  pa.ldw = ldq;
  int pa_grid = 0;
  switch (p.nmax) {
    case 16: pa_grid = launch_passes_A<16>(p, pa, st); break;
    case 32: pa_grid = launch_passes_A<32>(p, pa, st); break;
    case 48: pa_grid = launch_passes_A<48>(p, pa, st); break;
    default: pa_grid = launch_passes_A<64>(p, pa, st); break;
  }
  if (hipGetLastError() != hipSuccess) return RPCHOLQR_EHIP;
  const int g2 = (pa_grid + kReduceChunk - 1) / kReduceChunk;  // <= p.G2
  mark();
  if (A1 && hipMemcpy2DAsync(A1, (size_t)m * sizeof(double), Q, (size_t)ldq * sizeof(double),
                             (size_t)m * sizeof(double), (size_t)n, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return RPCHOLQR_EHIP;

  hipLaunchKernelGGL(k_reduce_partials, dim3((p.E + kReduceThreads - 1) / kReduceThreads, g2),
                     dim3(kReduceThreads), 0, st, (const double*)part, pa_grid, p.E, part2, (const int32_t*)inf);
  if (hipGetLastError() != hipSuccess) return RPCHOLQR_EHIP;
  mark();

  // Lines 5-6 (Cholesky) and 8 (R = R2 R_s).
  CholArgs ca;
  ca.partial2 = part2;
  ca.G2 = g2;
  ca.E = p.E;
  ca.NB = p.NB;
  ca.n = (int32_t)n;
  ca.nmax = p.nmax;
  ca.Rs = Rs_ws;
  ca.T2 = tri2;
  ca.R = R;
  ca.ldr = ldr;
  ca.info = inf;
  ca.G1_out = G1;
  ca.R2_out = R2;
  switch (p.nmax) {
    case 16: hipLaunchKernelGGL((k_cholesky<16>), dim3(1), dim3(kCholThreads), 0, st, ca); break;
    case 32: hipLaunchKernelGGL((k_cholesky<32>), dim3(1), dim3(kCholThreads), 0, st, ca); break;
    case 48: hipLaunchKernelGGL((k_cholesky<48>), dim3(1), dim3(kCholThreads), 0, st, ca); break;
    default: hipLaunchKernelGGL((k_cholesky<64>), dim3(1), dim3(kCholThreads), 0, st, ca); break;
  }
  if (hipGetLastError() != hipSuccess) return RPCHOLQR_EHIP;
  mark();

  // Line 6: Q = A1 R2^{-1}, A1 recomputed from A.
  PassBArgs pb;
  pb.m = m;
  pb.n = (int32_t)n;
  pb.T2 = tri2;
  pb.Q = Q;
  pb.ldq = ldq;
  pb.info = inf;
  switch (p.nmax) {
    case 16: launch_pass_B<16>(p, pb, st); break;
    case 32: launch_pass_B<32>(p, pb, st); break;
    case 48: launch_pass_B<48>(p, pb, st); break;
    default: launch_pass_B<64>(p, pb, st); break;
  }
  if (hipGetLastError() != hipSuccess) return RPCHOLQR_EHIP;
  mark();
  return RPCHOLQR_OK;
}

}  // namespace

extern "C" {

int32_t rpcholqr_max_n(void) { return kMaxN; }

size_t rpcholqr_workspace_bytes(int64_t m, int64_t n, int64_t s, int32_t precision) {
  if (precision != RPCHOLQR_FP64) return 0;
  Plan p;
  if (!make_plan(m, n, s, &p)) return 0;
  return p.total;
}

int32_t rpcholqr_factor(int64_t m, int64_t n, int64_t s, uint64_t seed, const double* A, int64_t lda,
                        double* Q, int64_t ldq, double* R, int64_t ldr, int32_t precision,
                        void* workspace, size_t workspace_bytes, rpcholqr_info* info, void* stream) {
  return factor_impl(m, n, s, seed, A, lda, Q, ldq, R, ldr, precision, workspace, workspace_bytes, info,
                     stream, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
}

int32_t rpcholqr_factor_debug(int64_t m, int64_t n, int64_t s, uint64_t seed, const double* A,
                              int64_t lda, double* Q, int64_t ldq, double* R, int64_t ldr,
                              int32_t precision, void* workspace, size_t workspace_bytes,
                              rpcholqr_info* info, void* stream, int64_t* idx, double* As, double* Rs,
                              double* A1, double* G1, double* R2) {
  return factor_impl(m, n, s, seed, A, lda, Q, ldq, R, ldr, precision, workspace, workspace_bytes, info,
                     stream, idx, As, Rs, A1, G1, R2);
}

int32_t rpcholqr_timing_enable(int32_t on) {
  g_timing.on = on != 0;
  g_timing.used = 0;
  return RPCHOLQR_OK;
}

int32_t rpcholqr_timing_read(double* ms, int32_t count) {
  if (!ms || count < 0) return RPCHOLQR_EINVAL;
  for (int i = 0; i < count; ++i) ms[i] = 0.0;
  const size_t calls = g_timing.used;
  for (size_t c = 0; c < calls; ++c) {
    auto& ev = g_timing.sets[c];
    if (hipEventSynchronize(ev[RPCHOLQR_NSTAGES]) != hipSuccess) return RPCHOLQR_EHIP;
    for (int i = 0; i < RPCHOLQR_NSTAGES && i < count; ++i) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) != hipSuccess) return RPCHOLQR_EHIP;
      ms[i] += t;
    }
  }
  g_timing.used = 0;
  return (int32_t)calls;
}

}  // extern "C"

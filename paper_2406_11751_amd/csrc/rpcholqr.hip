// Host side of the rpCholesky-QR library: argument checks, workspace layout,
// kernel selection and the launch sequence behind the C ABI in rpcholqr.h.
#include "../../include/rpcholqr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <map>
#include <mutex>
#include <type_traits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "passes.h"
#include "sketch.h"
#include "small.h"
#include "wide.h"
#include "big.h"
#include "smooth.h"
#include "batched.h"

namespace {

using namespace rpq;

constexpr int kMaxN = kBigMaxN;
constexpr int kWideN = 128;  // column class of 64 < n <= 128 (two-half row solve, separate Gram pass)
constexpr int kMaxSketchRows = 1536;  // generic sketch kernel keeps 2*s doubles in LDS
constexpr int kPassAMaxBlocks = 512;
static_assert(kPassAMaxBlocks <= kReduceChunk * kMaxPartial2, "second-level partial count");
constexpr int kPassBMaxBlocks = 2048;

struct Plan {
  int nmax = 0, NB = 0, E = 0;
  int64_t panels = 0;
  int PA = 0, PB = 0, G2 = 0;
  int rpt = 0;  // sample rows per lane in the register sketch QR; 0 = generic kernel
  size_t off_tri = 0, off_tri2 = 0, off_tri3 = 0, off_Rs = 0, off_part = 0, off_part2 = 0, off_As = 0, off_R1 = 0, off_R2 = 0;
  size_t total = 0;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int pick_nmax(int64_t n) {
  if (n <= 16) return 16;
  if (n <= 32) return 32;
  if (n <= 48) return 48;
  if (n <= 64) return 64;
  return kWideN;
}

// Workspace layout of one problem.  pa_cap bounds the number of pass-A
// workgroups (= Gram partials).  With direct_partials the Cholesky kernel sums
// the partials itself (no second-level region; the batched path, pa_cap <= 64).
bool make_plan(int64_t m, int64_t n, int64_t s, Plan* p, int64_t pa_cap = kPassAMaxBlocks,
               bool direct_partials = false, bool refine = false) {
  if (n < 1 || m < n || s < n || n > kWideN) return false;
  p->nmax = pick_nmax(n);
  if (p->nmax == kWideN && refine) return false;  // refined precisions: n <= 64
  p->NB = (p->nmax + 15) / 16;
  p->E = p->NB * (p->NB + 1) / 2 * 256;
  p->panels = (m + kWave - 1) / kWave;
  const int64_t blocks = (p->panels + kPassWaves - 1) / kPassWaves;
  p->PA = (int)(blocks < pa_cap ? blocks : pa_cap);
  const int64_t bblocks = ((m + 15) / 16 + kPassBThreads / kWave - 1) / (kPassBThreads / kWave);
  p->PB = (int)(bblocks < kPassBMaxBlocks ? bblocks : kPassBMaxBlocks);
  p->G2 = direct_partials ? p->PA : (p->PA + kReduceChunk - 1) / kReduceChunk;
  const int64_t rows = (s + 15) / 16;
  p->rpt = rows <= 4 ? 4 : rows <= 8 ? 8 : rows <= 12 ? 12 : rows <= 16 ? 16 : rows <= 24 ? 24 : 0;
  if (p->nmax == kWideN && p->rpt > 0 && p->rpt < 8) p->rpt = 8;  // rows 64..127 live in slots 4..7
  if (p->rpt == 0 && s > kMaxSketchRows) return false;
  // nmax <= 64: one packed triangle; nmax = 128: R11, R22 packed and R12 64 x 64,
  // 2 * 2080 + 4096 = 128 * 129 / 2 doubles as well.
  const size_t tri = (size_t)p->nmax * (p->nmax + 1) / 2 * sizeof(double);
  size_t off = 0;
  p->off_tri = off;
  off = align256(off + tri);
  p->off_tri2 = off;
  off = align256(off + (size_t)p->nmax * p->nmax * sizeof(double));
  p->off_tri3 = off;  // R2 as row-solve operands (substitution form of line 6)
  off = align256(off + tri);
  p->off_Rs = off;
  off = align256(off + (size_t)n * n * sizeof(double));
  p->off_part = off;
  off = align256(off + (size_t)p->PA * p->E * sizeof(double));
  p->off_part2 = off;
  if (!direct_partials) off = align256(off + (size_t)p->G2 * p->E * sizeof(double));
  p->off_As = off;
  off = align256(off + (size_t)s * n * sizeof(double));
  p->off_R1 = off;  // refined precisions: R2 R_s of the first pass, n x n, ld n
  if (refine) off = align256(off + (size_t)n * n * sizeof(double));
  p->off_R2 = off;  // R2 for the substitution form of line 6, n x n, ld n
  off = align256(off + (size_t)n * n * sizeof(double));
  p->total = off;
  return true;
}

// Plan of the columns class 128 < n <= 512 (big.h).  nmax = 128 ceil(n/128).
struct BigPlan {
  int nmax = 0, NB = 0, NP = 0, rpt = 0, ngroups = 0, nsplit = 0, G2 = 0;
  int wl = 0;  // rpt == 0: rows per lane and lane row of the wave-per-column sketch (0: streaming)
  int64_t E = 0;
  size_t off_tri = 0, off_full = 0, off_T2 = 0, off_tri3 = 0, off_full3 = 0, off_Gg = 0, off_Rs = 0, off_Rg = 0,
         off_tau = 0, off_part = 0, off_part2 = 0, off_As = 0;
  size_t total = 0;
};

bool make_big_plan(int64_t m, int64_t n, int64_t s, BigPlan* p, int64_t pa_cap = kPassAMaxBlocks,
                   bool refine = false) {
  if (n <= kWideN || n > kBigMaxN || m < n || s < n || refine) return false;
  if (s > kGmMaxRows) return false;  // s > 16 * 96: the streaming panel sketch
  p->nmax = (int)((n + kBigBlock - 1) / kBigBlock) * kBigBlock;
  p->NB = p->nmax / 16;
  p->NP = p->nmax / kWH;
  p->E = (int64_t)p->NB * (p->NB + 1) / 2 * 256;
  const int64_t rows = (s + 15) / 16;
  p->rpt = rows <= 16 ? 16 : rows <= 24 ? 24 : rows <= 32 ? 32 : rows <= 48 ? 48 : rows <= 64 ? 64 : rows <= 96 ? 96 : 0;
  const int64_t wl = (rows + 3) / 4;
  p->wl = p->rpt > 0 ? 0 : wl <= 32 ? 32 : wl <= 64 ? 64 : wl <= 96 ? 96 : 0;
  const int ng = p->nmax / kBigBlock;
  p->ngroups = ng * (ng - 1) / 2 + (ng + 1) / 2;  // k_gram_big groups: off-diagonal pairs, diagonal pairs
  const int64_t rblocks = (m + kGRows - 1) / kGRows;
  // row splits of the Gram: about 2048 workgroups in all (1024 measured 2-3 % slower at
  // 384 and 768 columns, the same at 256 and 512)
  int64_t ns = (2048 + p->ngroups - 1) / p->ngroups;
  ns = std::min<int64_t>(std::min<int64_t>(ns, rblocks), std::min<int64_t>(pa_cap, kPassAMaxBlocks));
  if (ns >= kXcds) ns -= ns % kXcds;  // XCD-aware Gram schedule (k_gram_big)
  p->nsplit = (int)std::max<int64_t>(ns, 1);
  p->G2 = (p->nsplit + kReduceChunk - 1) / kReduceChunk;
  const size_t d = sizeof(double), nm = (size_t)p->nmax;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  p->off_tri = take((size_t)p->NP * kBigTri * d);
  p->off_full = take(nm * nm * d);
  p->off_T2 = take(nm * nm * d);
  p->off_tri3 = take((size_t)p->NP * kBigTri * d);
  p->off_full3 = take(nm * nm * d);
  p->off_Gg = take(nm * (nm + 1) * d);
  p->off_Rs = take((size_t)n * n * d);
  p->off_Rg = take((size_t)n * n * d);
  p->off_tau = take((size_t)n * d);
  p->off_part = take((size_t)p->nsplit * p->E * d);
  p->off_part2 = take((size_t)p->G2 * p->E * d);
  p->off_As = take((size_t)s * n * d);
  p->total = off;
  return true;
}

// Chunk sums of the smoothed sample (smooth.h): [chunks][n][s] doubles.
size_t smooth_bytes(int64_t m, int64_t n, int64_t s) {
  const int64_t chunk = smooth_chunk_rows(m), chunks = (m + chunk - 1) / chunk;
  return align256((size_t)chunks * (size_t)n * (size_t)s * sizeof(double));
}

// Workspace bytes for any supported size (0 if unsupported); with smoothing the
// chunk sums follow the plan's own region.
size_t plan_total(int64_t m, int64_t n, int64_t s, int64_t pa_cap, bool refine, bool smooth = false) {
  size_t total = 0;
  if (n > kWideN) {
    BigPlan b;
    if (!make_big_plan(m, n, s, &b, pa_cap, refine)) return 0;
    total = b.total;
  } else {
    Plan p;
    if (!make_plan(m, n, s, &p, pa_cap, false, refine)) return 0;
    total = p.total;
  }
  return total + (smooth ? smooth_bytes(m, n, s) : 0);
}

bool is_refine(int32_t prec) { return prec == RPCHOLQR_FP32_REFINE || prec == RPCHOLQR_BF16X2_REFINE; }

// Workspace bytes for a precision value (RPCHOLQR_SMOOTH masked off); 0 when
// the combination is not supported.
size_t precision_total(int64_t m, int64_t n, int64_t s, int64_t pa_cap, int32_t prec, bool smooth) {
  if (prec != RPCHOLQR_FP64 && !is_refine(prec) && prec != RPCHOLQR_A1_FP32) return 0;
  if (prec == RPCHOLQR_A1_FP32 && n > kSketchMaxN) return 0;
  return plan_total(m, n, s, pa_cap, is_refine(prec), smooth);
}

// Line 2: the sample A_s into sa.As (and the optional idx / As copies): the
// rows of A themselves (F = I), or the rows of the smoothed F [A; 0]
// (smooth.h) with its chunk sums in smooth_ws.
bool launch_sample(const SketchArgs& sa, bool smooth, double* smooth_ws, hipStream_t st) {
  const int64_t m = sa.m, n = sa.n, s = sa.s;
  if (!smooth) {
    const int64_t gather_blocks = (s * n + kGatherThreads - 1) / kGatherThreads;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)gather_blocks), dim3(kGatherThreads), 0, st, sa);
    return hipGetLastError() == hipSuccess;
  }
  SmoothArgs ma{};
  ma.m = m;
  ma.n = (int32_t)n;
  ma.s = (int32_t)s;
  ma.seed = sa.seed;
  ma.M = smooth_padded_rows(m);
  ma.chunk = smooth_chunk_rows(m);
  ma.nchunks = (int32_t)((m + ma.chunk - 1) / ma.chunk);
  ma.scale = 1.0 / std::sqrt((double)s);
  ma.A = sa.A;
  ma.lda = sa.lda;
  ma.partials = smooth_ws;
  ma.As = sa.As;
  ma.idx_out = sa.idx_out;
  ma.As_out = sa.As_out;
  const int64_t nrb = (s + 15) / 16;
  const dim3 grid((unsigned)ma.nchunks, (unsigned)((n + 15) / 16),
                  (unsigned)((nrb + kPassWaves * kSmoothTPW - 1) / (kPassWaves * kSmoothTPW)));
  hipLaunchKernelGGL(k_smooth_partials, grid, dim3(kSmoothThreads), 0, st, ma);
  hipLaunchKernelGGL(k_smooth_finish, dim3((unsigned)((s * n + kSmoothThreads - 1) / kSmoothThreads)),
                     dim3(kSmoothThreads), 0, st, ma);
  return hipGetLastError() == hipSuccess;
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
  if (p.nmax == kWideN && p.rpt > 0) {
    switch (p.rpt) {
      case 8: hipLaunchKernelGGL((k_sketch_qr_wide<8>), dim3(1), blk, 0, st, a); break;
      case 12: hipLaunchKernelGGL((k_sketch_qr_wide<12>), dim3(1), blk, 0, st, a); break;
      case 16: hipLaunchKernelGGL((k_sketch_qr_wide<16>), dim3(1), blk, 0, st, a); break;
      default: hipLaunchKernelGGL((k_sketch_qr_wide<24>), dim3(1), blk, 0, st, a); break;
    }
    return;
  }
  switch (p.rpt) {
    case 4: hipLaunchKernelGGL((k_sketch_qr<4>), dim3(1), blk, 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_sketch_qr<8>), dim3(1), blk, 0, st, a); break;
    case 12: hipLaunchKernelGGL((k_sketch_qr<12>), dim3(1), blk, 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_sketch_qr<16>), dim3(1), blk, 0, st, a); break;
    case 24: hipLaunchKernelGGL((k_sketch_qr<24>), dim3(1), blk, 0, st, a); break;
    default:
      if (p.nmax == kWideN)
        hipLaunchKernelGGL((k_sketch_qr_generic<kWideN>), dim3(1), blk, 2 * (size_t)a.s * sizeof(double), st, a);
      else
        hipLaunchKernelGGL((k_sketch_qr_generic<64>), dim3(1), blk, 2 * (size_t)a.s * sizeof(double), st, a);
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

// Pass A launch.  Returns the number of workgroups launched (= Gram partials
// written).
template <int NMAX, int MODE = kSolveGram, int GP = kGramF64, bool F32A1 = false>
int launch_passes_A(const Plan& p, const PassAArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_passA_mfma<NMAX, MODE, GP, F32A1>), dim3(p.PA), dim3(kPassThreads), 0, st, a);
  return p.PA;
}

template <int NMAX, bool F32A1 = false>
void launch_pass_B(const Plan& p, const PassBArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_passB<NMAX, F32A1>), dim3(p.PB), dim3(kPassBThreads), 0, st, a);
}

// Pass A for 64 < n <= 128: the two-half row solve, then the Gram pass.
// Returns the number of Gram partials written.
int launch_passes_A_wide(const Plan& p, const PassAArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_passW, dim3(p.PA), dim3(kPassThreads), 0, st, a);
  hipLaunchKernelGGL(k_gramW, dim3(p.PA), dim3(kPassThreads), 0, st, a);
  return p.PA;
}

// Pass B for 64 < n <= 128: R2^{-1} takes 128 KB of LDS, one workgroup per CU.
void launch_pass_B_wide(int64_t m, const PassBArgs& a, hipStream_t st) {
  const int64_t groups = ((m + 15) / 16 + kPassB128Waves - 1) / kPassB128Waves;
  const int cus = device_cus();
  const int64_t cap = cus > 0 ? cus : 256;
  const int64_t grid = groups < cap ? groups : cap;
  hipLaunchKernelGGL(k_passB128, dim3((unsigned)grid), dim3(kPassB128Threads), 0, st, a);
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

// Calls fn(std::integral_constant<int, NMAX>) for the plan's NMAX.
template <typename F>
void with_nmax(int nmax, F&& fn) {
  switch (nmax) {
    case 16: fn(std::integral_constant<int, 16>{}); break;
    case 32: fn(std::integral_constant<int, 32>{}); break;
    case 48: fn(std::integral_constant<int, 48>{}); break;
    default: fn(std::integral_constant<int, 64>{}); break;
  }
}

template <typename F>
void with_big_nmax(int nmax, F&& fn) {
  switch (nmax) {
    case 256: fn(std::integral_constant<int, 256>{}); break;
    case 384: fn(std::integral_constant<int, 384>{}); break;
    case 512: fn(std::integral_constant<int, 512>{}); break;
    case 640: fn(std::integral_constant<int, 640>{}); break;
    case 768: fn(std::integral_constant<int, 768>{}); break;
    case 896: fn(std::integral_constant<int, 896>{}); break;
    default: fn(std::integral_constant<int, 1024>{}); break;
  }
}

template <typename F>
void with_big_rpt(int rpt, F&& fn) {
  switch (rpt) {
    case 16: fn(std::integral_constant<int, 16>{}); break;
    case 24: fn(std::integral_constant<int, 24>{}); break;
    case 32: fn(std::integral_constant<int, 32>{}); break;
    case 48: fn(std::integral_constant<int, 48>{}); break;
    case 64: fn(std::integral_constant<int, 64>{}); break;
    default: fn(std::integral_constant<int, 96>{}); break;
  }
}

// The 128 < n <= 512 class (big.h); arguments as factor_impl, already checked
// for sizes, pointers and precision.
int32_t factor_big(int64_t m, int64_t n, int64_t s, uint64_t seed, const double* A, int64_t lda, double* Q,
                   int64_t ldq, double* R, int64_t ldr, int32_t precision, void* ws, size_t ws_bytes,
                   rpcholqr_info* info, void* stream, int64_t* idx, double* As, double* Rs, double* A1, double* G1,
                   double* R2, const double* Rs_in, int64_t ldrs, int64_t pa_cap, bool timed, bool smooth) {
  BigPlan p;
  if (!make_big_plan(m, n, s, &p, pa_cap, precision != RPCHOLQR_FP64)) return RPCHOLQR_EUNSUPPORTED;
  const size_t a_bytes = span_bytes(m, n, lda), q_bytes = span_bytes(m, n, ldq), r_bytes = span_bytes(n, n, ldr);
  if (overlaps(A, a_bytes, Q, q_bytes) || overlaps(A, a_bytes, R, r_bytes) || overlaps(Q, q_bytes, R, r_bytes))
    return RPCHOLQR_EINVAL;
  const size_t total = p.total + (smooth ? smooth_bytes(m, n, s) : 0);
  if (!ws || ws_bytes < total || ((uintptr_t)ws & 255)) return RPCHOLQR_EWORKSPACE;
  if (overlaps(ws, total, A, a_bytes) || overlaps(ws, total, Q, q_bytes) || overlaps(ws, total, R, r_bytes))
    return RPCHOLQR_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  auto at_ws = [&](size_t off) { return (double*)(base + off); };
  int32_t* inf = (int32_t*)info;
  hipEvent_t* ev = timed ? timing_slot() : nullptr;
  int stage = 0;
  auto mark = [&]() {
    if (ev) (void)hipEventRecord(ev[stage++], st);
  };
  auto launched = [&]() { return hipGetLastError() == hipSuccess; };
  mark();

  // Lines 2-3: sample and gather, then the panel sketch QR, then R_s and the
  // row-solve operands.  With Rs_in the finishing kernel takes the caller's R_s.
  BigFinishArgs fa{};
  fa.n = (int32_t)n;
  fa.nmax = p.nmax;
  fa.Rs = at_ws(p.off_Rs);
  fa.Rs_out = Rs;
  fa.tri = at_ws(p.off_tri);
  fa.full = at_ws(p.off_full);
  fa.info = inf;
  if (Rs_in) {
    fa.Rg = Rs_in;
    fa.rs_k = 1;
    fa.rs_j = ldrs;
    fa.normalize = 0;
    fa.init_info = 1;
  } else {
    SketchArgs sa{};
    sa.m = m;
    sa.n = (int32_t)n;
    sa.s = (int32_t)s;
    sa.seed = seed;
    sa.scale = std::sqrt((double)m / (double)s);
    sa.A = A;
    sa.lda = lda;
    sa.As = at_ws(p.off_As);
    sa.info = inf;
    sa.idx_out = idx;
    sa.As_out = As;
    if (!launch_sample(sa, smooth, at_ws(p.total), st)) return RPCHOLQR_EHIP;
    BigSketchArgs ba{};
    ba.n = (int32_t)n;
    ba.s = (int32_t)s;
    ba.As = at_ws(p.off_As);
    ba.tau = at_ws(p.off_tau);
    ba.Rg = at_ws(p.off_Rg);
    ba.info = inf;
    if (p.rpt == 0 && p.wl > 0) {
      auto run = [&](auto wl) {
        constexpr int L = decltype(wl)::value, kWPW = w_pw<L>(), kWThreads = kWave * kWPW;
        ba.pw = kWPW;
        for (int c0 = 0; c0 < n; c0 += kWPW) {
          ba.c0 = c0;
          hipLaunchKernelGGL((k_sketch_panel_w<L>), dim3(1), dim3(kWThreads), 0, st, ba);
          const int64_t trail = n - std::min<int64_t>(c0 + kWPW, n);
          if (trail > 0)
            hipLaunchKernelGGL((k_sketch_trail_w<L>), dim3((unsigned)((trail + kWPW - 1) / kWPW)), dim3(kWThreads), 0,
                               st, ba);
        }
      };
      if (p.wl == 32)
        run(std::integral_constant<int, 32>{});
      else if (p.wl == 64)
        run(std::integral_constant<int, 64>{});
      else
        run(std::integral_constant<int, 96>{});
    } else if (p.rpt == 0) {
      ba.pw = kGmPW;
      for (int c0 = 0; c0 < n; c0 += kGmPW) {
        ba.c0 = c0;
        hipLaunchKernelGGL(k_sketch_panel_gm, dim3(1), dim3(kGmThreads), 0, st, ba);
        const int64_t trail = n - std::min<int64_t>(c0 + kGmPW, n);
        if (trail > 0)
          hipLaunchKernelGGL(k_sketch_trail_gm, dim3((unsigned)((trail + kGmPW - 1) / kGmPW)), dim3(kGmThreads), 0,
                             st, ba);
      }
    } else {
      with_big_rpt(p.rpt, [&](auto rp) {
        constexpr int RPT = decltype(rp)::value;
        constexpr int PW = panel_width<RPT>();
        ba.pw = PW;
        for (int c0 = 0; c0 < n; c0 += PW) {
          ba.c0 = c0;
          hipLaunchKernelGGL((k_sketch_panel<RPT>), dim3(1), dim3(16 * PW), 0, st, ba);
          const int64_t trail = n - std::min<int64_t>(c0 + PW, n);
          if (trail > 0)
            hipLaunchKernelGGL((k_sketch_trail<RPT>), dim3((unsigned)((trail + 15) / 16)), dim3(kTrailThreads), 0,
                               st, ba);
        }
      });
    }
    fa.Rg = at_ws(p.off_Rg);
    fa.rs_k = n;
    fa.rs_j = 1;
    fa.normalize = 1;
    fa.init_info = 0;
  }
  hipLaunchKernelGGL(k_big_finish, dim3(1), dim3(1024), 0, st, fa);
  if (!launched()) return RPCHOLQR_EHIP;
  mark();

  // Line 2 (A1 = A R_s^{-1} into Q, one launch per 64-column panel) and line 4 (Gram partials).
  const int cus = std::max(device_cus(), 1);
  const int64_t pgroups = ((m + kWave - 1) / kWave + kPassWaves - 1) / kPassWaves;
  const unsigned trsm_grid = (unsigned)std::min<int64_t>(pgroups, 2 * cus);
  auto trsm = [&](const double* src, int64_t ldsrc, const double* tri, const double* full) {
    BigTrsmArgs ta{};
    ta.m = m;
    ta.n = (int32_t)n;
    ta.nmax = p.nmax;
    ta.A = src;
    ta.lda = ldsrc;
    ta.W = Q;
    ta.ldw = ldq;
    ta.tri = tri;
    ta.full = full;
    ta.info = inf;
    for (int P = 0; P * kWH < n; ++P) {
      ta.P = P;
      hipLaunchKernelGGL(k_trsm_panel, dim3(trsm_grid), dim3(kPassThreads), 0, st, ta);
    }
  };
  trsm(A, lda, at_ws(p.off_tri), at_ws(p.off_full));
  BigGramArgs ga{};
  ga.m = m;
  ga.n = (int32_t)n;
  ga.nmax = p.nmax;
  ga.ngroups = p.ngroups;
  ga.nsplit = p.nsplit;
  ga.X = Q;
  ga.ldx = ldq;
  ga.partials = at_ws(p.off_part);
  ga.E = p.E;
  ga.info = inf;
  hipLaunchKernelGGL(k_gram_big, dim3((unsigned)(p.ngroups * p.nsplit)), dim3(kPassThreads), 0, st, ga);
  if (!launched()) return RPCHOLQR_EHIP;
  mark();
  if (A1 && hipMemcpy2DAsync(A1, (size_t)m * sizeof(double), Q, (size_t)ldq * sizeof(double),
                             (size_t)m * sizeof(double), (size_t)n, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return RPCHOLQR_EHIP;
  hipLaunchKernelGGL(k_reduce_partials, dim3((unsigned)((p.E + kReduceThreads - 1) / kReduceThreads), p.G2),
                     dim3(kReduceThreads), 0, st, (const double*)at_ws(p.off_part), p.nsplit, (int)p.E,
                     at_ws(p.off_part2), (const int32_t*)inf);
  if (!launched()) return RPCHOLQR_EHIP;
  mark();

  // Lines 5 (Cholesky, R2^{-1}) and 8 (R = R2 R_s).
  const bool substitute = Rs_in != nullptr;
  CholArgs ca{};
  ca.partial2 = at_ws(p.off_part2);
  ca.G2 = p.G2;
  ca.E = (int32_t)p.E;
  ca.NB = p.NB;
  ca.n = (int32_t)n;
  ca.nmax = p.nmax;
  ca.Rs = at_ws(p.off_Rs);
  ca.T2 = at_ws(p.off_T2);
  ca.R = R;
  ca.ldr = ldr;
  ca.info = inf;
  ca.G1_out = G1;
  ca.R2_out = R2;
  ca.fail_code = RPCHOLQR_INFO_ECHOL;
  if (substitute) ca.R2_out = at_ws(p.off_Rg);  // R2, n x n (the sketch's R is no longer needed)
  ca.Gg = at_ws(p.off_Gg);
  with_big_nmax(p.nmax, [&](auto nm) {
    hipLaunchKernelGGL((k_cholesky<decltype(nm)::value>), dim3(1), dim3(kCholThreads), 0, st, ca);
  });
  if (!launched()) return RPCHOLQR_EHIP;
  mark();

  // Line 6: Q = A1 R2^{-1} in place (explicit inverse), or by substitution with
  // a caller's preconditioner (see factor_impl).
  if (substitute) {
    hipLaunchKernelGGL(k_solve_operands, dim3(1), dim3(kCholThreads), 0, st, (const double*)at_ws(p.off_Rg), (int)n,
                       p.nmax, at_ws(p.off_tri3), at_ws(p.off_full3), (const int32_t*)inf);
    trsm(Q, ldq, at_ws(p.off_tri3), at_ws(p.off_full3));
  } else {
    PassBArgs pb{};
    pb.m = m;
    pb.n = (int32_t)n;
    pb.T2 = at_ws(p.off_T2);
    pb.Q = Q;
    pb.ldq = ldq;
    pb.info = inf;
    with_big_nmax(p.nmax, [&](auto nm) {
      constexpr int NM = decltype(nm)::value, rows = 16 * passb_rows<NM>();
      const int64_t groups = (m + rows - 1) / rows;
      const unsigned grid = (unsigned)std::min<int64_t>(groups, cus);
      hipLaunchKernelGGL((k_passB_big<NM>), dim3(grid), dim3(64 * kPassBBigWaves), 0, st, pb);
    });
  }
  if (!launched()) return RPCHOLQR_EHIP;
  mark();
  return RPCHOLQR_OK;
}

// With Rs_in (n x n upper triangular, ld ldrs) the sketch is skipped and R_s is
// taken as given (Algorithm Preconditioned Cholesky-QR); s is then n.
int32_t factor_impl(int64_t m, int64_t n, int64_t s, uint64_t seed, const double* A, int64_t lda,
                    double* Q, int64_t ldq, double* R, int64_t ldr, int32_t precision, void* ws,
                    size_t ws_bytes, rpcholqr_info* info, void* stream, int64_t* idx, double* As,
                    double* Rs, double* A1, double* G1, double* R2, const double* Rs_in = nullptr,
                    int64_t ldrs = 0, int64_t pa_cap = kPassAMaxBlocks, bool timed = true) {
  const bool smooth = (precision & RPCHOLQR_SMOOTH) != 0;
  precision &= ~RPCHOLQR_SMOOTH;
  if (smooth && Rs_in) return RPCHOLQR_EUNSUPPORTED;
  if (n < 1 || m < n || s < n || lda < m || ldq < m || ldr < n) return RPCHOLQR_EINVAL;
  if (!A || !Q || !R || !info) return RPCHOLQR_EINVAL;
  if (Rs_in && ldrs < n) return RPCHOLQR_EINVAL;
  if (s > INT32_MAX) return RPCHOLQR_EUNSUPPORTED;
  const bool refine = is_refine(precision);
  const bool a1f = precision == RPCHOLQR_A1_FP32;
  if (precision != RPCHOLQR_FP64 && !refine && !a1f) return RPCHOLQR_EUNSUPPORTED;
  if (a1f && (n > kSketchMaxN || Rs_in)) return RPCHOLQR_EUNSUPPORTED;
  if (n > kWideN)
    return factor_big(m, n, s, seed, A, lda, Q, ldq, R, ldr, precision, ws, ws_bytes, info, stream, idx, As, Rs,
                      A1, G1, R2, Rs_in, ldrs, pa_cap, timed, smooth);
  Plan p;
  if (!make_plan(m, n, s, &p, pa_cap, false, refine)) return RPCHOLQR_EUNSUPPORTED;
  const size_t a_bytes = span_bytes(m, n, lda), q_bytes = span_bytes(m, n, ldq), r_bytes = span_bytes(n, n, ldr);
  if (overlaps(A, a_bytes, Q, q_bytes) || overlaps(A, a_bytes, R, r_bytes) || overlaps(Q, q_bytes, R, r_bytes))
    return RPCHOLQR_EINVAL;
  const size_t total = p.total + (smooth ? smooth_bytes(m, n, s) : 0);
  if (!ws || ws_bytes < total || ((uintptr_t)ws & 255)) return RPCHOLQR_EWORKSPACE;
  if (overlaps(ws, total, A, a_bytes) || overlaps(ws, total, Q, q_bytes) || overlaps(ws, total, R, r_bytes))
    return RPCHOLQR_EINVAL;

  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  double* tri = (double*)(base + p.off_tri);
  double* tri2 = (double*)(base + p.off_tri2);
  double* tri3 = (double*)(base + p.off_tri3);
  double* Rs_ws = (double*)(base + p.off_Rs);
  double* part = (double*)(base + p.off_part);
  double* part2 = (double*)(base + p.off_part2);
  double* R1 = (double*)(base + p.off_R1);
  int32_t* inf = (int32_t*)info;
  hipEvent_t* ev = timed ? timing_slot() : nullptr;
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
  if (Rs_in) {
    sa.A = Rs_in;
    sa.lda = ldrs;
    if (p.nmax == kWideN)
      hipLaunchKernelGGL((k_precond_setup<kWideN>), dim3(1), dim3(kSketchThreads), 0, st, sa);
    else
      hipLaunchKernelGGL((k_precond_setup<kSketchMaxN>), dim3(1), dim3(kSketchThreads), 0, st, sa);
  } else {
    if (!launch_sample(sa, smooth, (double*)(base + p.total), st)) return RPCHOLQR_EHIP;
    launch_sketch(p, sa, st);
  }
  if (hipGetLastError() != hipSuccess) return RPCHOLQR_EHIP;
  mark();

  // Lines 4 (A1 = A R_s^{-1}, stored in Q) and 5 (Gram partials; FP32 when refining).
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
  if (p.nmax == kWideN) {
    pa_grid = launch_passes_A_wide(p, pa, st);
  } else with_nmax(p.nmax, [&](auto nm) {
    constexpr int NM = decltype(nm)::value;
    if (precision == RPCHOLQR_FP32_REFINE)
      pa_grid = launch_passes_A<NM, kSolveGram, kGramF32>(p, pa, st);
    else if (precision == RPCHOLQR_BF16X2_REFINE)
      pa_grid = launch_passes_A<NM, kSolveGram, kGramBF16x2>(p, pa, st);
    else if (a1f)
      pa_grid = launch_passes_A<NM, kSolveGram, kGramF64, true>(p, pa, st);
    else
      pa_grid = launch_passes_A<NM>(p, pa, st);
  });
  if (hipGetLastError() != hipSuccess) return RPCHOLQR_EHIP;
  const int g2 = (pa_grid + kReduceChunk - 1) / kReduceChunk;  // <= p.G2
  mark();
  if (A1 && a1f) {
    hipLaunchKernelGGL(k_export_a1f, dim3((unsigned)((m + 255) / 256), (unsigned)n), dim3(256), 0, st,
                       (const double*)Q, ldq, m, (int32_t)n, A1, m);
  } else if (A1 && hipMemcpy2DAsync(A1, (size_t)m * sizeof(double), Q, (size_t)ldq * sizeof(double),
                                    (size_t)m * sizeof(double), (size_t)n, hipMemcpyDeviceToDevice, st) != hipSuccess) {
    return RPCHOLQR_EHIP;
  }

  hipLaunchKernelGGL(k_reduce_partials, dim3((p.E + kReduceThreads - 1) / kReduceThreads, g2),
                     dim3(kReduceThreads), 0, st, (const double*)part, pa_grid, p.E, part2, (const int32_t*)inf);
  if (hipGetLastError() != hipSuccess) return RPCHOLQR_EHIP;
  mark();

  // Lines 5-6 (Cholesky, R2^{-1}) and 8 (R = R2 R_s; into R1 when refining).
  CholArgs ca;
  ca.partial2 = part2;
  ca.G2 = g2;
  ca.E = p.E;
  ca.NB = p.NB;
  ca.n = (int32_t)n;
  ca.nmax = p.nmax;
  ca.Rs = Rs_ws;
  ca.T2 = tri2;
  ca.R = refine ? R1 : R;
  ca.ldr = refine ? n : ldr;
  ca.info = inf;
  ca.G1_out = G1;
  ca.R2_out = R2;
  ca.fail_code = RPCHOLQR_INFO_ECHOL;
  // With a caller's preconditioner kappa(A1) has no bound, so line 6 is solved
  // by row-wise substitution with R2, whose residual does not grow with
  // kappa(R2) (Theorem t_perturb1); with the sketch's R_s, kappa(A1) is small
  // (Lemma l_31) and the product with the explicit R2^{-1} is used.
  const bool substitute = Rs_in != nullptr;
  double* R2s = (double*)(base + p.off_R2);
  if (substitute) ca.R2_out = R2s;  // R2, n x n, for the row-solve operands
  auto cholesky = [&](const CholArgs& c) {
    if (p.nmax == kWideN) {
      hipLaunchKernelGGL((k_cholesky<kWideN>), dim3(1), dim3(kCholThreads), 0, st, c);
      return;
    }
    with_nmax(p.nmax, [&](auto nm) {
      constexpr int NM = decltype(nm)::value;
      hipLaunchKernelGGL((k_cholesky<NM>), dim3(1), dim3(kCholThreads), 0, st, c);
    });
  };
  cholesky(ca);
  if (hipGetLastError() != hipSuccess) return RPCHOLQR_EHIP;
  mark();

  // Line 6: Q = A1 R2^{-1} in place over A1.
  PassBArgs pb;
  pb.m = m;
  pb.n = (int32_t)n;
  pb.T2 = tri2;
  pb.Q = Q;
  pb.ldq = ldq;
  pb.info = inf;
  auto pass_b = [&]() {
    if (p.nmax == kWideN)
      launch_pass_B_wide(m, pb, st);
    else
      with_nmax(p.nmax, [&](auto nm) {
        if (a1f)
          launch_pass_B<decltype(nm)::value, true>(p, pb, st);
        else
          launch_pass_B<decltype(nm)::value>(p, pb, st);
      });
  };
  if (substitute) {
    hipLaunchKernelGGL(k_solve_operands, dim3(1), dim3(kCholThreads), 0, st, (const double*)R2s, (int)n, p.nmax, tri3,
                       (double*)nullptr, (const int32_t*)inf);
    PassAArgs ps = pa;
    ps.A = Q;
    ps.lda = ldq;
    ps.tri_s = tri3;
    if (p.nmax == kWideN)
      hipLaunchKernelGGL(k_passW, dim3(p.PA), dim3(kPassThreads), 0, st, ps);
    else
      with_nmax(p.nmax, [&](auto nm) { launch_passes_A<decltype(nm)::value, kSolveOnly>(p, ps, st); });
  } else {
    pass_b();
  }
  if (hipGetLastError() != hipSuccess) return RPCHOLQR_EHIP;

  if (refine) {
    // Second pass in FP64 (Cholesky-QR on Q1 = A1 R2^{-1}): G = Q1^T Q1,
    // G = R3^T R3, Q = Q1 R3^{-1} in place, R = R3 (R2 R_s).
    PassAArgs pg = pa;
    pg.A = Q;
    pg.lda = ldq;
    pg.tri_s = nullptr;
    pg.W = nullptr;
    int pg_grid = 0;
    with_nmax(p.nmax, [&](auto nm) {
      pg_grid = launch_passes_A<decltype(nm)::value, kGramOnly, kGramF64>(p, pg, st);
    });
    const int g2b = (pg_grid + kReduceChunk - 1) / kReduceChunk;
    hipLaunchKernelGGL(k_reduce_partials, dim3((p.E + kReduceThreads - 1) / kReduceThreads, g2b),
                       dim3(kReduceThreads), 0, st, (const double*)part, pg_grid, p.E, part2, (const int32_t*)inf);
    CholArgs c2 = ca;
    c2.G2 = g2b;
    c2.Rs = R1;
    c2.R = R;
    c2.ldr = ldr;
    c2.G1_out = nullptr;
    c2.R2_out = nullptr;
    c2.fail_code = RPCHOLQR_INFO_ECHOL2;
    cholesky(c2);
    pass_b();
    if (hipGetLastError() != hipSuccess) return RPCHOLQR_EHIP;
  }
  mark();
  return RPCHOLQR_OK;
}

// ---------------------------------------------------------------------------
// Workspace for callers that cannot allocate (rpcholqr_factor_noalloc): one
// static device array per GPU.  In host code `scratch` only names the symbol;
// its device address on the current device comes from hipGetSymbolAddress,
// taken once per device on the first call there and kept in g_scratch.
constexpr size_t kScratchBytes = RPCHOLQR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the current device's scratch array, or nullptr.
void* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}

// The largest pass-A partial count (a power of two, at most kPassAMaxBlocks)
// whose workspace fits the scratch array, or 0 if none does.
int64_t noalloc_pa_cap(int64_t m, int64_t n, int64_t s, bool refine, bool smooth) {
  for (int64_t cap = kPassAMaxBlocks; cap >= 1; cap /= 2) {
    const size_t total = plan_total(m, n, s, cap, refine, smooth);
    if (total == 0) return -1;
    if (total <= kScratchBytes) return cap;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Batched plans.
//
// Per column class (NMAX) and m bucket, a tuning entry fixes the panel height
// of pass A (rows of one problem per pass-A workgroup), the largest number of
// pass-A workgroups (Gram partials) of one problem, and the rows per pass-B
// workgroup.  The built-in entry is used unless rpcholqr_batched_set_tuning
// installed a table (written by the autotuner).

struct TuneEntry {
  int nmax = 0;
  int64_t m_max = 0;
  int pa_rows = 0, pa_max = 0, pb_rows = 0;
};

std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;  // sorted by (nmax, m_max)

TuneEntry default_tuning(int nmax) {
  TuneEntry e;
  e.nmax = nmax;
  e.m_max = INT64_MAX;
  e.pa_rows = 8 * kPassWaves * kWave;  // eight panel groups of four 64-row panels
  e.pa_max = 64;
  e.pb_rows = (nmax == kWideN ? kPassB128Waves : kPassBThreads / kWave) * 16 * 16;  // 16 iterations of 16-row blocks
  return e;
}

TuneEntry tuning_for(int nmax, int64_t m) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  for (const TuneEntry& e : g_tune)
    if (e.nmax == nmax && m <= e.m_max) return e;
  return default_tuning(nmax);
}

constexpr int kBatchMaxPartials = 128;

// Sketch class of a problem: the register kernel's RPT (plus 100 for the wide
// register kernel), 0 for the generic kernel with n <= 64, -1 for the generic
// kernel with n <= 128.
int sketch_key(const Plan& p) {
  if (p.nmax == kWideN) return p.rpt > 0 ? 100 + p.rpt : -1;
  return p.rpt;
}

// Pass-B workgroups of one problem: pb_rows rows each.
int64_t pass_b_items(int64_t m, int pb_rows) {
  const int64_t blocks16 = (m + 15) / 16, per_wg = std::max(1, pb_rows / 16);
  return std::max<int64_t>(1, (blocks16 + per_wg - 1) / per_wg);
}

struct SketchGroup {
  int key = 0;
  size_t probs_off = 0;
  int nprobs = 0;
  int64_t max_s = 0;
};

// One column class: its problems run as one chain of launches (gather, sketch
// per RPT group, pass A, Cholesky, pass B) on a stream of their own.
struct PassClass {
  int nmax = 0;
  size_t probs_off = 0, items_g_off = 0, items_a_off = 0, items_b_off = 0;
  int nprobs = 0;
  int64_t items_g = 0, items_a = 0, items_b = 0;
  std::vector<SketchGroup> sketches;
};

int32_t check_problem(int64_t m, int64_t n, int64_t s, const double* A, int64_t lda, const double* Q,
                      int64_t ldq, const double* R, int64_t ldr) {
  if (n < 1 || m < n || s < n || lda < m || ldq < m || ldr < n) return RPCHOLQR_EINVAL;
  if (!A || !Q || !R) return RPCHOLQR_EINVAL;
  if (s > INT32_MAX) return RPCHOLQR_EUNSUPPORTED;
  const size_t a_bytes = span_bytes(m, n, lda), q_bytes = span_bytes(m, n, ldq), r_bytes = span_bytes(n, n, ldr);
  if (overlaps(A, a_bytes, Q, q_bytes) || overlaps(A, a_bytes, R, r_bytes) || overlaps(Q, q_bytes, R, r_bytes))
    return RPCHOLQR_EINVAL;
  return RPCHOLQR_OK;
}

}  // namespace

struct rpcholqr_batched_plan {
  int64_t batch = 0;
  void* dmem = nullptr;
  size_t dbytes = 0;
  size_t sk_off = 0, pa_off = 0, ch_off = 0, pb_off = 0;
  std::vector<PassClass> classes;
  // one stream per column class beyond the first (default priority), and the
  // events that fork them from and join them to the caller's stream
  std::vector<hipStream_t> streams;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;
};

namespace {

template <typename T>
T* at(const rpcholqr_batched_plan* p, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(p->dmem) + off);
}

void release(rpcholqr_batched_plan* p) {
  for (hipStream_t s : p->streams) (void)hipStreamDestroy(s);
  for (hipEvent_t e : p->joins) (void)hipEventDestroy(e);
  if (p->fork) (void)hipEventDestroy(p->fork);
  if (p->dmem) (void)hipFree(p->dmem);
  delete p;
}

int32_t batched_create(int64_t batch, const int64_t* m, const int64_t* n, const int64_t* s, const uint64_t* seed,
                       const double* const* A, const int64_t* lda, double* const* Q, const int64_t* ldq,
                       double* const* R, const int64_t* ldr, int32_t precision, rpcholqr_batched_plan** out,
                       int64_t* bad_problem) {
  if (bad_problem) *bad_problem = -1;
  if (!out) return RPCHOLQR_EINVAL;
  *out = nullptr;
  if (batch < 1 || batch > INT32_MAX || !m || !n || !s || !seed || !A || !lda || !Q || !ldq || !R || !ldr)
    return RPCHOLQR_EINVAL;
  if (precision != RPCHOLQR_FP64) return RPCHOLQR_EUNSUPPORTED;
  std::vector<Plan> plans((size_t)batch);
  std::vector<int> pb_rows((size_t)batch);
  for (int64_t b = 0; b < batch; ++b) {
    int32_t rc = check_problem(m[b], n[b], s[b], A[b], lda[b], Q[b], ldq[b], R[b], ldr[b]);
    if (rc == RPCHOLQR_OK) {
      if (n[b] > kWideN) {
        rc = RPCHOLQR_EUNSUPPORTED;
      } else {
        const TuneEntry t = tuning_for(pick_nmax(n[b]), m[b]);
        const int64_t panels = (m[b] + kWave - 1) / kWave;
        const int64_t pgroups = (panels + kPassWaves - 1) / kPassWaves;
        const int64_t per_wg = std::max(1, t.pa_rows / (kPassWaves * kWave));
        int64_t pa = (pgroups + per_wg - 1) / per_wg;
        pa = std::min<int64_t>(std::max<int64_t>(pa, 1), std::min(t.pa_max, kBatchMaxPartials));
        pb_rows[b] = t.pb_rows;
        if (!make_plan(m[b], n[b], s[b], &plans[b], pa, true)) rc = RPCHOLQR_EUNSUPPORTED;
      }
    }
    if (rc != RPCHOLQR_OK) {
      if (bad_problem) *bad_problem = b;
      return rc;
    }
  }
  auto* p = new rpcholqr_batched_plan();
  p->batch = batch;
  // Column classes; problems within a class in decreasing m (largest work first).
  std::vector<int64_t> order((size_t)batch);
  for (int64_t b = 0; b < batch; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return m[x] > m[y]; });
  std::map<int, std::vector<int32_t>> by_nmax;
  for (int64_t b : order) by_nmax[plans[b].nmax].push_back((int32_t)b);
  // Device buffer layout: argument tables, per-class lists, then the workspaces.
  size_t off = 0;
  auto reserve = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  p->sk_off = reserve(sizeof(SketchArgs) * batch);
  p->pa_off = reserve(sizeof(PassAArgs) * batch);
  p->ch_off = reserve(sizeof(CholArgs) * batch);
  p->pb_off = reserve(sizeof(PassBArgs) * batch);
  struct HostLists {
    std::vector<int32_t> probs;
    std::vector<BatchItem> g, a, b;
    std::vector<std::vector<int32_t>> sk;
  };
  std::vector<HostLists> lists;
  for (auto& kv : by_nmax) {
    PassClass c;
    HostLists h;
    c.nmax = kv.first;
    h.probs = kv.second;
    c.nprobs = (int)h.probs.size();
    std::map<int, std::vector<int32_t>> by_key;
    for (int32_t b : h.probs) {
      const int64_t ng = ((int64_t)s[b] * n[b] + kGatherThreads - 1) / kGatherThreads;
      for (int64_t i = 0; i < ng; ++i) h.g.push_back(BatchItem{b, (int32_t)i, (int32_t)ng});
      const int32_t na = plans[b].PA;
      for (int32_t k = 0; k < na; ++k) h.a.push_back(BatchItem{b, k, na});
      const int32_t nb = (int32_t)pass_b_items(m[b], pb_rows[b]);
      for (int32_t k = 0; k < nb; ++k) h.b.push_back(BatchItem{b, k, nb});
      by_key[sketch_key(plans[b])].push_back(b);
    }
    c.probs_off = reserve(sizeof(int32_t) * h.probs.size());
    c.items_g = (int64_t)h.g.size();
    c.items_a = (int64_t)h.a.size();
    c.items_b = (int64_t)h.b.size();
    c.items_g_off = reserve(sizeof(BatchItem) * h.g.size());
    c.items_a_off = reserve(sizeof(BatchItem) * h.a.size());
    c.items_b_off = reserve(sizeof(BatchItem) * h.b.size());
    for (auto& kk : by_key) {
      SketchGroup g;
      g.key = kk.first;
      g.nprobs = (int)kk.second.size();
      g.probs_off = reserve(sizeof(int32_t) * kk.second.size());
      for (int32_t b : kk.second) g.max_s = std::max<int64_t>(g.max_s, s[b]);
      c.sketches.push_back(g);
      h.sk.push_back(kk.second);
    }
    p->classes.push_back(c);
    lists.push_back(std::move(h));
  }
  std::vector<size_t> ws_off((size_t)batch);
  for (int64_t b = 0; b < batch; ++b) ws_off[b] = reserve(plans[b].total);
  p->dbytes = off;
  bool ok = hipMalloc(&p->dmem, p->dbytes) == hipSuccess;
  if (ok && p->classes.size() > 1) {
    ok = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) == hipSuccess;
    for (size_t c = 1; ok && c < p->classes.size(); ++c) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
      if (ok) p->streams.push_back(st);
      ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
      if (ok) p->joins.push_back(ev);
    }
  }
  if (!ok) {
    release(p);
    return RPCHOLQR_EHIP;
  }
  // Host images of the argument tables.
  std::vector<SketchArgs> sk((size_t)batch);
  std::vector<PassAArgs> pa((size_t)batch);
  std::vector<CholArgs> ch((size_t)batch);
  std::vector<PassBArgs> pb((size_t)batch);
  char* base = static_cast<char*>(p->dmem);
  for (int64_t b = 0; b < batch; ++b) {
    const Plan& pl = plans[b];
    char* w = base + ws_off[b];
    SketchArgs& sa = sk[b];
    sa = SketchArgs{};
    sa.m = m[b];
    sa.n = (int32_t)n[b];
    sa.s = (int32_t)s[b];
    sa.seed = seed[b];
    sa.scale = std::sqrt((double)m[b] / (double)s[b]);
    sa.A = A[b];
    sa.lda = lda[b];
    sa.As = (double*)(w + pl.off_As);
    sa.tri = (double*)(w + pl.off_tri);
    sa.Rs = (double*)(w + pl.off_Rs);
    sa.nmax = pl.nmax;
    PassAArgs& a = pa[b];
    a = PassAArgs{};
    a.m = m[b];
    a.n = (int32_t)n[b];
    a.A = A[b];
    a.lda = lda[b];
    a.tri_s = (const double*)(w + pl.off_tri);
    a.partials = (double*)(w + pl.off_part);
    a.W = Q[b];
    a.ldw = ldq[b];
    CholArgs& c = ch[b];
    c = CholArgs{};
    c.partial2 = (const double*)(w + pl.off_part);
    c.G2 = pl.PA;
    c.E = pl.E;
    c.NB = pl.NB;
    c.n = (int32_t)n[b];
    c.nmax = pl.nmax;
    c.Rs = (const double*)(w + pl.off_Rs);
    c.T2 = (double*)(w + pl.off_tri2);
    c.R = R[b];
    c.ldr = ldr[b];
    c.fail_code = RPCHOLQR_INFO_ECHOL;
    PassBArgs& q = pb[b];
    q = PassBArgs{};
    q.m = m[b];
    q.n = (int32_t)n[b];
    q.T2 = (const double*)(w + pl.off_tri2);
    q.Q = Q[b];
    q.ldq = ldq[b];
  }
  auto up = [&](size_t dst, const void* src, size_t bytes) {
    return bytes == 0 || hipMemcpy(base + dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  ok = up(p->sk_off, sk.data(), sizeof(SketchArgs) * batch) && up(p->pa_off, pa.data(), sizeof(PassAArgs) * batch) &&
       up(p->ch_off, ch.data(), sizeof(CholArgs) * batch) && up(p->pb_off, pb.data(), sizeof(PassBArgs) * batch);
  for (size_t c = 0; ok && c < p->classes.size(); ++c) {
    const PassClass& pc = p->classes[c];
    const HostLists& h = lists[c];
    ok = up(pc.probs_off, h.probs.data(), sizeof(int32_t) * h.probs.size()) &&
         up(pc.items_g_off, h.g.data(), sizeof(BatchItem) * h.g.size()) &&
         up(pc.items_a_off, h.a.data(), sizeof(BatchItem) * h.a.size()) &&
         up(pc.items_b_off, h.b.data(), sizeof(BatchItem) * h.b.size());
    for (size_t k = 0; ok && k < pc.sketches.size(); ++k)
      ok = up(pc.sketches[k].probs_off, h.sk[k].data(), sizeof(int32_t) * h.sk[k].size());
  }
  if (!ok) {
    release(p);
    return RPCHOLQR_EHIP;
  }
  *out = p;
  return RPCHOLQR_OK;
}

// The chain of one column class on stream st.
void launch_class(const rpcholqr_batched_plan* p, const PassClass& c, int32_t* inf, hipStream_t st) {
  const SketchArgs* sk = at<SketchArgs>(p, p->sk_off);
  const PassAArgs* pa = at<PassAArgs>(p, p->pa_off);
  const CholArgs* ch = at<CholArgs>(p, p->ch_off);
  const PassBArgs* pb = at<PassBArgs>(p, p->pb_off);
  // Lines 2-3 of Algorithm rpCholesky-QR.
  hipLaunchKernelGGL(kb_gather, dim3((unsigned)c.items_g), dim3(kGatherThreads), 0, st, sk,
                     at<BatchItem>(p, c.items_g_off));
  for (const SketchGroup& g : c.sketches) {
    const int32_t* probs = at<int32_t>(p, g.probs_off);
    const dim3 grid((unsigned)g.nprobs), blk(kSketchThreads);
    switch (g.key) {
      case 4: hipLaunchKernelGGL((kb_sketch_qr<4>), grid, blk, 0, st, sk, probs, inf); break;
      case 8: hipLaunchKernelGGL((kb_sketch_qr<8>), grid, blk, 0, st, sk, probs, inf); break;
      case 12: hipLaunchKernelGGL((kb_sketch_qr<12>), grid, blk, 0, st, sk, probs, inf); break;
      case 16: hipLaunchKernelGGL((kb_sketch_qr<16>), grid, blk, 0, st, sk, probs, inf); break;
      case 24: hipLaunchKernelGGL((kb_sketch_qr<24>), grid, blk, 0, st, sk, probs, inf); break;
      case 108: hipLaunchKernelGGL((kb_sketch_qr_wide<8>), grid, blk, 0, st, sk, probs, inf); break;
      case 112: hipLaunchKernelGGL((kb_sketch_qr_wide<12>), grid, blk, 0, st, sk, probs, inf); break;
      case 116: hipLaunchKernelGGL((kb_sketch_qr_wide<16>), grid, blk, 0, st, sk, probs, inf); break;
      case 124: hipLaunchKernelGGL((kb_sketch_qr_wide<24>), grid, blk, 0, st, sk, probs, inf); break;
      case 0:
        hipLaunchKernelGGL((kb_sketch_qr_generic<64>), grid, blk, 2 * (size_t)g.max_s * sizeof(double), st, sk, probs,
                           inf);
        break;
      default:
        hipLaunchKernelGGL((kb_sketch_qr_generic<kWideN>), grid, blk, 2 * (size_t)g.max_s * sizeof(double), st, sk,
                           probs, inf);
        break;
    }
  }
  // Lines 4-8 of Algorithm Preconditioned Cholesky-QR.
  const BatchItem* ia = at<BatchItem>(p, c.items_a_off);
  const BatchItem* ib = at<BatchItem>(p, c.items_b_off);
  const int32_t* probs = at<int32_t>(p, c.probs_off);
  const dim3 ga((unsigned)c.items_a), gc((unsigned)c.nprobs), gb((unsigned)c.items_b);
  const dim3 bp(kPassThreads), bc(kCholThreads), bb(kPassBThreads);
  switch (c.nmax) {
    case 16:
      hipLaunchKernelGGL((kb_passA<16>), ga, bp, 0, st, pa, ia, inf);
      hipLaunchKernelGGL((kb_cholesky<16>), gc, bc, 0, st, ch, probs, inf);
      hipLaunchKernelGGL((kb_passB<16>), gb, bb, 0, st, pb, ib, inf);
      break;
    case 32:
      hipLaunchKernelGGL((kb_passA<32>), ga, bp, 0, st, pa, ia, inf);
      hipLaunchKernelGGL((kb_cholesky<32>), gc, bc, 0, st, ch, probs, inf);
      hipLaunchKernelGGL((kb_passB<32>), gb, bb, 0, st, pb, ib, inf);
      break;
    case 48:
      hipLaunchKernelGGL((kb_passA<48>), ga, bp, 0, st, pa, ia, inf);
      hipLaunchKernelGGL((kb_cholesky<48>), gc, bc, 0, st, ch, probs, inf);
      hipLaunchKernelGGL((kb_passB<48>), gb, bb, 0, st, pb, ib, inf);
      break;
    case 64:
      hipLaunchKernelGGL((kb_passA<64>), ga, bp, 0, st, pa, ia, inf);
      hipLaunchKernelGGL((kb_cholesky<64>), gc, bc, 0, st, ch, probs, inf);
      hipLaunchKernelGGL((kb_passB<64>), gb, bb, 0, st, pb, ib, inf);
      break;
    default:
      hipLaunchKernelGGL(kb_passW, ga, bp, 0, st, pa, ia, inf);
      hipLaunchKernelGGL(kb_gramW, ga, bp, 0, st, pa, ia, inf);
      hipLaunchKernelGGL((kb_cholesky<kWideN>), gc, bc, 0, st, ch, probs, inf);
      hipLaunchKernelGGL(kb_passB128, gb, dim3(kPassB128Threads), 0, st, pb, ib, inf);
      break;
  }
}

// The column classes run concurrently: the first on the caller's stream, the
// others on the plan's streams, forked from and joined to the caller's stream
// by events (both are recorded by a stream capture).  Classes with the most
// work start first.
int32_t batched_execute(const rpcholqr_batched_plan* p, rpcholqr_info* info, void* stream) {
  if (!p || !info) return RPCHOLQR_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int32_t* inf = (int32_t*)info;
  const size_t nc = p->classes.size();
  if (nc > 1) {
    if (hipEventRecord(p->fork, st) != hipSuccess) return RPCHOLQR_EHIP;
    for (size_t c = 1; c < nc; ++c)
      if (hipStreamWaitEvent(p->streams[c - 1], p->fork, 0) != hipSuccess) return RPCHOLQR_EHIP;
  }
  for (size_t c = 0; c < nc; ++c) launch_class(p, p->classes[c], inf, c == 0 ? st : p->streams[c - 1]);
  if (hipGetLastError() != hipSuccess) return RPCHOLQR_EHIP;
  for (size_t c = 1; c < nc; ++c) {
    if (hipEventRecord(p->joins[c - 1], p->streams[c - 1]) != hipSuccess) return RPCHOLQR_EHIP;
    if (hipStreamWaitEvent(st, p->joins[c - 1], 0) != hipSuccess) return RPCHOLQR_EHIP;
  }
  return RPCHOLQR_OK;
}

int32_t set_tuning(const rpcholqr_batched_tuning* entries, int32_t count) {
  if (count < 0 || (count > 0 && !entries)) return RPCHOLQR_EINVAL;
  std::vector<TuneEntry> t;
  for (int32_t i = 0; i < count; ++i) {
    const rpcholqr_batched_tuning& e = entries[i];
    const bool nmax_ok = e.nmax == 16 || e.nmax == 32 || e.nmax == 48 || e.nmax == 64 || e.nmax == kWideN;
    if (!nmax_ok || e.m_max < 1 || e.pa_rows < kPassWaves * kWave || e.pa_rows % (kPassWaves * kWave) != 0 ||
        e.pa_max < 1 || e.pa_max > kBatchMaxPartials || e.pb_rows < 16 || e.pb_rows % 16 != 0)
      return RPCHOLQR_EINVAL;
    TuneEntry x;
    x.nmax = e.nmax;
    x.m_max = e.m_max;
    x.pa_rows = e.pa_rows;
    x.pa_max = e.pa_max;
    x.pb_rows = e.pb_rows;
    t.push_back(x);
  }
  std::stable_sort(t.begin(), t.end(), [](const TuneEntry& x, const TuneEntry& y) {
    return x.nmax != y.nmax ? x.nmax < y.nmax : x.m_max < y.m_max;
  });
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune = std::move(t);
  return RPCHOLQR_OK;
}

}  // namespace

extern "C" {

int32_t rpcholqr_max_n(void) { return kMaxN; }

size_t rpcholqr_workspace_bytes(int64_t m, int64_t n, int64_t s, int32_t precision) {
  const bool smooth = (precision & RPCHOLQR_SMOOTH) != 0;
  precision &= ~RPCHOLQR_SMOOTH;
  return precision_total(m, n, s, kPassAMaxBlocks, precision, smooth);
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

int32_t rpcholqr_factor_noalloc(int64_t m, int64_t n, int64_t s, uint64_t seed, const double* A, int64_t lda,
                                double* Q, int64_t ldq, double* R, int64_t ldr, int32_t precision,
                                rpcholqr_info* info, void* stream) {
  if (n < 1 || m < n || s < n || lda < m || ldq < m || ldr < n || !A || !Q || !R || !info) return RPCHOLQR_EINVAL;
  const int32_t prec = precision & ~RPCHOLQR_SMOOTH;
  if (prec != RPCHOLQR_FP64 && prec != RPCHOLQR_FP32_REFINE && prec != RPCHOLQR_BF16X2_REFINE)
    return RPCHOLQR_EUNSUPPORTED;
  const int64_t cap = noalloc_pa_cap(m, n, s, is_refine(prec), (precision & RPCHOLQR_SMOOTH) != 0);
  if (cap < 0) return RPCHOLQR_EUNSUPPORTED;
  if (cap == 0) return RPCHOLQR_EWORKSPACE;
  void* ws = scratch_address();
  if (!ws) return RPCHOLQR_EHIP;
  return factor_impl(m, n, s, seed, A, lda, Q, ldq, R, ldr, precision, ws, kScratchBytes, info, stream, nullptr,
                     nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, cap, false);
}

int32_t rpcholqr_precond_factor(int64_t m, int64_t n, const double* A, int64_t lda, const double* Rs,
                                int64_t ldrs, double* Q, int64_t ldq, double* R, int64_t ldr, int32_t precision,
                                void* workspace, size_t workspace_bytes, rpcholqr_info* info, void* stream) {
  if (!Rs) return RPCHOLQR_EINVAL;
  return factor_impl(m, n, n, 0, A, lda, Q, ldq, R, ldr, precision, workspace, workspace_bytes, info, stream,
                     nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, Rs, ldrs);
}

int32_t rpcholqr_sample_indices(int64_t m, int64_t s, uint64_t seed, int64_t* idx) {
  if (m < 1 || s < 0 || (s > 0 && !idx)) return RPCHOLQR_EINVAL;
  for (int64_t r = 0; r < s; ++r) {
    // SplitMix64 output r in counter form, reduced to [0, m) by multiply-high.
    uint64_t z = seed + ((uint64_t)r + 1u) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    idx[r] = (int64_t)(((unsigned __int128)z * (uint64_t)m) >> 64);
  }
  return RPCHOLQR_OK;
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

int32_t rpcholqr_batched_plan_create(int64_t batch, const int64_t* m, const int64_t* n, const int64_t* s,
                                     const uint64_t* seed, const double* const* A, const int64_t* lda,
                                     double* const* Q, const int64_t* ldq, double* const* R, const int64_t* ldr,
                                     int32_t precision, rpcholqr_batched_plan** plan, int64_t* bad_problem) {
  return batched_create(batch, m, n, s, seed, A, lda, Q, ldq, R, ldr, precision, plan, bad_problem);
}

int32_t rpcholqr_batched_execute(const rpcholqr_batched_plan* plan, rpcholqr_info* info, void* stream) {
  return batched_execute(plan, info, stream);
}

size_t rpcholqr_batched_plan_device_bytes(const rpcholqr_batched_plan* plan) { return plan ? plan->dbytes : 0; }

int32_t rpcholqr_batched_plan_destroy(rpcholqr_batched_plan* plan) {
  if (!plan) return RPCHOLQR_OK;
  release(plan);
  return RPCHOLQR_OK;
}

int32_t rpcholqr_batched_set_tuning(const rpcholqr_batched_tuning* entries, int32_t count) {
  return set_tuning(entries, count);
}

int32_t rpcholqr_factor_batched(int64_t batch, const int64_t* m, const int64_t* n, const int64_t* s,
                                const uint64_t* seed, const double* const* A, const int64_t* lda,
                                double* const* Q, const int64_t* ldq, double* const* R, const int64_t* ldr,
                                int32_t precision, rpcholqr_info* info, void* stream, int64_t* bad_problem) {
  rpcholqr_batched_plan* plan = nullptr;
  int32_t rc = batched_create(batch, m, n, s, seed, A, lda, Q, ldq, R, ldr, precision, &plan, bad_problem);
  if (rc != RPCHOLQR_OK) return rc;
  rc = batched_execute(plan, info, stream);
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && rc == RPCHOLQR_OK) rc = RPCHOLQR_EHIP;
  const int32_t rc2 = rpcholqr_batched_plan_destroy(plan);
  return rc != RPCHOLQR_OK ? rc : rc2;
}

}  // extern "C"

/*
 * rpcholqr.h -- C ABI of the MI355X (gfx950) library for randomized
 * preconditioned Cholesky-QR (rpCholesky-QR), Garrison & Ipsen,
 * "A randomized preconditioned Cholesky-QR algorithm", arXiv 2406.11751.
 *
 * Problem (Section 1; Section 2.1): given A in R^{m x n} with rank n and
 * m >= n, compute a thin QR factorization A = Q R with Q^T Q = I_n and R upper
 * triangular, nonsingular, with a positive diagonal (the factorization with a
 * positive diagonal is unique, Lemma l_r1r2).
 *
 * Method (Algorithm rpCholesky-QR, Section 4), with the smoothing matrix F = I:
 *   1. sample s >= n row indices uniformly, independently, with replacement,
 *      from `seed` (SplitMix64 output r, reduced to [0, m) by a 64x64->128 bit
 *      multiply-high; 0-based);
 *   2. A_s = sqrt(m/s) * A(idx, :)  (scale of the paper's Remark r_exp);
 *   3. Householder QR of A_s, keep R_s (diagonal made positive);
 *   4. A1 = A R_s^{-1} by row-wise substitution;
 *   5. G1 = A1^T A1;  6. G1 = R2^T R2 (Cholesky);  7. Q = A1 R2^{-1};
 *   8. R = R2 R_s.
 * Steps 4-8 are Algorithm "Preconditioned Cholesky-QR" (Section 3.1).
 *
 * Conventions for every entry point:
 *  - Matrices are IEEE binary64, column-major: element (i, j) of a matrix with
 *    leading dimension ld is at [i + j*ld].
 *  - Matrix and workspace pointers are DEVICE pointers (HIP device memory on
 *    the current device); `stream` is a hipStream_t passed as void* (NULL = the
 *    default stream).  The caller owns every buffer; the library never frees
 *    caller memory.
 *  - Calls are asynchronous and stream-ordered.  The return value reports only
 *    argument and launch problems (rpcholqr_status).  Numerical failures are
 *    written to the device rpcholqr_info the caller passes; read it after
 *    synchronizing the stream.  On a numerical failure Q and R are unspecified.
 *  - A is read only.  Q must not overlap A (Q holds A1 = A R_s^{-1} while A
 *    is still being read), R must not overlap A or Q.  The strictly lower
 *    triangle of R is written as zero.
 */
#ifndef RPCHOLQR_H
#define RPCHOLQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Synchronous status returned by every call. */
typedef enum {
  RPCHOLQR_OK = 0,
  RPCHOLQR_EINVAL = -1,      /* n < 1, m < n, s < n, ld* too small, NULL or overlapping buffers */
  RPCHOLQR_EHIP = -2,        /* a HIP runtime call or kernel launch failed */
  RPCHOLQR_EWORKSPACE = -3,  /* workspace NULL or smaller than rpcholqr_workspace_bytes() */
  RPCHOLQR_EUNSUPPORTED = -4 /* n or s beyond what this library supports (rpcholqr_max_n()) */
} rpcholqr_status;

/* Arithmetic of the passes over A.
 *   RPCHOLQR_FP64          every step in binary64 (the paper's algorithm).
 *   RPCHOLQR_FP32_REFINE   not in the paper: step 5's Gram matrix A1^T A1 is
 *       formed in binary32 (A1 rounded to float, float products and sums); the
 *       row solves of steps 4 and 7 stay binary64, so A = Q1 (R2 R_s) holds to
 *       binary64 accuracy, and Q1's loss of orthogonality (about u32 kappa(A1)^2)
 *       is removed by a second, binary64 Cholesky-QR pass on Q1 (Cholesky-QR2,
 *       Section 1): G = Q1^T Q1 = R3^T R3, Q = Q1 R3^{-1}, R = R3 (R2 R_s).
 *       Needs a larger workspace (rpcholqr_workspace_bytes with this value).
 *   RPCHOLQR_BF16X2_REFINE as RPCHOLQR_FP32_REFINE, but step 5 splits each
 *       float-rounded entry of A1 into bfloat16 hi + lo and forms
 *       hi^T hi + hi^T lo + lo^T hi with float accumulation (about 16
 *       significant bits); the second pass is the same binary64 pass.
 *   RPCHOLQR_A1_FP32       not in the paper: the preconditioned matrix
 *       A1 = A R_s^{-1} (step 4, computed in binary64 exactly as with
 *       RPCHOLQR_FP64) is rounded to binary32 where it is kept between the two
 *       passes, halving that traffic; the Gram matrix (step 5) and Q = A1 R2^{-1}
 *       (step 7) are formed in binary64 from the stored binary32 values, so Q is
 *       as orthogonal as with RPCHOLQR_FP64, while ||A - Q R|| / ||A|| grows to
 *       about u32 kappa(A1) (the rounding of A1 enters the residual only; Theorem
 *       t_perturb2).  n <= 64.  The float copy of A1 lives in the Q buffer
 *       itself: row r of column j, 64 b <= r < 64 b + 64, at byte offset
 *       8 (64 b + j ldq) + 4 (r - 64 b), inside the memory of the same rows of Q. */
typedef enum {
  RPCHOLQR_FP64 = 0,
  RPCHOLQR_FP32_REFINE = 1,
  RPCHOLQR_BF16X2_REFINE = 2,
  RPCHOLQR_A1_FP32 = 3
} rpcholqr_precision;

/* Option OR'ed into the precision argument of rpcholqr_factor,
 * rpcholqr_factor_debug, rpcholqr_factor_noalloc and rpcholqr_workspace_bytes:
 * sample rows of the smoothed matrix F A instead of A's own rows (Algorithm
 * rpCholesky-QR line 2 with F = F_T D; the remark after Theorem t_prob), for
 * inputs whose rows are coherent (a few rows carry the column space, such as
 * the [I; 0] R test matrices of Section 5.1), where sampling A's rows leaves
 * the sketch rank deficient.  F = F_T D P: A is padded with zero rows to
 * M = 2^p >= m rows, P moves row i to position pi(i) (x = i * 0x9e3779b97f4a7c15,
 * x ^= x >> h, x *= 0xbf58476d1ce4e5b9, x ^= x >> h, all mod M, h = max(1, p/2)),
 * D multiplies it by a random sign (D_i = +1 when bit 63 of SplitMix64 output i
 * seeded with seed XOR 0x5851f42d4c957f2d is 0), and F_T is the Walsh-Hadamard
 * transform (F_T(k, q) = (-1)^popcount(k AND q) / sqrt(M)); s row indices are
 * drawn from [0, M) and A_s = sqrt(M/s) (F [A; 0])(idx, :), formed without
 * the transform as A_s(r, j) = T(r, j) / sqrt(s) with
 * T(r, j) = sum_i D_i (-1)^popcount(idx_r AND pi(i)) A(i, j), summed in a fixed
 * order (chunks of G * 4096 rows, G = max(1, ceil(ceil(m / 4096) / 256)); an
 * fma chain in ascending i within a chunk; chunks added in ascending order).
 * Steps 3-8 are unchanged (line 4 uses A itself).  Costs s * m * n extra
 * multiply-adds and ceil(m / chunk) * s * n doubles of workspace.  Not
 * available in rpcholqr_precond_factor or the batched entry points. */
#define RPCHOLQR_SMOOTH 0x100

/* Numerical outcome, written on the device by the library. */
typedef struct {
  int32_t code;  /* RPCHOLQR_INFO_* */
  int32_t index; /* 0-based failing column, -1 when code == RPCHOLQR_INFO_OK */
} rpcholqr_info;

#define RPCHOLQR_INFO_OK 0
/* Sketch QR (step 3): a Householder column norm of A_s is zero or not finite. */
#define RPCHOLQR_INFO_ESKETCH 1
/* Cholesky of G1 (step 6): a pivot is not positive or not finite (the
 * hypothesis kappa(A1)^2 gamma_2 < 1 of Theorem t_perturb2 failed). */
#define RPCHOLQR_INFO_ECHOL 2
/* Cholesky of the second pass of a refined precision (G = Q1^T Q1) failed. */
#define RPCHOLQR_INFO_ECHOL2 3

/* Largest n the library accepts (1024).  Supported sizes: n <= 1024 for
 * RPCHOLQR_FP64 with s <= 1536, and s <= 8192 when n > 128 (the sketch then
 * streams the sample from the workspace); n <= 64 for the refined precisions
 * and RPCHOLQR_A1_FP32;
 * n <= 128 and s <= 1536 in the batched entry points; other sizes give
 * RPCHOLQR_EUNSUPPORTED. */
int32_t rpcholqr_max_n(void);

/* Device workspace in bytes needed by rpcholqr_factor / rpcholqr_factor_debug
 * for these sizes (0 if the sizes are invalid or unsupported). */
size_t rpcholqr_workspace_bytes(int64_t m, int64_t n, int64_t s, int32_t precision);

/* Thin QR A = Q R by rpCholesky-QR (Algorithm rpCholesky-QR, Section 4).
 *   m, n, s     rows, columns, sampled rows (1 <= n <= m, n <= s)
 *   seed        seed of the sampled row indices
 *   A, lda      input, m x n, lda >= m (device, read only)
 *   Q, ldq      output, m x n, ldq >= m (device)
 *   R, ldr      output, n x n upper triangular, ldr >= n (device)
 *   precision   rpcholqr_precision
 *   workspace   device scratch of at least rpcholqr_workspace_bytes() bytes,
 *               256-byte aligned; contents on entry are ignored
 *   info        device rpcholqr_info receiving the numerical outcome
 *   stream      hipStream_t as void*
 * The result is deterministic: the same inputs give the same bits.  The call
 * allocates nothing and issues only kernel launches on `stream`, so a stream
 * capture records it into a HIP graph whose replays give the same bits. */
int32_t rpcholqr_factor(int64_t m, int64_t n, int64_t s, uint64_t seed, const double* A, int64_t lda,
                        double* Q, int64_t ldq, double* R, int64_t ldr, int32_t precision,
                        void* workspace, size_t workspace_bytes, rpcholqr_info* info, void* stream);

/* rpcholqr_factor plus copies of the intermediates, for checking each step.
 * Every extra pointer is a device pointer and may be NULL (not written):
 *   idx  int64[s]              sampled row indices (step 1)
 *   As   s x n, ld s           scaled sample (step 2)
 *   Rs   n x n, ld n           sketch factor R_s, positive diagonal (step 3)
 *   A1   m x n, ld m           preconditioned matrix A R_s^{-1} (step 4)
 *   G1   n x n, ld n           Gram matrix, upper triangle (step 5)
 *   R2   n x n, ld n           Cholesky factor of G1 (step 6)
 * The workspace requirement is the same as for rpcholqr_factor. */
int32_t rpcholqr_factor_debug(int64_t m, int64_t n, int64_t s, uint64_t seed, const double* A,
                              int64_t lda, double* Q, int64_t ldq, double* R, int64_t ldr,
                              int32_t precision, void* workspace, size_t workspace_bytes,
                              rpcholqr_info* info, void* stream, int64_t* idx, double* As, double* Rs,
                              double* A1, double* G1, double* R2);

/* Algorithm "Preconditioned Cholesky-QR" (Section 3.1) with a preconditioner
 * the caller supplies: A1 = A R_s^{-1}, G1 = A1^T A1 = R2^T R2, Q = A1 R2^{-1}
 * (by row-wise substitution with R2, since a caller's R_s puts no bound on
 * kappa(A1)), R = R2 R_s.  With R_s = I this is Algorithm "Basic Cholesky-QR"
 * (Section 2.1).  rpCholesky-QR is this algorithm with R_s from the sketch; here
 * R_s is used exactly as given (no sign change, no check of its diagonal: a
 * singular or badly conditioned R_s shows up as RPCHOLQR_INFO_ECHOL).
 *   Rs, ldrs    n x n upper triangular, column-major, ldrs >= n (device, read
 *               only; its strictly lower part is ignored)
 *   workspace   at least rpcholqr_workspace_bytes(m, n, n, precision) bytes
 * Other arguments, status returns and info codes as for rpcholqr_factor
 * (RPCHOLQR_INFO_ESKETCH does not occur). */
int32_t rpcholqr_precond_factor(int64_t m, int64_t n, const double* A, int64_t lda, const double* Rs,
                                int64_t ldrs, double* Q, int64_t ldq, double* R, int64_t ldr, int32_t precision,
                                void* workspace, size_t workspace_bytes, rpcholqr_info* info, void* stream);

/* rpcholqr_factor without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  The call allocates nothing: its workspace
 * is a static device array of RPCHOLQR_NOALLOC_SCRATCH_BYTES bytes that the
 * library holds on every GPU it runs this call on, until the process ends
 * (its address is looked up on the first call on each device).
 *   Arguments, status returns, info codes and asynchrony as for
 *   rpcholqr_factor, on the current device.
 *   Sizes: as for rpcholqr_factor.  If the sizes need more workspace than the
 *   array holds with the usual number of Gram partials, fewer (larger) partials
 *   are used, so Q and R then agree with rpcholqr_factor to rounding (about
 *   1e-15) rather than to the bit; sizes whose workspace does not fit even with
 *   one partial return RPCHOLQR_EWORKSPACE.
 *   Every call on a GPU uses that GPU's one array and leaves its contents
 *   behind (nothing in it needs to start at zero): calls that overlap in time on
 *   one GPU (different streams, host threads or processes sharing the library
 *   instance) race and give undefined results; serialize them. */
#define RPCHOLQR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int32_t rpcholqr_factor_noalloc(int64_t m, int64_t n, int64_t s, uint64_t seed, const double* A, int64_t lda,
                                double* Q, int64_t ldq, double* R, int64_t ldr, int32_t precision,
                                rpcholqr_info* info, void* stream);

/* The s sampled row indices of rpcholqr_factor for (m, seed), 0-based, computed
 * on the host (Algorithm rpCholesky-QR line 2; Section 4: uniform, independent,
 * with replacement): index r = floor(SplitMix64_r(seed) * m / 2^64), where
 * SplitMix64_r(seed) = mix64(seed + (r + 1) * 0x9e3779b97f4a7c15).
 *   idx   host array of s int64 (caller-owned)
 * Returns RPCHOLQR_EINVAL if m < 1, s < 0 or idx is NULL with s > 0.  Touches no
 * device. */
int32_t rpcholqr_sample_indices(int64_t m, int64_t s, uint64_t seed, int64_t* idx);

/* Per-kernel timing with HIP events, for measurement.  While enabled, every
 * factor call records an event on its stream before the first kernel and after
 * each of its NSTAGES kernels (in order: sketch = sample + gather + sketch QR,
 * pass A = A1 and Gram partials, reduce = partial Gram sum, cholesky =
 * Cholesky, R2^{-1} and R product, pass B = Q = A1 R2^{-1} in place; with a
 * refined precision the last stage also holds the whole second pass).  No device memory is
 * allocated.  Process-wide state: do not time calls from several host threads
 * at once.
 *   rpcholqr_timing_enable(1) starts recording (and discards earlier records),
 *   rpcholqr_timing_enable(0) stops it; returns RPCHOLQR_OK or RPCHOLQR_EHIP.
 *   rpcholqr_timing_read(ms, count) waits for the recorded events, writes into
 *   ms[i] (host array of `count` doubles) the summed milliseconds of stage i
 *   over all calls recorded since the last read, clears the records, and
 *   returns the number of calls summed (negative rpcholqr_status on error). */
#define RPCHOLQR_NSTAGES 5
int32_t rpcholqr_timing_enable(int32_t on);
int32_t rpcholqr_timing_read(double* ms, int32_t count);

/* Batched factorization: many independent problems, one plan.  Not in the
 * paper; the use it serves is the one Section 1 motivates Cholesky-QR with,
 * block methods (block Krylov, LOBPCG) that need many thin QRs of modest size.
 * Each problem b is factored with exactly the arithmetic of rpcholqr_factor
 * (same sampling, sketch, row solves and info semantics); only the number of
 * row blocks over which the Gram matrix is partially summed differs, so Q and
 * R agree with rpcholqr_factor to rounding (about 1e-15).
 *
 * rpcholqr_batched_plan_create
 *   batch          number of problems (>= 1)
 *   m, n, s, seed, lda, ldq, ldr
 *                  HOST arrays of length batch, per problem as in
 *                  rpcholqr_factor (1 <= n <= 128, s <= 1536)
 *   A, Q, R        HOST arrays of length batch holding DEVICE pointers; within
 *                  a problem Q must not overlap A, R must not overlap A or Q;
 *                  different problems must not share Q or R memory
 *   precision      rpcholqr_precision
 *   plan           receives the plan
 *   bad_problem    optional; receives the index of the first invalid problem
 *                  (-1 if none)
 *   Validates every problem (EINVAL / EUNSUPPORTED), allocates the plan's device
 *   memory on the current device (descriptor tables and one workspace per
 *   problem, rpcholqr_batched_plan_device_bytes) and streams, and uploads the
 *   tables with blocking copies.  Launch shapes come from the tuning table
 *   (rpcholqr_batched_set_tuning).  The plan refers to the caller's A, Q and R, which must
 *   stay valid while it is executed.
 * rpcholqr_batched_execute
 *   Launches every problem (hipStream_t as void*): per column class one chain
 *   of launches (gather, sketch, pass A, Cholesky, pass B), the classes
 *   concurrently on streams the plan owns, forked from and joined to `stream`
 *   by events; no allocation and no host-to-device copy, so a stream capture
 *   into a HIP graph records it (with the fork and join).  info is a DEVICE
 *   array of batch rpcholqr_info, one per problem.  Executions of the same plan
 *   must not overlap (they share its workspace and streams).
 * rpcholqr_batched_plan_destroy frees the plan; the caller first waits for the
 *   work that uses it.
 * rpcholqr_factor_batched is create + execute + stream synchronize + destroy. */
typedef struct rpcholqr_batched_plan rpcholqr_batched_plan;

/* Launch shape of the batched passes for one column class and m bucket (not in
 * the paper; picked per GPU by the autotuner in paper_2406_11751_amd/autotune.py).
 *   nmax      column class: 16, 32, 48, 64 (n rounded up) or 128 (64 < n <= 128)
 *   m_max     the entry covers problems of the class with m <= m_max; a class's
 *             entries are searched in increasing m_max
 *   pa_rows   pass-A panel height: rows of one problem per pass-A workgroup (a
 *             multiple of 256); a problem gets ceil(m / pa_rows) workgroups,
 *             at most pa_max (1 .. 128), each writing one partial Gram matrix
 *   pb_rows   rows of one problem per pass-B workgroup (a multiple of 16)
 * The number of partials changes the order in which the Gram matrix is summed,
 * so results under different tunings agree to rounding (about 1e-15). */
typedef struct {
  int32_t nmax;
  int32_t reserved0;
  int64_t m_max;
  int32_t pa_rows;
  int32_t pa_max;
  int32_t pb_rows;
  int32_t reserved1;
} rpcholqr_batched_tuning;

/* Installs the tuning table used by every later rpcholqr_batched_plan_create
 * (process-wide; existing plans keep their shapes).  count = 0 restores the
 * built-in shapes (pa_rows 2048, pa_max 64, pb_rows 1024, or 2048 for the
 * 128-column class).  A class or m without an entry uses the built-in shape.
 * Returns RPCHOLQR_EINVAL for a malformed entry (the table is then unchanged). */
int32_t rpcholqr_batched_set_tuning(const rpcholqr_batched_tuning* entries, int32_t count);
int32_t rpcholqr_batched_plan_create(int64_t batch, const int64_t* m, const int64_t* n, const int64_t* s,
                                     const uint64_t* seed, const double* const* A, const int64_t* lda,
                                     double* const* Q, const int64_t* ldq, double* const* R, const int64_t* ldr,
                                     int32_t precision, rpcholqr_batched_plan** plan, int64_t* bad_problem);
int32_t rpcholqr_batched_execute(const rpcholqr_batched_plan* plan, rpcholqr_info* info, void* stream);
size_t rpcholqr_batched_plan_device_bytes(const rpcholqr_batched_plan* plan);
int32_t rpcholqr_batched_plan_destroy(rpcholqr_batched_plan* plan);
int32_t rpcholqr_factor_batched(int64_t batch, const int64_t* m, const int64_t* n, const int64_t* s,
                                const uint64_t* seed, const double* const* A, const int64_t* lda,
                                double* const* Q, const int64_t* ldq, double* const* R, const int64_t* ldr,
                                int32_t precision, rpcholqr_info* info, void* stream, int64_t* bad_problem);

#ifdef __cplusplus
}
#endif

#endif /* RPCHOLQR_H */

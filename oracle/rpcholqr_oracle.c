/*
 * Plain FP64 CPU oracle for randomized preconditioned Cholesky-QR
 * (Garrison & Ipsen, "A randomized preconditioned Cholesky-QR algorithm",
 * arXiv 2406.11751).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent checker of the GPU
 * library.  Only the test suite, the smoke entry point and the CPU-baseline leg
 * of the benchmark may load it.  The GPU library never links, calls or includes
 * anything from here, and this file includes nothing from the GPU library.
 *
 * Everything is IEEE binary64, column-major (element (i,j) of a matrix with
 * leading dimension ld sits at [i + j*ld]).  Build with
 *     gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp
 * so that every multiply-add that is not an explicit fma() is rounded twice.
 *
 * Structure follows the paper's algorithms:
 *   Algorithm "rpCholesky-QR" (Section 4):
 *     line 2  A_s = S F A         -> orc_sample_indices + orc_gather (F = I, see below)
 *     line 3  A_s = Q_s R_s       -> orc_householder_r + orc_sign_normalize
 *     lines 4-10 = Algorithm "Preconditioned Cholesky-QR" (Section 3.1) -> orc_alg1:
 *       line 2  A1 = A R_s^{-1}   -> orc_trsm_rows   (m row-wise triangular solves, Section 2.1)
 *       line 4  G1 = A1^T A1      -> orc_gram
 *       line 5  G1 = R2^T R2      -> orc_cholesky_upper
 *       line 6  Q  = A1 R2^{-1}   -> orc_trsm_rows
 *       line 8  R  = R2 R_s       -> orc_trmm_upper
 *
 * Readings where the paper is silent (each is also listed in the design notes):
 *  - The smoothing matrix F is the identity (rows of A are sampled directly),
 *    or, on request, F = H D with a Walsh-Hadamard H on A padded to a power of
 *    two rows (orc_smooth_sample).
 *  - Row indices come from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) in
 *    counter form, z_r = mix64(seed + (r+1)*0x9e3779b97f4a7c15), reduced to [0,m)
 *    by a 64x64->128-bit multiply-high (Lemire, ACM TOMACS 2019).  0-based.
 *  - The sample is scaled by sqrt(m/c) as in the paper's Matlab listing
 *    (Remark "r_exp", Section 5).
 *  - The thin QR of the sample is Householder QR with beta = -sign(alpha)*nu and
 *    dot products summed in a fixed 16-way interleaved order with a fixed
 *    pairwise tree (CR16 below); the resulting R_s is then made to have a
 *    positive diagonal by flipping row signs.
 *  - Triangular solves multiply by a correctly rounded reciprocal of the
 *    diagonal and accumulate with fma in ascending k.
 * Only these fixed orders make the result reproducible bit for bit by another
 * implementation; the paper's mathematics does not depend on them.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Status codes reported in *info_code. */
#define ORC_OK 0
#define ORC_ESKETCH 1 /* sketch QR: a Householder column norm is zero or not finite */
#define ORC_ECHOL 2   /* Cholesky of G1: a pivot is not positive or not finite */
#define ORC_EINVAL -1

#define AT(M, ld, i, j) ((M)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

/* ---------------------------------------------------------------------------
 * Sampling (Algorithm rpCholesky-QR line 2; Section 4: c rows sampled
 * uniformly, independently and with replacement).
 * ------------------------------------------------------------------------- */

/* SplitMix64 output number r (0-based) of the generator seeded with `seed`. */
uint64_t orc_splitmix64_at(uint64_t seed, uint64_t r) {
  uint64_t z = seed + (r + 1u) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

/* idx[r] = floor(z_r * m / 2^64), r = 0..s-1: uniform on {0,..,m-1}. */
void orc_sample_indices(int64_t m, int64_t s, uint64_t seed, int64_t* idx) {
  for (int64_t r = 0; r < s; ++r) {
    unsigned __int128 p = (unsigned __int128)orc_splitmix64_at(seed, (uint64_t)r) * (uint64_t)m;
    idx[r] = (int64_t)(uint64_t)(p >> 64);
  }
}

/* A_s = sqrt(m/c) * A(idx, :)  (Remark r_exp, Section 5), s x n, leading dimension s. */
void orc_gather(int64_t m, int64_t n, int64_t s, const int64_t* idx, const double* A, int64_t lda,
                double* As) {
  const double c = sqrt((double)m / (double)s);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t r = 0; r < s; ++r) AT(As, s, r, j) = c * AT(A, lda, idx[r], j);
}

/* ---------------------------------------------------------------------------
 * Smoothed sample (Algorithm rpCholesky-QR line 2 with F = F_T D; the remark
 * after Theorem t_prob: F_T a Walsh-Hadamard transform, D a diagonal of
 * independent random signs).  A is padded with zero rows to M = 2^p >= m rows;
 * F = H D P with H(k, q) = (-1)^popcount(k AND q) / sqrt(M) (Sylvester order)
 * and P the permutation moving row i to position pi(i) (orc_scramble) is
 * orthogonal on R^M, and only the c sampled rows of F [A; 0] are formed:
 *   A_s(r, j) = sqrt(M/c) (F [A;0])(idx_r, j) = T(r, j) / sqrt(c),
 *   T(r, j)   = sum_{i < m} D_i (-1)^popcount(idx_r AND pi(i)) A(i, j),
 * (D indexed by the row of A, a relabeling of the independent signs).  Without
 * P, rows k and k' of F A agree whenever k = k' mod 2^q and A lives in its
 * first 2^q rows, which makes the sampled matrix singular for such coherent
 * inputs; pi spreads every bit of i over all p bits.
 * with idx_r uniform on [0, M) (orc_sample_indices with M).  Every term is an
 * exact signed copy of A(i, j); the order of the sum is fixed:
 *   rows are cut into chunks of G * 4096 consecutive rows, G = max(1,
 *   ceil(ceil(m / 4096) / 256)) (so at most 256 chunks); within a chunk the
 *   terms are accumulated with fma in ascending i starting from 0; the chunk
 *   sums are then added in ascending chunk order (T = P_0, T = T + P_1, ...);
 *   finally A_s = T * (1 / sqrt(c)) with both operations correctly rounded.
 * D_i = +1 if bit 63 of SplitMix64 output i of the generator seeded with
 * (seed XOR ORC_SIGN_SALT) is 0, else -1. */
#define ORC_SIGN_SALT 0x5851f42d4c957f2dull
#define ORC_SMOOTH_BLOCK 4096

int64_t orc_smooth_rows(int64_t m) {
  int64_t M = 1;
  while (M < m) M <<= 1;
  return M;
}

/* pi(i) on p-bit integers (M = 2^p): multiply by an odd constant, xorshift,
 * multiply, xorshift, all mod M; each step is a bijection of [0, M). */
uint64_t orc_scramble(uint64_t i, int64_t M) {
  const uint64_t mask = (uint64_t)M - 1u;
  int p = 0;
  while (((int64_t)1 << p) < M) ++p;
  const int h = p / 2 > 1 ? p / 2 : 1;
  uint64_t x = (i * 0x9e3779b97f4a7c15ull) & mask;
  x ^= x >> h;
  x = (x * 0xbf58476d1ce4e5b9ull) & mask;
  x ^= x >> h;
  return x;
}

int64_t orc_smooth_chunk_rows(int64_t m) {
  const int64_t blocks = (m + ORC_SMOOTH_BLOCK - 1) / ORC_SMOOTH_BLOCK;
  int64_t g = (blocks + 255) / 256;
  if (g < 1) g = 1;
  return g * ORC_SMOOTH_BLOCK;
}

double orc_rademacher(uint64_t seed, int64_t i) {
  return (orc_splitmix64_at(seed ^ ORC_SIGN_SALT, (uint64_t)i) >> 63) ? -1.0 : 1.0;
}

/* Smoothed sample: idx[s] in [0, M) and As (s x n, ld s). */
void orc_smooth_sample(int64_t m, int64_t n, int64_t s, uint64_t seed, const double* A, int64_t lda,
                       int64_t* idx, double* As, int nthreads) {
  const int64_t M = orc_smooth_rows(m), chunk = orc_smooth_chunk_rows(m);
  const double sc = 1.0 / sqrt((double)s);
  double* D = (double*)malloc((size_t)m * sizeof(double));
  uint64_t* pi = (uint64_t*)malloc((size_t)m * sizeof(uint64_t));
  orc_sample_indices(M, s, seed, idx);
  for (int64_t i = 0; i < m; ++i) {
    D[i] = orc_rademacher(seed, i);
    pi[i] = orc_scramble((uint64_t)i, M);
  }
#pragma omp parallel for collapse(2) schedule(static) num_threads(nthreads)
  for (int64_t j = 0; j < n; ++j)
    for (int64_t r = 0; r < s; ++r) {
      const uint64_t k = (uint64_t)idx[r];
      double T = 0.0;
      for (int64_t c0 = 0; c0 < m; c0 += chunk) {
        const int64_t c1 = c0 + chunk < m ? c0 + chunk : m;
        double p = 0.0;
        for (int64_t i = c0; i < c1; ++i) {
          const double sg = (__builtin_popcountll(k & pi[i]) & 1) ? -D[i] : D[i];
          p = fma(sg, AT(A, lda, i, j), p);
        }
        T = (c0 == 0) ? p : T + p;
      }
      AT(As, s, r, j) = T * sc;
    }
  free(D);
  free(pi);
}

/* ---------------------------------------------------------------------------
 * Thin QR of the sample (Algorithm rpCholesky-QR line 3), R factor only.
 * ------------------------------------------------------------------------- */

/* CR16: sum over rows r = k..len-1 of x[r]*y[r].  Row r is accumulated with
 * fma into partial p[r mod 16] in ascending r; the 16 partials are then added
 * as a pairwise tree: p[i] += p[i+h] for h = 1, 2, 4, 8 and i a multiple of 2h.
 * Returns p[0]. */
static double cr16(const double* x, const double* y, int64_t k, int64_t len) {
  double p[16];
  for (int l = 0; l < 16; ++l) p[l] = 0.0;
  for (int64_t r = k; r < len; ++r) p[r % 16] = fma(x[r], y[r], p[r % 16]);
  for (int h = 1; h < 16; h *= 2)
    for (int i = 0; i < 16; i += 2 * h) p[i] = p[i] + p[i + h];
  return p[0];
}

/* Householder QR of the s x n matrix W (overwritten), upper triangle of the
 * n x n factor into Rs (leading dimension ldr; strictly lower part set to 0).
 * Returns ORC_OK, or ORC_ESKETCH with *bad_k = the column whose norm was zero
 * or not finite. */
int orc_householder_r(int64_t s, int64_t n, double* W, int64_t ldw, double* Rs, int64_t ldr,
                      int32_t* bad_k) {
  double* v = (double*)malloc((size_t)s * sizeof(double));
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) AT(Rs, ldr, i, j) = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    double* wk = &AT(W, ldw, 0, k);
    double nu2 = cr16(wk, wk, k, s);
    if (nu2 == 0.0 || !isfinite(nu2)) {
      *bad_k = (int32_t)k;
      free(v);
      return ORC_ESKETCH;
    }
    double nu = sqrt(nu2);
    double alpha = wk[k];
    double beta = (alpha >= 0.0) ? -nu : nu;
    double d = 1.0 / (alpha - beta);
    v[k] = 1.0;
    for (int64_t r = k + 1; r < s; ++r) v[r] = wk[r] * d;
    double tau = (beta - alpha) / beta;
    AT(Rs, ldr, k, k) = beta;
    /* Apply H_k = I - tau v v^T to the remaining columns. */
    for (int64_t j = k + 1; j < n; ++j) {
      double* wj = &AT(W, ldw, 0, j);
      double t = tau * cr16(v, wj, k, s);
      for (int64_t r = k; r < s; ++r) wj[r] = fma(-t, v[r], wj[r]);
      AT(Rs, ldr, k, j) = wj[k];
    }
  }
  free(v);
  return ORC_OK;
}

/* Make diag(R) positive by negating rows (exact).  With a positive diagonal
 * the thin QR factor is unique (Lemma l_r1r2, Section 2.1). */
void orc_sign_normalize(int64_t n, double* R, int64_t ldr) {
  for (int64_t k = 0; k < n; ++k)
    if (AT(R, ldr, k, k) < 0.0)
      for (int64_t j = k; j < n; ++j) AT(R, ldr, k, j) = -AT(R, ldr, k, j);
}

/* ---------------------------------------------------------------------------
 * Algorithm "Preconditioned Cholesky-QR" (Section 3.1).
 * ------------------------------------------------------------------------- */

/* X = B U^{-1} for upper triangular U, computed as m independent solves
 * U^T x_i^T = b_i^T, one per row (Section 2.1, Algorithm "Basic Cholesky-QR"
 * discussion).  Per row: x_j = (b_j - sum_{k<j} x_k U(k,j)) * (1/U(j,j)), the
 * sum accumulated with fma in ascending k starting from b_j.  X may alias B
 * only if ldx == ldb. */
void orc_trsm_rows(int64_t m, int64_t n, const double* B, int64_t ldb, const double* U, int64_t ldu,
                   double* X, int64_t ldx, int nthreads) {
  double* rinv = (double*)malloc((size_t)n * sizeof(double));
  for (int64_t j = 0; j < n; ++j) rinv[j] = 1.0 / AT(U, ldu, j, j);
#pragma omp parallel num_threads(nthreads)
  {
    double* x = (double*)malloc((size_t)n * sizeof(double));
#pragma omp for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
      for (int64_t j = 0; j < n; ++j) {
        double t = AT(B, ldb, i, j);
        for (int64_t k = 0; k < j; ++k) t = fma(-x[k], AT(U, ldu, k, j), t);
        x[j] = t * rinv[j];
      }
      for (int64_t j = 0; j < n; ++j) AT(X, ldx, i, j) = x[j];
    }
    free(x);
  }
  free(rinv);
}

/* G = X^T X, upper triangle (strictly lower part set to 0).  Each entry is a
 * plain sum over rows i = 0..m-1 in ascending order. */
void orc_gram(int64_t m, int64_t n, const double* X, int64_t ldx, double* G, int64_t ldg,
              int nthreads) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = j + 1; i < n; ++i) AT(G, ldg, i, j) = 0.0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t jj = 0; jj < n * n; ++jj) {
    int64_t a = jj % n, b = jj / n;
    if (a > b) continue;
    const double* xa = &AT(X, ldx, 0, a);
    const double* xb = &AT(X, ldx, 0, b);
    double acc = 0.0;
    for (int64_t i = 0; i < m; ++i) acc += xa[i] * xb[i];
    AT(G, ldg, a, b) = acc;
  }
}

/* Upper Cholesky G = R^T R without pivoting or shifting, reading the upper
 * triangle of G.  Returns ORC_OK or ORC_ECHOL with *bad_j = first column whose
 * pivot is not positive (or not finite). */
int orc_cholesky_upper(int64_t n, const double* G, int64_t ldg, double* R, int64_t ldr,
                       int32_t* bad_j) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) AT(R, ldr, i, j) = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    for (int64_t i = 0; i < j; ++i) {
      double t = AT(G, ldg, i, j);
      for (int64_t k = 0; k < i; ++k) t -= AT(R, ldr, k, i) * AT(R, ldr, k, j);
      AT(R, ldr, i, j) = t / AT(R, ldr, i, i);
    }
    double d = AT(G, ldg, j, j);
    for (int64_t k = 0; k < j; ++k) d -= AT(R, ldr, k, j) * AT(R, ldr, k, j);
    if (!(d > 0.0) || !isfinite(d)) {
      *bad_j = (int32_t)j;
      return ORC_ECHOL;
    }
    AT(R, ldr, j, j) = sqrt(d);
  }
  return ORC_OK;
}

/* C = U V for upper triangular U and V (C upper, strictly lower part 0). */
void orc_trmm_upper(int64_t n, const double* U, int64_t ldu, const double* V, int64_t ldv, double* C,
                    int64_t ldc) {
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      if (i <= j)
        for (int64_t k = i; k <= j; ++k) acc += AT(U, ldu, i, k) * AT(V, ldv, k, j);
      AT(C, ldc, i, j) = acc;
    }
}

/* Algorithm "Preconditioned Cholesky-QR" with a given nonsingular upper
 * triangular R_s.  Q is m x n (ldq), R is n x n (ldr).  Optional outputs
 * (NULL to skip): A1 (m x n, ld m), G1 and R2 (n x n, ld n).
 * Returns ORC_OK or ORC_ECHOL (bad index in *info_index). */
int orc_alg1(int64_t m, int64_t n, const double* A, int64_t lda, const double* Rs, int64_t ldrs,
             double* Q, int64_t ldq, double* R, int64_t ldr, double* A1_out, double* G1_out,
             double* R2_out, int32_t* info_index, int nthreads) {
  double* A1 = A1_out ? A1_out : (double*)malloc((size_t)m * (size_t)n * sizeof(double));
  double* G1 = G1_out ? G1_out : (double*)malloc((size_t)n * (size_t)n * sizeof(double));
  double* R2 = R2_out ? R2_out : (double*)malloc((size_t)n * (size_t)n * sizeof(double));
  int rc;
  orc_trsm_rows(m, n, A, lda, Rs, ldrs, A1, m, nthreads);  /* line 2 */
  orc_gram(m, n, A1, m, G1, n, nthreads);                   /* line 4 */
  rc = orc_cholesky_upper(n, G1, n, R2, n, info_index);     /* line 5 */
  if (rc == ORC_OK) {
    orc_trsm_rows(m, n, A1, m, R2, n, Q, ldq, nthreads);     /* line 6 */
    orc_trmm_upper(n, R2, n, Rs, ldrs, R, ldr);              /* line 8 */
  }
  if (!A1_out) free(A1);
  if (!G1_out) free(G1);
  if (!R2_out) free(R2);
  return rc;
}

/* Algorithm "rpCholesky-QR" (Section 4) with F = I.
 * Inputs: A (m x n, lda >= m), sample count s >= n, seed.
 * Outputs: Q (m x n, ldq), R (n x n upper, ldr).
 * Optional diagnostics (NULL to skip): idx[s], As (s x n, ld s), Rs (n x n, ld n),
 * A1 (m x n, ld m), G1 and R2 (n x n, ld n).
 * Returns ORC_OK, ORC_EINVAL, ORC_ESKETCH or ORC_ECHOL; *info_index gets the
 * failing column for the last two. */
int orc_rpcholqr_ex(int64_t m, int64_t n, int64_t s, uint64_t seed, int smooth, const double* A, int64_t lda,
                    double* Q, int64_t ldq, double* R, int64_t ldr, int64_t* idx_out, double* As_out,
                    double* Rs_out, double* A1_out, double* G1_out, double* R2_out, int32_t* info_index,
                    int nthreads);

int orc_rpcholqr(int64_t m, int64_t n, int64_t s, uint64_t seed, const double* A, int64_t lda,
                 double* Q, int64_t ldq, double* R, int64_t ldr, int64_t* idx_out, double* As_out,
                 double* Rs_out, double* A1_out, double* G1_out, double* R2_out, int32_t* info_index,
                 int nthreads) {
  return orc_rpcholqr_ex(m, n, s, seed, 0, A, lda, Q, ldq, R, ldr, idx_out, As_out, Rs_out, A1_out, G1_out,
                         R2_out, info_index, nthreads);
}

/* As orc_rpcholqr; with smooth != 0 the sample is the smoothed one
 * (orc_smooth_sample) instead of A's own rows. */
int orc_rpcholqr_ex(int64_t m, int64_t n, int64_t s, uint64_t seed, int smooth, const double* A, int64_t lda,
                    double* Q, int64_t ldq, double* R, int64_t ldr, int64_t* idx_out, double* As_out,
                    double* Rs_out, double* A1_out, double* G1_out, double* R2_out, int32_t* info_index,
                    int nthreads) {
  int rc;
  int64_t* idx;
  double *As, *Rs;
  *info_index = -1;
  if (n < 1 || m < n || s < n || lda < m || ldq < m || ldr < n) return ORC_EINVAL;
  idx = idx_out ? idx_out : (int64_t*)malloc((size_t)s * sizeof(int64_t));
  As = (double*)malloc((size_t)s * (size_t)n * sizeof(double));
  Rs = Rs_out ? Rs_out : (double*)malloc((size_t)n * (size_t)n * sizeof(double));
  if (smooth) {
    orc_smooth_sample(m, n, s, seed, A, lda, idx, As, nthreads); /* line 2, F = F_T D */
  } else {
    orc_sample_indices(m, s, seed, idx);        /* line 2: which rows */
    orc_gather(m, n, s, idx, A, lda, As);       /* line 2: scaled sample (F = I) */
  }
  if (As_out) memcpy(As_out, As, (size_t)s * (size_t)n * sizeof(double));
  rc = orc_householder_r(s, n, As, s, Rs, n, info_index); /* line 3 */
  if (rc == ORC_OK) {
    orc_sign_normalize(n, Rs, n);
    rc = orc_alg1(m, n, A, lda, Rs, n, Q, ldq, R, ldr, A1_out, G1_out, R2_out, info_index,
                  nthreads);                    /* lines 4-10 */
  }
  if (!idx_out) free(idx);
  free(As);
  if (!Rs_out) free(Rs);
  return rc;
}

/* Thread count actually available to OpenMP (1 without OpenMP). */
int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

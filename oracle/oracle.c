/*
 * oracle.c -- plain, slow, CPU reference for semiring matrix multiplication
 * and Strassen's algorithm, written from the paper "Balanced Partitioning of
 * Several Cache-Oblivious Algorithms" (Tang & Gao).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library calls this code.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no source, header, table or helper with the GPU library.
 *
 * What it computes (section "PACO MM", problem statement): C = A (x) B over a
 * closed semiring (S, (+), (x), 0, 1) with A n-by-k, B k-by-m, C n-by-m; every
 * matrix is row-major with an explicit leading dimension.  Each entry is the
 * plain definition, an ascending-l fold
 *
 *     C[i][j] = 0  (+)  A[i][0] (x) B[0][j]  (+)  ...  (+)  A[i][k-1] (x) B[k-1][j]
 *
 * with no blocking, no reordering and no partitioning.  The PACO partition does
 * not change this value for the integer semirings, and changes only rounding
 * for the (+,x) ring.  When `accumulate` is set the fold starts from the old
 * C[i][j] instead of 0, which gives C <- C (+) A (x) B (the experiments section
 * computes C = C + A x B).  k = 0 leaves the empty fold: 0, or the old C.
 *
 * The paper does not fix the semiring constants.  The readings used here:
 *   (min,+) int32: 0 = INF = 2^30, (x) is the saturating add min(a+b, INF),
 *                  domain {0 .. 2^30}.  Arithmetic in int64, so a+b cannot
 *                  overflow.
 *   (max,+) int32: 0 = NEG_INF = -2^30, (x) is a+b when both are finite and
 *                  NEG_INF when either is NEG_INF (NEG_INF absorbs), finite
 *                  domain [-2^28, 2^28].  Arithmetic in int64.
 *   boolean:       (+) = OR, (x) = AND, 0 = false.
 *   (+,x) ring:    IEEE binary64 for every product and sum (products of two
 *                  binary32 values are exact in binary64).
 *
 * Strassen (section "PACO Strassen"): the seven products of the 1-based
 * formulas S1..S7, T1..T7, M_r = S_r (x) T_r and the four quadrant sums of C,
 * applied recursively for a given number of levels and finished by the
 * classic triple loop.
 *
 * Loops over i may run under OpenMP; each C[i][j] is still one sequential fold.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_INF ((int64_t)1 << 30)
#define OR_NEG_INF (-((int64_t)1 << 30))

/* ---------------------------------------------------------------- (min,+) */
static int64_t minplus_mul(int64_t a, int64_t b) {
  int64_t s = a + b;
  return s < OR_INF ? s : OR_INF;
}

void oracle_minplus(int64_t n, int64_t m, int64_t k,
                    const int32_t* A, int64_t lda,
                    const int32_t* B, int64_t ldb,
                    int32_t* C, int64_t ldc, int accumulate) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < m; ++j) {
      int64_t acc = accumulate ? (int64_t)C[i * ldc + j] : OR_INF;
      for (int64_t l = 0; l < k; ++l) {
        int64_t t = minplus_mul(A[i * lda + l], B[l * ldb + j]);
        if (t < acc) acc = t;
      }
      C[i * ldc + j] = (int32_t)acc;
    }
  }
}

/* ---------------------------------------------------------------- (max,+) */
static int64_t maxplus_mul(int64_t a, int64_t b) {
  if (a == OR_NEG_INF || b == OR_NEG_INF) return OR_NEG_INF;
  return a + b;
}

void oracle_maxplus(int64_t n, int64_t m, int64_t k,
                    const int32_t* A, int64_t lda,
                    const int32_t* B, int64_t ldb,
                    int32_t* C, int64_t ldc, int accumulate) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < m; ++j) {
      int64_t acc = accumulate ? (int64_t)C[i * ldc + j] : OR_NEG_INF;
      for (int64_t l = 0; l < k; ++l) {
        int64_t t = maxplus_mul(A[i * lda + l], B[l * ldb + j]);
        if (t > acc) acc = t;
      }
      C[i * ldc + j] = (int32_t)acc;
    }
  }
}

/* ---------------------------------------------------------------- boolean */
/* Bit-by-bit definition on unpacked 0/1 bytes. */
void oracle_bool_bits(int64_t n, int64_t m, int64_t k,
                      const uint8_t* A, const uint8_t* B, uint8_t* C,
                      int accumulate) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j < m; ++j) {
      int acc = accumulate ? (C[i * m + j] != 0) : 0;
      for (int64_t l = 0; l < k; ++l)
        acc = acc | ((A[i * k + l] != 0) & (B[l * m + j] != 0));
      C[i * m + j] = (uint8_t)acc;
    }
  }
}

/* Packed layout: row r of an R-by-W bit matrix is ceil(W/32) uint32 words,
 * bit w of the row is bit (w % 32) of word (w / 32), least significant first.
 * Row-OR form of the same definition: row i of C is the OR of the rows l of B
 * for which bit l of row i of A is set.  Padding bits of C are written 0. */
void oracle_bool_packed(int64_t n, int64_t m, int64_t k,
                        const uint32_t* A, const uint32_t* B, uint32_t* C,
                        int accumulate) {
  int64_t kw = (k + 31) / 32, mw = (m + 31) / 32;
  uint32_t last_mask = (m % 32) ? ((1u << (m % 32)) - 1u) : 0xffffffffu;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i) {
    uint32_t* c = C + i * mw;
    if (!accumulate)
      for (int64_t w = 0; w < mw; ++w) c[w] = 0;
    for (int64_t l = 0; l < k; ++l) {
      if ((A[i * kw + l / 32] >> (l % 32)) & 1u) {
        const uint32_t* b = B + l * mw;
        for (int64_t w = 0; w < mw; ++w) c[w] |= b[w];
      }
    }
    if (mw > 0) c[mw - 1] &= last_mask;
  }
}

/* ---------------------------------------------------------------- ring */
/* C64[i][j] = sum_l A[i][l]*B[l][j] in binary64, ascending l; when absC is
 * not NULL it also receives sum_l |A[i][l]|*|B[l][j]| (the scale used for
 * the componentwise error bound).  Only the `nrows` rows listed in `rows`
 * are computed (rows == NULL means all n rows); output row r of C64 is input
 * row rows[r]. */
void oracle_ring_f64(int64_t n, int64_t m, int64_t k,
                     const float* A, int64_t lda,
                     const float* B, int64_t ldb,
                     const int64_t* rows, int64_t nrows,
                     double* C64, double* absC) {
  if (rows == NULL) nrows = n;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r = 0; r < nrows; ++r) {
    int64_t i = rows ? rows[r] : r;
    for (int64_t j = 0; j < m; ++j) {
      double acc = 0.0, aacc = 0.0;
      for (int64_t l = 0; l < k; ++l) {
        double p = (double)A[i * lda + l] * (double)B[l * ldb + j];
        acc += p;
        aacc += fabs(p);
      }
      C64[r * m + j] = acc;
      if (absC) absC[r * m + j] = aacc;
    }
  }
}

/* Same fold on binary64 operands (used by the Strassen oracle's leaves and
 * by callers holding binary64 data). */
void oracle_ring_f64_dd(int64_t n, int64_t m, int64_t k,
                        const double* A, int64_t lda,
                        const double* B, int64_t ldb,
                        double* C, int64_t ldc) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < m; ++j) {
      double acc = 0.0;
      for (int64_t l = 0; l < k; ++l) acc += A[i * lda + l] * B[l * ldb + j];
      C[i * ldc + j] = acc;
    }
}

void oracle_ring_i64(int64_t n, int64_t m, int64_t k,
                     const int64_t* A, int64_t lda,
                     const int64_t* B, int64_t ldb,
                     int64_t* C, int64_t ldc) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < m; ++j) {
      int64_t acc = 0;
      for (int64_t l = 0; l < k; ++l) acc += A[i * lda + l] * B[l * ldb + j];
      C[i * ldc + j] = acc;
    }
}

/* ---------------------------------------------------------------- Strassen */
/* One level of Strassen on an h-by-h quadrant split of n-by-n matrices
 * (n = 2h), written once for binary64 and once for int64 through a macro of
 * the element type.  Quadrant X_ab of a matrix X with leading dimension ld
 * starts at X + a*h*ld + b*h.  The level uses the 1-based formulas:
 *   S1 = A00+A11  S2 = A10+A11  S3 = A00      S4 = A11
 *   S5 = A00+A01  S6 = A10-A00  S7 = A01-A11
 *   T1 = B00+B11  T2 = B00      T3 = B01-B11  T4 = B10-B00
 *   T5 = B11      T6 = B00+B01  T7 = B10+B11
 *   M_r = S_r T_r
 *   C00 = M1+M4-M5+M7   C01 = M3+M5   C10 = M2+M4   C11 = M1+M3-M2+M6
 */
#define DEFINE_STRASSEN(NAME, T, LEAF)                                          \
  static void NAME##_add(int64_t h, const T* X, int64_t ldx, int sx,            \
                         const T* Y, int64_t ldy, int sy, T* Z) {               \
    for (int64_t i = 0; i < h; ++i)                                             \
      for (int64_t j = 0; j < h; ++j) {                                         \
        T v = 0;                                                                \
        if (sx) v = (sx > 0) ? X[i * ldx + j] : -X[i * ldx + j];                \
        if (sy) v = (sy > 0) ? v + Y[i * ldy + j] : v - Y[i * ldy + j];         \
        Z[i * h + j] = v;                                                       \
      }                                                                         \
  }                                                                             \
  static void NAME##_rec(int64_t n, const T* A, int64_t lda, const T* B,        \
                         int64_t ldb, T* C, int64_t ldc, int levels) {          \
    if (levels <= 0 || n % 2 != 0) {                                            \
      LEAF(n, n, n, A, lda, B, ldb, C, ldc);                                    \
      return;                                                                   \
    }                                                                           \
    int64_t h = n / 2;                                                          \
    const T *A00 = A, *A01 = A + h, *A10 = A + h * lda, *A11 = A + h * lda + h; \
    const T *B00 = B, *B01 = B + h, *B10 = B + h * ldb, *B11 = B + h * ldb + h; \
    T* buf = (T*)malloc(sizeof(T) * (size_t)(h * h) * 9);                       \
    T *S = buf, *Tm = buf + h * h, *M = buf + 2 * h * h;                        \
    /* S_r, T_r as (first operand, sign, second operand, sign). */              \
    const T* sa[7] = {A00, A10, A00, A11, A00, A10, A01};                       \
    const T* sb[7] = {A11, A11, A00, A11, A01, A00, A11};                       \
    int ss[7][2] = {{1, 1}, {1, 1}, {1, 0}, {1, 0}, {1, 1}, {1, -1}, {1, -1}};  \
    const T* ta[7] = {B00, B00, B01, B10, B11, B00, B10};                       \
    const T* tb[7] = {B11, B00, B11, B00, B11, B01, B11};                       \
    int ts[7][2] = {{1, 1}, {1, 0}, {1, -1}, {1, -1}, {1, 0}, {1, 1}, {1, 1}};  \
    for (int r = 0; r < 7; ++r) {                                               \
      NAME##_add(h, sa[r], lda, ss[r][0], sb[r], lda, ss[r][1], S);             \
      NAME##_add(h, ta[r], ldb, ts[r][0], tb[r], ldb, ts[r][1], Tm);            \
      NAME##_rec(h, S, h, Tm, h, M + r * h * h, h, levels - 1);                 \
    }                                                                           \
    const T *M1 = M, *M2 = M + h * h, *M3 = M + 2 * h * h, *M4 = M + 3 * h * h; \
    const T *M5 = M + 4 * h * h, *M6 = M + 5 * h * h, *M7 = M + 6 * h * h;      \
    for (int64_t i = 0; i < h; ++i)                                             \
      for (int64_t j = 0; j < h; ++j) {                                         \
        int64_t e = i * h + j;                                                  \
        C[i * ldc + j] = M1[e] + M4[e] - M5[e] + M7[e];                         \
        C[i * ldc + h + j] = M3[e] + M5[e];                                     \
        C[(h + i) * ldc + j] = M2[e] + M4[e];                                   \
        C[(h + i) * ldc + h + j] = M1[e] + M3[e] - M2[e] + M6[e];               \
      }                                                                         \
    free(buf);                                                                  \
  }

DEFINE_STRASSEN(strassen_f64, double, oracle_ring_f64_dd)
DEFINE_STRASSEN(strassen_i64, int64_t, oracle_ring_i64)

/* C = A B for n-by-n row-major matrices through `levels` Strassen levels
 * (fewer if n stops being even), classic triple loop below. */
void oracle_strassen_f64(int64_t n, const double* A, const double* B,
                         double* C, int levels) {
  strassen_f64_rec(n, A, n, B, n, C, n, levels);
}

void oracle_strassen_i64(int64_t n, const int64_t* A, const int64_t* B,
                         int64_t* C, int levels) {
  strassen_i64_rec(n, A, n, B, n, C, n, levels);
}

/* ------------------------------------------------------------- 1D problem */
/* Section "PACO 1D", equation (1D): given D[0] and a weight function w that
 * needs no memory, D[j] = min over 0 <= i < j of D[i] + w(i, j), j = 1..n.
 *
 * Readings (the section states w real-valued and otherwise leaves it open):
 *   values are integers, with the (min,+) semiring's INF = 2^30 as "no
 *   path" and saturating sums min(D[i] + w, INF), int64 arithmetic;
 *   two weight families, both O(1) with no memory access:
 *     kind 0, affine:  w(i, j) = a + b (j - i), saturated at INF
 *     kind 1, hashed:  w(i, j) = a + (fmix32(key) mod 2^b) with
 *                      key = (i * 0x9E3779B9 + j) mod 2^32, XOR seed, and
 *                      fmix32 the published MurmurHash3 32-bit finaliser
 *                      (Appleby): h ^= h >> 16; h *= 0x85EBCA6B;
 *                      h ^= h >> 13; h *= 0xC2B2AE35; h ^= h >> 16.
 */
static uint32_t or_fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

uint32_t oracle_fmix32(uint32_t h) { return or_fmix32(h); }

static int64_t dp_w(int kind, int64_t a, int64_t b, uint32_t seed, int64_t i, int64_t j) {
  int64_t w;
  if (kind == 0) {
    w = a + b * (j - i);
  } else {
    const uint32_t key = ((uint32_t)i * 0x9E3779B9u + (uint32_t)j) ^ seed;
    const uint32_t mask = b >= 32 ? 0xFFFFFFFFu : (((uint32_t)1 << b) - 1u);
    w = a + (int64_t)(or_fmix32(key) & mask);
  }
  return w < OR_INF ? w : OR_INF;
}

int64_t oracle_dp1d_w(int kind, int64_t a, int64_t b, uint32_t seed, int64_t i, int64_t j) {
  return dp_w(kind, a, b, seed, i, j);
}

/* min over 0 <= i < j of min(D[i] + w(i, j), INF); INF when j = 0 */
static int64_t dp1d_at(int kind, int64_t a, int64_t b, uint32_t seed, const int32_t* D, int64_t j) {
  int64_t acc = OR_INF;
#pragma omp parallel for reduction(min : acc) if (j > 8192)
  for (int64_t i = 0; i < j; ++i) {
    int64_t t = (int64_t)D[i] + dp_w(kind, a, b, seed, i, j);
    if (t > OR_INF) t = OR_INF;
    if (t < acc) acc = t;
  }
  return acc;
}

/* D has n + 1 entries: D[0] is read, D[1..n] are written in ascending j. */
void oracle_dp1d(int64_t n, int kind, int64_t a, int64_t b, uint32_t seed, int32_t* D) {
  for (int64_t j = 1; j <= n; ++j) D[j] = (int32_t)dp1d_at(kind, a, b, seed, D, j);
}

/* For each listed j >= 1, whether D[j] equals the recurrence applied to the
 * given D[0..j-1]; returns how many do not. */
int64_t oracle_dp1d_check(int kind, int64_t a, int64_t b, uint32_t seed, const int32_t* D,
                          const int64_t* js, int64_t count) {
  int64_t bad = 0;
  for (int64_t t = 0; t < count; ++t)
    if (js[t] >= 1 && (int64_t)D[js[t]] != dp1d_at(kind, a, b, seed, D, js[t])) ++bad;
  return bad;
}

/* -------------------------------------------------------------- GAP problem */
/* Section "PACO GAP", equation (gap): D[0][0] = d0 and, for 0 <= i <= m,
 * 0 <= j <= n, (i, j) != (0, 0),
 *   D[i][j] = min( D[i-1][j-1] + s(i, j)           (i, j >= 1),
 *                  min over q < j of D[i][q] + w(q, j),
 *                  min over p < i of D[p][j] + w'(p, i) ),
 * saturated at INF.  w and w' are weight functions of the 1D problem's two
 * families (kind, a, b, seed each).  Reading for s (the section only asks
 * for O(1) with no memory): the substitution cost of two symbol sequences,
 * x_i = fmix32(i XOR sx) mod 2^bits and y_j = fmix32(j XOR sy) mod 2^bits,
 * s(i, j) = s_match when x_i = y_j, else s_mismatch.  D is row-major with
 * leading dimension ld >= n + 1, filled in row-major order (every term is
 * then already final). */
static int64_t gap_s(int64_t sm, int64_t sx, int bits, uint32_t seedx, uint32_t seedy, int64_t i, int64_t j) {
  const uint32_t mask = bits >= 32 ? 0xFFFFFFFFu : (((uint32_t)1 << bits) - 1u);
  const uint32_t xi = or_fmix32((uint32_t)i ^ seedx) & mask;
  const uint32_t yj = or_fmix32((uint32_t)j ^ seedy) & mask;
  return xi == yj ? sm : sx;
}

int64_t oracle_gap_s(int64_t sm, int64_t sx, int bits, uint32_t seedx, uint32_t seedy, int64_t i, int64_t j) {
  return gap_s(sm, sx, bits, seedx, seedy, i, j);
}

/* one cell from its row prefix, column prefix and diagonal neighbour */
static int64_t gap_cell(int64_t m, int64_t n, const int32_t* D, int64_t ld, int64_t i, int64_t j,
                        const int64_t* wr, const int64_t* wc, const int64_t* sp) {
  (void)m; (void)n;
  int64_t best = OR_INF;
  if (i >= 1 && j >= 1) {
    int64_t t = (int64_t)D[(i - 1) * ld + (j - 1)] +
                gap_s(sp[0], sp[1], (int)sp[2], (uint32_t)sp[3], (uint32_t)sp[4], i, j);
    if (t < best) best = t;
  }
  for (int64_t q = 0; q < j; ++q) {
    int64_t t = (int64_t)D[i * ld + q] + dp_w((int)wr[0], wr[1], wr[2], (uint32_t)wr[3], q, j);
    if (t < best) best = t;
  }
  for (int64_t p = 0; p < i; ++p) {
    int64_t t = (int64_t)D[p * ld + j] + dp_w((int)wc[0], wc[1], wc[2], (uint32_t)wc[3], p, i);
    if (t < best) best = t;
  }
  return best < OR_INF ? best : OR_INF;
}

/* wr, wc: (kind, a, b, seed) of w and w'; sp: (s_match, s_mismatch, bits,
 * seed x, seed y).  D[0][0] is read; every other entry of the (m+1) x (n+1)
 * grid is written. */
void oracle_gap(int64_t m, int64_t n, const int64_t* wr, const int64_t* wc, const int64_t* sp,
                int32_t* D, int64_t ld) {
  for (int64_t i = 0; i <= m; ++i)
    for (int64_t j = 0; j <= n; ++j)
      if (i != 0 || j != 0) D[i * ld + j] = (int32_t)gap_cell(m, n, D, ld, i, j, wr, wc, sp);
}

/* how many listed cells (pairs of i, j) differ from the recurrence applied
 * to the given D */
int64_t oracle_gap_check(int64_t m, int64_t n, const int64_t* wr, const int64_t* wc, const int64_t* sp,
                         const int32_t* D, int64_t ld, const int64_t* cells, int64_t count) {
  int64_t bad = 0;
#pragma omp parallel for reduction(+ : bad)
  for (int64_t t = 0; t < count; ++t) {
    const int64_t i = cells[2 * t], j = cells[2 * t + 1];
    if (i == 0 && j == 0) continue;
    if ((int64_t)D[i * ld + j] != gap_cell(m, n, D, ld, i, j, wr, wc, sp)) ++bad;
  }
  return bad;
}

/* Threads for the OpenMP loops that follow (no effect without OpenMP). */
void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* Threads an OpenMP loop of this library runs on (1 without OpenMP). */
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

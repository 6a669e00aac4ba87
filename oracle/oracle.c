/*
 * CPU oracle for the triangular solve L X = B.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library.  The GPU library never links, includes or calls it, and
 * it shares no code, header or constant with the GPU path.
 *
 * Problem statement (Sec. I, Introduction): L is an n x n lower-triangular
 * matrix, B and X are dense n x k matrices, and X solves L X = B.  The
 * inversion-based method of Sec. VI (Alg. It-Inv-TRSM) ensures B = L X, i.e.
 * it reaches X = L^{-1} B exactly up to rounding order, so the oracle is that
 * plain definition written out: forward substitution,
 *
 *     x[i][c] = ( b[i][c] - sum_{j<i} l[i][j] * x[j][c] ) / l[i][i],
 *
 * with i ascending, the sum taken with j ascending, IEEE binary64 arithmetic,
 * a true division, and no contraction into fused multiply-adds (the build
 * uses -ffp-contract=off -fno-fast-math).
 *
 * Threads split the right-hand-side columns: the column split of
 * Sec. II-C.4 (L [X1 X2] = [B1 B2] gives two independent solves).  Every column
 * is computed by exactly the same sequence of operations whatever the thread
 * count, so the result is bitwise identical to a serial run.
 *
 * Storage is row-major with leading dimensions: element (i,j) of L is
 * L[i*ldl + j], of B is B[i*ldb + c], of X is X[i*ldx + c].  Entries of L above
 * the diagonal are never read.
 *
 * Only the lower triangle including the diagonal is read; a zero diagonal
 * entry simply produces IEEE infinities / NaNs (no pivoting, no scaling).
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <stdlib.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Column-chunk width a thread works on at a time.  Any width gives the same
 * bits: each column's arithmetic does not depend on its neighbours. */
#define ORACLE_COLS 64

static int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }

/* Forward substitution on columns [c0, c1).  Row i of X is used as the running
 * value of every column's sum: it starts at b[i][c], then for j = 0..i-1 in
 * order subtracts the rounded product l[i][j]*x[j][c], then is divided by
 * l[i][i]. */
static void subst_cols_f64(int64_t n, int64_t c0, int64_t c1,
                           const double* L, int64_t ldl,
                           const double* B, int64_t ldb,
                           double* X, int64_t ldx) {
  for (int64_t i = 0; i < n; ++i) {
    double* xi = X + i * ldx;
    const double* bi = B + i * ldb;
    const double* li = L + i * ldl;
    if (xi != bi)
      for (int64_t c = c0; c < c1; ++c) xi[c] = bi[c];
    for (int64_t j = 0; j < i; ++j) {
      const double lij = li[j];
      const double* xj = X + j * ldx;
      for (int64_t c = c0; c < c1; ++c) {
        double prod = lij * xj[c];
        xi[c] = xi[c] - prod;
      }
    }
    const double d = li[i];
    for (int64_t c = c0; c < c1; ++c) xi[c] = xi[c] / d;
  }
}

/* X = L^{-1} B by forward substitution (Sec. I problem statement).  X may be
 * the same buffer as B (with ldx == ldb).  Returns 0, or -1 on bad sizes. */
int oracle_trsm_f64(int64_t n, int64_t k,
                    const double* L, int64_t ldl,
                    const double* B, int64_t ldb,
                    double* X, int64_t ldx, int nthreads) {
  if (n < 0 || k < 0) return -1;
  if (n == 0 || k == 0) return 0;
  if (ldl < n || ldb < k || ldx < k) return -1;
  const int64_t nchunks = (k + ORACLE_COLS - 1) / ORACLE_COLS;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    const int64_t c0 = ch * ORACLE_COLS;
    const int64_t c1 = min64(k, c0 + ORACLE_COLS);
    subst_cols_f64(n, c0, c1, L, ldl, B, ldb, X, ldx);
  }
  (void)nthreads;
  return 0;
}

/* Backward substitution with the transpose of L on columns [c0, c1): the
 * solve L^T X = B, L^T upper triangular with (L^T)[i][j] = l[j][i].  Row i
 * of X (i descending) starts at b[i][c], then for j = i+1..n-1 in order
 * subtracts the rounded product l[j][i]*x[j][c], then is divided by l[i][i]. */
static void subst_t_cols_f64(int64_t n, int64_t c0, int64_t c1,
                             const double* L, int64_t ldl,
                             const double* B, int64_t ldb,
                             double* X, int64_t ldx) {
  for (int64_t i = n - 1; i >= 0; --i) {
    double* xi = X + i * ldx;
    const double* bi = B + i * ldb;
    if (xi != bi)
      for (int64_t c = c0; c < c1; ++c) xi[c] = bi[c];
    for (int64_t j = i + 1; j < n; ++j) {
      const double lji = L[j * ldl + i];
      const double* xj = X + j * ldx;
      for (int64_t c = c0; c < c1; ++c) {
        double prod = lji * xj[c];
        xi[c] = xi[c] - prod;
      }
    }
    const double d = L[i * ldl + i];
    for (int64_t c = c0; c < c1; ++c) xi[c] = xi[c] / d;
  }
}

/* X = L^{-T} B by backward substitution: the transposed problem L^T X = B
 * (the second half of a solve with A = L L^T).  Reads only the lower triangle
 * of L.  X may be the same buffer as B (with ldx == ldb).  Returns 0, or -1
 * on bad sizes. */
int oracle_trsm_t_f64(int64_t n, int64_t k,
                      const double* L, int64_t ldl,
                      const double* B, int64_t ldb,
                      double* X, int64_t ldx, int nthreads) {
  if (n < 0 || k < 0) return -1;
  if (n == 0 || k == 0) return 0;
  if (ldl < n || ldb < k || ldx < k) return -1;
  const int64_t nchunks = (k + ORACLE_COLS - 1) / ORACLE_COLS;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    const int64_t c0 = ch * ORACLE_COLS;
    const int64_t c1 = min64(k, c0 + ORACLE_COLS);
    subst_t_cols_f64(n, c0, c1, L, ldl, B, ldb, X, ldx);
  }
  (void)nthreads;
  return 0;
}

/* Residual R = B - L X, summed plainly: r[i][c] = b[i][c] - sum_{j<=i}
 * l[i][j] x[j][c], j ascending, each product rounded then subtracted.
 * This is the postcondition B = L X of Alg. It-Inv-TRSM written as a defect. */
int oracle_residual_f64(int64_t n, int64_t k,
                        const double* L, int64_t ldl,
                        const double* X, int64_t ldx,
                        const double* B, int64_t ldb,
                        double* R, int64_t ldr, int nthreads) {
  if (n < 0 || k < 0) return -1;
  if (n == 0 || k == 0) return 0;
  if (ldl < n || ldb < k || ldx < k || ldr < k) return -1;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
  for (int64_t i = 0; i < n; ++i) {
    double* ri = R + i * ldr;
    const double* bi = B + i * ldb;
    const double* li = L + i * ldl;
    for (int64_t c = 0; c < k; ++c) ri[c] = bi[c];
    for (int64_t j = 0; j <= i; ++j) {
      const double lij = li[j];
      const double* xj = X + j * ldx;
      for (int64_t c = 0; c < k; ++c) {
        double prod = lij * xj[c];
        ri[c] = ri[c] - prod;
      }
    }
  }
  (void)nthreads;
  return 0;
}

/* The same forward substitution carried out in binary128 (__float128), with
 * inputs taken exactly from binary64 and the result rounded once to binary64.
 * Used to arbitrate accuracy questions on ill-conditioned inputs: its own
 * error is about cond(L) * 2^-113, far below any binary64 solve. */
int oracle_trsm_q(int64_t n, int64_t k,
                  const double* L, int64_t ldl,
                  const double* B, int64_t ldb,
                  double* X, int64_t ldx, int nthreads) {
  if (n < 0 || k < 0) return -1;
  if (n == 0 || k == 0) return 0;
  if (ldl < n || ldb < k || ldx < k) return -1;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
#endif
  for (int64_t c = 0; c < k; ++c) {
    __float128* x = (__float128*)malloc(sizeof(__float128) * (size_t)n);
    if (!x) continue;
    for (int64_t i = 0; i < n; ++i) {
      const double* li = L + i * ldl;
      __float128 s = (__float128)B[i * ldb + c];
      for (int64_t j = 0; j < i; ++j) s -= (__float128)li[j] * x[j];
      x[i] = s / (__float128)li[i];
    }
    for (int64_t i = 0; i < n; ++i) X[i * ldx + c] = (double)x[i];
    free(x);
  }
  (void)nthreads;
  return 0;
}

/* Frobenius norm of the lower triangle (diagonal included) of L, and of a
 * dense n x k matrix, accumulated in binary128 so that the norm itself is
 * correctly rounded to binary64 for all practical sizes. */
double oracle_fro_lower(int64_t n, const double* L, int64_t ldl) {
  __float128 s = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j <= i; ++j) {
      __float128 v = (__float128)L[i * ldl + j];
      s += v * v;
    }
  /* square root by Newton steps in binary128, seeded from binary64 */
  double s64 = (double)s;
  if (s64 <= 0) return 0.0;
  __float128 r = (__float128)__builtin_sqrt(s64);
  for (int it = 0; it < 3; ++it) r = 0.5Q * (r + s / r);
  return (double)r;
}

double oracle_fro_dense(int64_t n, int64_t k, const double* A, int64_t lda) {
  __float128 s = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t c = 0; c < k; ++c) {
      __float128 v = (__float128)A[i * lda + c];
      s += v * v;
    }
  double s64 = (double)s;
  if (s64 <= 0) return 0.0;
  __float128 r = (__float128)__builtin_sqrt(s64);
  for (int it = 0; it < 3; ++it) r = 0.5Q * (r + s / r);
  return (double)r;
}

/* Cholesky factor of a symmetric positive definite A: the lower-triangular L
 * with positive diagonal and A = L L^T.  The factorization whose panel step
 * is a triangular solve with many right-hand sides (the abstract and Sec. I
 * name Cholesky and LU as the factorizations TRSM serves).  The definition
 * written out column by column, j ascending:
 *
 *     l[j][j] = sqrt( a[j][j] - sum_{p<j} l[j][p]^2 )
 *     l[i][j] = ( a[i][j] - sum_{p<j} l[i][p] * l[j][p] ) / l[j][j],   i > j,
 *
 * each sum taken with p ascending, every product rounded before it is
 * subtracted, a correctly rounded square root and a true division.  Only the
 * lower triangle of A (diagonal included) is read; L is written to the lower
 * triangle of Lout with zeros above the diagonal.  Lout may be A itself
 * (ldl == lda).  Threads split the rows of each column: every element is
 * computed by the same operations whatever the thread count.
 *
 * Returns 0, or -1 on bad sizes.  *fail receives -1, or the first column j
 * whose pivot a[j][j] - sum l[j][p]^2 is not positive (or is NaN); the
 * factorization stops there and columns >= j of Lout are unspecified. */
int oracle_chol_f64(int64_t n, const double* A, int64_t lda,
                    double* Lout, int64_t ldl, int nthreads, int64_t* fail) {
  if (fail) *fail = -1;
  if (n < 0) return -1;
  if (n == 0) return 0;
  if (lda < n || ldl < n) return -1;
  /* copy the lower triangle first so that Lout == A works */
  for (int64_t i = 0; i < n; ++i) {
    double* li = Lout + i * ldl;
    const double* ai = A + i * lda;
    if (li != ai)
      for (int64_t j = 0; j <= i; ++j) li[j] = ai[j];
    for (int64_t j = i + 1; j < n; ++j) li[j] = 0.0;
  }
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#endif
  for (int64_t j = 0; j < n; ++j) {
    double* lj = Lout + j * ldl;
    double piv = lj[j];
    for (int64_t p = 0; p < j; ++p) {
      double prod = lj[p] * lj[p];
      piv = piv - prod;
    }
    if (!(piv > 0.0)) {
      if (fail) *fail = j;
      return 0;
    }
    const double d = sqrt(piv);
    lj[j] = d;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads) if (n - j > 256)
#endif
    for (int64_t i = j + 1; i < n; ++i) {
      double* li = Lout + i * ldl;
      double v = li[j];
      for (int64_t p = 0; p < j; ++p) {
        double prod = li[p] * lj[p];
        v = v - prod;
      }
      li[j] = v / d;
    }
  }
  (void)nthreads;
  return 0;
}

/* LU factors without pivoting, A = L U, L unit lower triangular and U upper
 * triangular: the other factorization the abstract and Sec. I name as built
 * on TRSM, in its no-exchange form (the matrices it is meant for need no row
 * exchanges, e.g. diagonally dominant ones).  Doolittle's definition written
 * out, step j ascending:
 *
 *     u[j][c] = a[j][c] - sum_{p<j} l[j][p] * u[p][c],          c >= j
 *     l[i][j] = ( a[i][j] - sum_{p<j} l[i][p] * u[p][j] ) / u[j][j],   i > j
 *
 * each sum taken with p ascending, every product rounded before it is
 * subtracted, a true division.  A is n x n row-major (lda); LU receives L
 * strictly below the diagonal (its unit diagonal is not stored) and U on and
 * above it, the compact form.  LU may be A itself (ldu == lda).  Threads
 * split the rows of each column of L and the columns of each row of U.
 *
 * Returns 0, or -1 on bad sizes.  *fail receives -1, or the first j whose
 * pivot u[j][j] is zero or not finite; LU is then unspecified from row and
 * column j on. */
int oracle_lu_nopiv_f64(int64_t n, const double* A, int64_t lda,
                        double* LU, int64_t ldu, int nthreads, int64_t* fail) {
  if (fail != NULL) *fail = -1;
  if (n < 0) return -1;
  if (n == 0) return 0;
  if (lda < n || ldu < n) return -1;
  for (int64_t i = 0; i < n; ++i) {
    double* ui = LU + i * ldu;
    const double* ai = A + i * lda;
    if (ui != ai)
      for (int64_t j = 0; j < n; ++j) ui[j] = ai[j];
  }
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#endif
  for (int64_t j = 0; j < n; ++j) {
    double* uj = LU + j * ldu;
    /* row j of U */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads) if (n - j > 256)
#endif
    for (int64_t c = j; c < n; ++c) {
      double acc = uj[c];
      for (int64_t p = 0; p < j; ++p) {
        double term = uj[p] * LU[p * ldu + c];
        acc = acc - term;
      }
      uj[c] = acc;
    }
    const double ujj = uj[j];
    if (!(ujj != 0.0) || !isfinite(ujj)) {
      if (fail != NULL) *fail = j;
      return 0;
    }
    /* column j of L */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads) if (n - j > 256)
#endif
    for (int64_t i = j + 1; i < n; ++i) {
      double* li = LU + i * ldu;
      double acc = li[j];
      for (int64_t p = 0; p < j; ++p) {
        double term = li[p] * LU[p * ldu + j];
        acc = acc - term;
      }
      li[j] = acc / ujj;
    }
  }
  (void)nthreads;
  return 0;
}

/* LU factorization with partial pivoting (row exchanges), P A = L U, L unit
 * lower triangular with |l_ij| <= 1, U upper triangular: the plain
 * right-looking elimination of Gaussian elimination with partial pivoting,
 * the unblocked form of LAPACK's dgetf2.  For j = 0, 1, ..., n - 1:
 *
 *   p = the first row i >= j with the largest |a[i][j]|   (ipiv[j] = p)
 *   exchange rows j and p of the whole working matrix (all n columns)
 *   if a[j][j] != 0:  l[i][j] = a[i][j] / a[j][j]                 (i > j)
 *                     a[i][c] = a[i][c] - l[i][j] * a[j][c]      (i, c > j)
 *
 * with IEEE binary64, a true division and no contraction.  The abstract and
 * Sec. I name LU as a factorization built on TRSM; the row exchanges are
 * what make it apply to every nonsingular matrix.  P A = L U with P the
 * product of the exchanges: applying "swap rows j and ipiv[j]" for j = 0 ..
 * n - 1 to A gives L U.
 *
 * LU receives L strictly below the diagonal (its unit diagonal is not
 * stored) and U on and above it (row-major, ld ldu; it may equal A with lda
 * == ldu); ipiv[j] the row exchanged with row j (0-based, ipiv[j] >= j).
 * Threads split the rows of each update; every element sees the same
 * operations in the same order whatever the thread count.  Returns 0, or -1
 * on bad sizes.  *fail receives -1, or the first j whose pivot is zero (or
 * not finite); that column is then left unscaled and the elimination goes on
 * (as LAPACK does with its INFO). */
int oracle_lu_piv_f64(int64_t n, const double* A, int64_t lda, double* LU, int64_t ldu,
                      int nthreads, int64_t* ipiv, int64_t* fail) {
  if (fail != NULL) *fail = -1;
  if (n < 0) return -1;
  if (n == 0) return 0;
  if (lda < n || ldu < n || ipiv == NULL) return -1;
  for (int64_t i = 0; i < n; ++i) {
    double* ui = LU + i * ldu;
    const double* ai = A + i * lda;
    if (ui != ai)
      for (int64_t j = 0; j < n; ++j) ui[j] = ai[j];
  }
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#endif
  for (int64_t j = 0; j < n; ++j) {
    /* the pivot: first largest magnitude in column j, rows j .. n-1 */
    int64_t p = j;
    double best = fabs(LU[j * ldu + j]);
    for (int64_t i = j + 1; i < n; ++i) {
      const double v = fabs(LU[i * ldu + j]);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    ipiv[j] = p;
    if (p != j) {
      double* rj = LU + j * ldu;
      double* rp = LU + p * ldu;
      for (int64_t c = 0; c < n; ++c) {
        const double t = rj[c];
        rj[c] = rp[c];
        rp[c] = t;
      }
    }
    const double piv = LU[j * ldu + j];
    if (!(piv != 0.0) || !isfinite(piv)) {
      if (fail != NULL && *fail < 0) *fail = j;
      continue;
    }
    const double* uj = LU + j * ldu;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads) if (n - j > 128)
#endif
    for (int64_t i = j + 1; i < n; ++i) {
      double* ri = LU + i * ldu;
      const double l = ri[j] / piv;
      ri[j] = l;
      for (int64_t c = j + 1; c < n; ++c) {
        const double term = l * uj[c];
        ri[c] = ri[c] - term;
      }
    }
  }
  (void)nthreads;
  return 0;
}

/* Number of threads the OpenMP runtime would use by default. */
int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

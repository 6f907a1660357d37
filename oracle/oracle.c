/*
 * CPU oracle for the dense LU solve path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library.  The GPU path never calls, links or includes it, and the
 * two share no code.
 *
 * What it computes (paper, section "High Performance Linpack"): the solution of
 * A x = b by first decomposing A into a lower and an upper factor, then solving
 * L y = b and U x = y.  The paper's own FPGA design skips pivoting because its
 * inputs are diagonally dominant (the HPL-AI rule); this oracle implements the
 * textbook method with partial pivoting (Gaussian elimination with row
 * interchanges, LAPACK getf2 semantics), which reduces to the paper's
 * no-pivot elimination whenever the pivot search keeps the diagonal row.  The
 * paper's blocked right-looking scheme ("Base Implementation", figure
 * fig:lu_iteration) is the same elimination with the updates grouped in
 * blocks; with block size one it is exactly the loop below.
 *
 * Conventions (shared with the GPU path only through their documentation):
 *   - matrices are row-major: element (i, j) at A[i * lda + j];
 *   - ipiv is 0-based with sequential-swap meaning: at step k, row k was
 *     exchanged with row ipiv[k] >= k;
 *   - pivot choice: the smallest row index i >= k whose |a_ik| is maximal, found
 *     by a left-to-right scan with a strict '>' (a NaN never replaces the
 *     current candidate; a NaN on the diagonal stays the pivot);
 *   - an exact zero pivot sets info = k + 1 (first one only) and the step is
 *     skipped (no scaling, no update), as LAPACK does;
 *   - scaling divides (correctly rounded IEEE division), the update is a
 *     separate multiply and subtract (the file is compiled with
 *     -ffp-contract=off and without fast-math);
 *   - sums run left to right.
 *
 * Residual check: the benchmark's scaled residual
 *     s = ||A x - b||_inf / (eps * (||A||_inf * ||x||_inf + ||b||_inf) * n),
 * with eps = 2^-53, evaluated per right-hand side on the original A and b.
 * The paper prints a garbled normalised-residual formula; the reading used here
 * is the standard HPL scaled residual above (pass if s < 16).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EPS 0x1.0p-53

int orc_version(void) { return 1; }

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/* Unblocked Gaussian elimination with partial pivoting on an m x n row-major
 * matrix (factors overwrite A: unit lower L below the diagonal, U on and above).
 * ipiv receives min(m, n) entries.  Returns 0, or -i for an illegal i-th
 * argument. */
int orc_getrf(int m, int n, double *A, int lda, int *ipiv, int *info) {
  if (m < 0) return -1;
  if (n < 0) return -2;
  if (lda < (n > 1 ? n : 1)) return -4;
  *info = 0;
  const int kmax = m < n ? m : n;
  for (int k = 0; k < kmax; ++k) {
    /* pivot search: strict '>' scan from the diagonal row downwards */
    int p = k;
    double best = fabs(A[(size_t)k * lda + k]);
    for (int i = k + 1; i < m; ++i) {
      double v = fabs(A[(size_t)i * lda + k]);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    ipiv[k] = p;
    if (A[(size_t)p * lda + k] == 0.0) {
      if (*info == 0) *info = k + 1;
      continue;
    }
    /* interchange whole rows k and p */
    if (p != k) {
      double *rk = A + (size_t)k * lda, *rp = A + (size_t)p * lda;
      for (int j = 0; j < n; ++j) {
        double t = rk[j];
        rk[j] = rp[j];
        rp[j] = t;
      }
    }
    const double piv = A[(size_t)k * lda + k];
    const double *uk = A + (size_t)k * lda;
    /* scale the column below the pivot, then the rank-1 update of the rest */
#pragma omp parallel for schedule(static) if (m - k > 512)
    for (int i = k + 1; i < m; ++i) {
      double *ri = A + (size_t)i * lda;
      const double l = ri[k] / piv;
      ri[k] = l;
      for (int j = k + 1; j < n; ++j) {
        const double prod = l * uk[j];
        ri[j] = ri[j] - prod;
      }
    }
  }
  return 0;
}

/* The paper's own elimination: no row interchanges (valid for diagonally
 * dominant A, the HPL-AI rule).  info as above. */
int orc_getrf_nopiv(int m, int n, double *A, int lda, int *info) {
  if (m < 0) return -1;
  if (n < 0) return -2;
  if (lda < (n > 1 ? n : 1)) return -4;
  *info = 0;
  const int kmax = m < n ? m : n;
  for (int k = 0; k < kmax; ++k) {
    const double piv = A[(size_t)k * lda + k];
    if (piv == 0.0) {
      if (*info == 0) *info = k + 1;
      continue;
    }
    const double *uk = A + (size_t)k * lda;
#pragma omp parallel for schedule(static) if (m - k > 512)
    for (int i = k + 1; i < m; ++i) {
      double *ri = A + (size_t)i * lda;
      const double l = ri[k] / piv;
      ri[k] = l;
      for (int j = k + 1; j < n; ++j) {
        const double prod = l * uk[j];
        ri[j] = ri[j] - prod;
      }
    }
  }
  return 0;
}

/* Solve with the factors of orc_getrf: B := P^-1-applied solve, i.e. apply the
 * interchanges to B, then L y = P b (unit lower), then U x = y.  B is n x nrhs
 * row-major.  ipiv == NULL means no interchanges.  Returns 0, -i for an
 * illegal argument, or 1 if U has an exact zero on its diagonal (B untouched). */
int orc_getrs(int n, const double *LU, int lda, const int *ipiv, double *B, int ldb,
              int nrhs) {
  if (n < 0) return -1;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (ldb < (nrhs > 1 ? nrhs : 1)) return -6;
  if (nrhs < 0) return -7;
  for (int i = 0; i < n; ++i)
    if (LU[(size_t)i * lda + i] == 0.0) return 1;
  if (ipiv) {
    for (int k = 0; k < n; ++k) {
      int p = ipiv[k];
      if (p != k) {
        for (int c = 0; c < nrhs; ++c) {
          double t = B[(size_t)k * ldb + c];
          B[(size_t)k * ldb + c] = B[(size_t)p * ldb + c];
          B[(size_t)p * ldb + c] = t;
        }
      }
    }
  }
  for (int c = 0; c < nrhs; ++c) {
    /* forward substitution, unit diagonal */
    for (int i = 0; i < n; ++i) {
      double s = B[(size_t)i * ldb + c];
      const double *li = LU + (size_t)i * lda;
      for (int j = 0; j < i; ++j) {
        const double prod = li[j] * B[(size_t)j * ldb + c];
        s = s - prod;
      }
      B[(size_t)i * ldb + c] = s;
    }
    /* back substitution */
    for (int i = n - 1; i >= 0; --i) {
      double s = B[(size_t)i * ldb + c];
      const double *ui = LU + (size_t)i * lda;
      for (int j = i + 1; j < n; ++j) {
        const double prod = ui[j] * B[(size_t)j * ldb + c];
        s = s - prod;
      }
      B[(size_t)i * ldb + c] = s / ui[i];
    }
  }
  return 0;
}

/* Solve A^T X = B with the factors of orc_getrf (P A = L U, so
 * A^T = U^T L^T P): U^T z = b by forward substitution (U^T is lower, with
 * the u_ii on its diagonal), L^T w = z by back substitution (unit upper),
 * then x = P^T w, i.e. the recorded interchanges undone in reverse order.
 * Used by the condition estimator, which needs products with A^-T.  Same
 * arguments and return values as orc_getrs. */
int orc_getrs_trans(int n, const double *LU, int lda, const int *ipiv, double *B, int ldb,
                    int nrhs) {
  if (n < 0) return -1;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (ldb < (nrhs > 1 ? nrhs : 1)) return -6;
  if (nrhs < 0) return -7;
  for (int i = 0; i < n; ++i)
    if (LU[(size_t)i * lda + i] == 0.0) return 1;
  for (int c = 0; c < nrhs; ++c) {
    /* U^T z = b: z_i = (b_i - sum_{j<i} u_ji z_j) / u_ii */
    for (int i = 0; i < n; ++i) {
      double s = B[(size_t)i * ldb + c];
      for (int j = 0; j < i; ++j) {
        const double prod = LU[(size_t)j * lda + i] * B[(size_t)j * ldb + c];
        s = s - prod;
      }
      B[(size_t)i * ldb + c] = s / LU[(size_t)i * lda + i];
    }
    /* L^T w = z: w_i = z_i - sum_{j>i} l_ji w_j */
    for (int i = n - 1; i >= 0; --i) {
      double s = B[(size_t)i * ldb + c];
      for (int j = i + 1; j < n; ++j) {
        const double prod = LU[(size_t)j * lda + i] * B[(size_t)j * ldb + c];
        s = s - prod;
      }
      B[(size_t)i * ldb + c] = s;
    }
  }
  if (ipiv) {
    for (int k = n - 1; k >= 0; --k) {
      int p = ipiv[k];
      if (p != k) {
        for (int c = 0; c < nrhs; ++c) {
          double t = B[(size_t)k * ldb + c];
          B[(size_t)k * ldb + c] = B[(size_t)p * ldb + c];
          B[(size_t)p * ldb + c] = t;
        }
      }
    }
  }
  return 0;
}

/* The PTRANS operation (paper, section "Parallel Matrix Transposition"):
 * C = B + A^T for n x n row-major matrices, element by element,
 * c_ij = b_ij + a_ji (one rounded addition each). */
void orc_ptrans(int n, const double *A, int lda, const double *B, int ldb, double *C, int ldc) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C[(size_t)i * ldc + j] = B[(size_t)i * ldb + j] + A[(size_t)j * lda + i];
}

/* The same in binary32. */
void orc_ptrans_f32(int n, const float *A, int lda, const float *B, int ldb, float *C, int ldc) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C[(size_t)i * ldc + j] = B[(size_t)i * ldb + j] + A[(size_t)j * lda + i];
}

/* Scaled residual per right-hand side, binary64 with left-to-right sums.
 * out[5*c + 0..4] = { s, ||r||_inf, ||A||_inf, ||x_c||_inf, ||b_c||_inf } with
 * r = A x - b.  A NaN anywhere propagates into s (and s < 16 is then false). */
void orc_residual(int n, const double *A, int lda, const double *X, int ldx,
                  const double *B, int ldb, int nrhs, double *out) {
  double anorm = 0.0;
  for (int i = 0; i < n; ++i) {
    double rs = 0.0;
    for (int j = 0; j < n; ++j) rs = rs + fabs(A[(size_t)i * lda + j]);
    if (rs > anorm || isnan(rs)) anorm = rs;
  }
  for (int c = 0; c < nrhs; ++c) {
    double rn = 0.0, xn = 0.0, bn = 0.0;
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) {
        const double prod = A[(size_t)i * lda + j] * X[(size_t)j * ldx + c];
        s = s + prod;
      }
      const double r = fabs(s - B[(size_t)i * ldb + c]);
      if (r > rn || isnan(r)) rn = r;
      const double xa = fabs(X[(size_t)i * ldx + c]);
      if (xa > xn || isnan(xa)) xn = xa;
      const double ba = fabs(B[(size_t)i * ldb + c]);
      if (ba > bn || isnan(ba)) bn = ba;
    }
    const double denom = ORC_EPS * (anorm * xn + bn) * (double)n;
    out[5 * c + 0] = rn / denom;
    out[5 * c + 1] = rn;
    out[5 * c + 2] = anorm;
    out[5 * c + 3] = xn;
    out[5 * c + 4] = bn;
  }
}

/* The same residual with long double (x87 extended) accumulation, used to
 * check the binary64 check. */
void orc_residual_ld(int n, const double *A, int lda, const double *X, int ldx,
                     const double *B, int ldb, int nrhs, double *out) {
  long double anorm = 0.0L;
  for (int i = 0; i < n; ++i) {
    long double rs = 0.0L;
    for (int j = 0; j < n; ++j) rs += fabsl((long double)A[(size_t)i * lda + j]);
    if (rs > anorm || isnan((double)rs)) anorm = rs;
  }
  for (int c = 0; c < nrhs; ++c) {
    long double rn = 0.0L, xn = 0.0L, bn = 0.0L;
    for (int i = 0; i < n; ++i) {
      long double s = 0.0L;
      for (int j = 0; j < n; ++j)
        s += (long double)A[(size_t)i * lda + j] * (long double)X[(size_t)j * ldx + c];
      const long double r = fabsl(s - (long double)B[(size_t)i * ldb + c]);
      if (r > rn || isnan((double)r)) rn = r;
      const long double xa = fabsl((long double)X[(size_t)i * ldx + c]);
      if (xa > xn) xn = xa;
      const long double ba = fabsl((long double)B[(size_t)i * ldb + c]);
      if (ba > bn) bn = ba;
    }
    const long double denom = (long double)ORC_EPS * (anorm * xn + bn) * (long double)n;
    out[5 * c + 0] = (double)(rn / denom);
    out[5 * c + 1] = (double)rn;
    out[5 * c + 2] = (double)anorm;
    out[5 * c + 3] = (double)xn;
    out[5 * c + 4] = (double)bn;
  }
}

/* Residual of selected rows only: r_i = sum_j a_ij x_j - b_i (left to right)
 * and sum_j |a_ij| |x_j| (for error bounds), for the `cnt` rows given by the
 * caller as dense rows `Arows` (cnt x n) with their b entries. */
void orc_row_residuals(int n, int cnt, const double *Arows, int lda, const double *X,
                       int ldx, const double *Brows, int ldb, int nrhs, double *r_out,
                       double *absdot_out) {
  for (int t = 0; t < cnt; ++t) {
    for (int c = 0; c < nrhs; ++c) {
      double s = 0.0, a = 0.0;
      for (int j = 0; j < n; ++j) {
        const double prod = Arows[(size_t)t * lda + j] * X[(size_t)j * ldx + c];
        s = s + prod;
        a = a + fabs(prod);
      }
      r_out[(size_t)t * nrhs + c] = s - Brows[(size_t)t * ldb + c];
      absdot_out[(size_t)t * nrhs + c] = a;
    }
  }
}

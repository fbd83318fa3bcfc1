/*
 * CPU oracle for the three small dense solvers of "Program Generation for
 * Linear Algebra Using Multiple Layers of DSLs" (Spampinato, Fabregat-Traver,
 * Pueschel, Bientinesi), Fig. 2 caption:
 *   (a) upper Cholesky            X^T X = A   (A SPD, X upper triangular)
 *   (b) triangular Lyapunov       L X + X L^T = S   (L lower, S and X symmetric)
 *   (c) triangular Sylvester      L X + X U = C     (L lower, U upper)
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU baseline leg of
 * the benchmark do.  It shares no code, header or constant with the HIP path.
 *
 * Every routine is the plain textbook definition, written as an element
 * recurrence in FP64 with no blocking, fusion or reordering.  The paper states
 * that all of its generated algorithm variants are mathematically equivalent
 * (Generator structure paragraph), so each variant must reproduce these
 * results up to rounding.  Build with -O2 -ffp-contract=off (no FMA
 * contraction, no fast-math) so rounding follows the source order.
 *
 * Storage convention (the paper is silent): column-major, leading dimension
 * ld >= n, element (i,j) at p[i + j*ld].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define E(p, ld, i, j) ((p)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

/*
 * Upper Cholesky X^T X = A (Fig. 2a).  Reads only the upper triangle of A.
 * Writes the full n x n X (zeros below the diagonal).  The diagonal of X is
 * taken positive, which makes X unique.
 *   x_ij = (a_ij - sum_{k<i} x_ki x_kj) / x_ii      (i < j)
 *   x_jj = sqrt(a_jj - sum_{k<j} x_kj^2)
 * Returns 0, or k > 0 when the leading minor of order k is not positive
 * definite (the pivot is <= 0 or NaN); X is then only partly written.
 */
int orc_potrf(int n, const double *A, int lda, double *X, int ldx) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) E(X, ldx, i, j) = 0.0;
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i <= j; ++i) {
      double s = E(A, lda, i, j);
      for (int k = 0; k < i; ++k) s -= E(X, ldx, k, i) * E(X, ldx, k, j);
      if (i < j) {
        E(X, ldx, i, j) = s / E(X, ldx, i, i);
      } else {
        if (!(s > 0.0)) return j + 1;
        E(X, ldx, j, j) = sqrt(s);
      }
    }
  }
  return 0;
}

/*
 * Solve with the upper Cholesky factor: the consumer of Fig. 2a that the
 * paper's motivation names next to the factorizations (LAPACK solvers).
 * Given X upper triangular with X^T X = A, overwrite the n x m right-hand
 * sides B with A^{-1} B: forward substitution with X^T, then back
 * substitution with X, column by column:
 *   z_ij = (b_ij - sum_{k<i} x_ki z_kj) / x_ii         (i = 0 .. n-1)
 *   y_ij = (z_ij - sum_{k>i} x_ik y_kj) / x_ii         (i = n-1 .. 0)
 * Reads only the upper triangle of X.  Returns 0, or k > 0 when x_kk
 * (1-based) is zero; B is then left unchanged.
 */
int orc_potrs(int n, int m, const double *X, int ldx, double *B, int ldb) {
  for (int k = 0; k < n; ++k)
    if (E(X, ldx, k, k) == 0.0) return k + 1;
  for (int j = 0; j < m; ++j) {
    for (int i = 0; i < n; ++i) {
      double s = E(B, ldb, i, j);
      for (int k = 0; k < i; ++k) s -= E(X, ldx, k, i) * E(B, ldb, k, j);
      E(B, ldb, i, j) = s / E(X, ldx, i, i);
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = E(B, ldb, i, j);
      for (int k = i + 1; k < n; ++k) s -= E(X, ldx, i, k) * E(B, ldb, k, j);
      E(B, ldb, i, j) = s / E(X, ldx, i, i);
    }
  }
  return 0;
}

/*
 * Inverse from the upper Cholesky factor: A^{-1} = (X^T X)^{-1}, the full n x n
 * matrix, obtained by solving with the factor for the columns of the
 * identity (orc_potrs above).  Returns 0, or k > 0 when x_kk (1-based) is
 * zero; Y is then the identity.
 */
int orc_potri(int n, const double *X, int ldx, double *Y, int ldy) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) E(Y, ldy, i, j) = i == j ? 1.0 : 0.0;
  return orc_potrs(n, n, X, ldx, Y, ldy);
}

/*
 * Triangular Sylvester L X + X U = C (Fig. 2c).  Reads the lower triangle of
 * L and the upper triangle of U.  Column by column, top to bottom:
 *   x_ij = (c_ij - sum_{k<i} l_ik x_kj - sum_{k<j} x_ik u_kj) / (l_ii + u_jj)
 * Returns 0, or 1 + (i + j*n) of the first zero denominator l_ii + u_jj in
 * column-major order (X is then only partly written).
 */
int orc_trsyl(int n, const double *L, int ldl, const double *U, int ldu,
              const double *C, int ldc, double *X, int ldx) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) E(X, ldx, i, j) = 0.0;
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) {
      double d = E(L, ldl, i, i) + E(U, ldu, j, j);
      if (d == 0.0) return 1 + i + j * n;
      double s = E(C, ldc, i, j);
      for (int k = 0; k < i; ++k) s -= E(L, ldl, i, k) * E(X, ldx, k, j);
      for (int k = 0; k < j; ++k) s -= E(X, ldx, i, k) * E(U, ldu, k, j);
      E(X, ldx, i, j) = s / d;
    }
  }
  return 0;
}

/*
 * Triangular Lyapunov L X + X L^T = S (Fig. 2b), taken literally as printed:
 * no sign change, S on the right-hand side.  Reads the lower triangle of L
 * and of S; computes the lower triangle of X column by column and mirrors it,
 * so the returned X is exactly symmetric.  For i >= j:
 *   x_ij = (s_ij - sum_{k<i} l_ik x_kj - sum_{k<j} x_ik l_jk) / (l_ii + l_jj)
 * where x_kj with k < j is read as its mirror x_jk.
 * Returns 0, or 1 + (i + j*n) of the first zero denominator l_ii + l_jj in
 * column-major order of the full matrix (which always lies in the lower
 * triangle, since the denominators are symmetric in i and j).
 */
int orc_trlyap(int n, const double *L, int ldl, const double *S, int lds,
               double *X, int ldx) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) E(X, ldx, i, j) = 0.0;
  for (int j = 0; j < n; ++j) {
    for (int i = j; i < n; ++i) {
      double d = E(L, ldl, i, i) + E(L, ldl, j, j);
      if (d == 0.0) return 1 + i + j * n;
      double s = E(S, lds, i, j);
      for (int k = 0; k < i; ++k) {
        double xkj = (k >= j) ? E(X, ldx, k, j) : E(X, ldx, j, k);
        s -= E(L, ldl, i, k) * xkj;
      }
      for (int k = 0; k < j; ++k) s -= E(X, ldx, i, k) * E(L, ldl, j, k);
      E(X, ldx, i, j) = s / d;
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) E(X, ldx, j, i) = E(X, ldx, i, j);
  return 0;
}

/*
 * Dense Gaussian elimination with partial pivoting on an m x m column-major
 * system M y = r (overwrites M and r; r becomes y).  Returns 0, or 1 when a
 * pivot is exactly zero.  Used only for the brute-force Kronecker solves.
 */
int orc_gepp(int m, double *M, double *r) {
  for (int k = 0; k < m; ++k) {
    int p = k;
    double best = fabs(E(M, m, k, k));
    for (int i = k + 1; i < m; ++i)
      if (fabs(E(M, m, i, k)) > best) { best = fabs(E(M, m, i, k)); p = i; }
    if (best == 0.0) return 1;
    if (p != k) {
      for (int j = 0; j < m; ++j) {
        double t = E(M, m, k, j); E(M, m, k, j) = E(M, m, p, j); E(M, m, p, j) = t;
      }
      double t = r[k]; r[k] = r[p]; r[p] = t;
    }
    /* multipliers l_ik = m_ik / m_kk, kept in column k until it is cleared;
     * then every entry m_ij (i, j > k) receives its one update of step k,
     * walked down the columns (storage order) */
    for (int i = k + 1; i < m; ++i) E(M, m, i, k) /= E(M, m, k, k);
    for (int j = k + 1; j < m; ++j) {
      const double mkj = E(M, m, k, j);
      for (int i = k + 1; i < m; ++i) E(M, m, i, j) -= E(M, m, i, k) * mkj;
    }
    for (int i = k + 1; i < m; ++i) {
      r[i] -= E(M, m, i, k) * r[k];
      E(M, m, i, k) = 0.0;
    }
  }
  for (int k = m - 1; k >= 0; --k) {
    double s = r[k];
    for (int j = k + 1; j < m; ++j) s -= E(M, m, k, j) * r[j];
    r[k] = s / E(M, m, k, k);
  }
  return 0;
}

/*
 * Brute-force Sylvester solve through the Kronecker form of L X + X U = C
 * with column-major vec:  (I (x) L + U^T (x) I) vec X = vec C.
 * tri != 0 uses only the referenced triangles of L (lower) and U (upper).
 * W must hold n^4 + n^2 doubles.  Returns the GEPP status.
 */
int orc_kron_sylv(int n, const double *L, int ldl, const double *U, int ldu,
                  const double *C, int ldc, double *X, int ldx, double *W) {
  int m = n * n;
  double *M = W, *r = W + (size_t)m * m;
  memset(M, 0, sizeof(double) * (size_t)m * m);
  /* row index (i + j n) of vec X, column index (p + q n) */
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      int row = i + j * n;
      for (int p = 0; p <= i; ++p) E(M, m, row, p + j * n) += E(L, ldl, i, p);  /* (I (x) L) */
      for (int q = 0; q <= j; ++q) E(M, m, row, i + q * n) += E(U, ldu, q, j);  /* (U^T (x) I) */
      r[row] = E(C, ldc, i, j);
    }
  int st = orc_gepp(m, M, r);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) E(X, ldx, i, j) = r[i + j * n];
  return st;
}

/* Brute-force Lyapunov solve: (I (x) L + L (x) I) vec X = vec S, with S given
 * by its lower triangle (mirrored).  W holds n^4 + n^2 doubles. */
int orc_kron_lyap(int n, const double *L, int ldl, const double *S, int lds,
                  double *X, int ldx, double *W) {
  int m = n * n;
  double *M = W, *r = W + (size_t)m * m;
  memset(M, 0, sizeof(double) * (size_t)m * m);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      int row = i + j * n;
      for (int p = 0; p <= i; ++p) E(M, m, row, p + j * n) += E(L, ldl, i, p);  /* L X   */
      for (int q = 0; q <= j; ++q) E(M, m, row, i + q * n) += E(L, ldl, j, q);  /* X L^T */
      r[row] = (i >= j) ? E(S, lds, i, j) : E(S, lds, j, i);
    }
  int st = orc_gepp(m, M, r);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) E(X, ldx, i, j) = r[i + j * n];
  return st;
}

/*
 * General (non-triangular) Sylvester A X + X B = C and Lyapunov
 * A X + X A^T = S: the equations of Fig. 2 before any reduction to triangular
 * form, which the Bartels-Stewart method brings them to (the paper treats only
 * the triangular cores).  The oracle is the plain definition, the Kronecker
 * system with column-major vec, solved by the dense elimination above:
 *   Sylvester: (I (x) A + B^T (x) I) vec X = vec C
 *   Lyapunov : (I (x) A + A (x) I) vec X = vec S   (S given by its lower triangle)
 * A and B are read in full.  W must hold n^4 + n^2 doubles.  Returns the GEPP
 * status (1: the operator is singular to working precision at a pivot).
 */
int orc_kron_gesyl(int n, const double *A, int lda, const double *B, int ldb,
                   const double *C, int ldc, double *X, int ldx, double *W) {
  int m = n * n;
  double *M = W, *r = W + (size_t)m * m;
  memset(M, 0, sizeof(double) * (size_t)m * m);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      int row = i + j * n;
      for (int p = 0; p < n; ++p) E(M, m, row, p + j * n) += E(A, lda, i, p);  /* (I (x) A)   */
      for (int q = 0; q < n; ++q) E(M, m, row, i + q * n) += E(B, ldb, q, j);  /* (B^T (x) I) */
      r[row] = E(C, ldc, i, j);
    }
  int st = orc_gepp(m, M, r);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) E(X, ldx, i, j) = r[i + j * n];
  return st;
}

int orc_kron_gelyap(int n, const double *A, int lda, const double *S, int lds,
                    double *X, int ldx, double *W) {
  int m = n * n;
  double *M = W, *r = W + (size_t)m * m;
  memset(M, 0, sizeof(double) * (size_t)m * m);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      int row = i + j * n;
      for (int p = 0; p < n; ++p) E(M, m, row, p + j * n) += E(A, lda, i, p);  /* A X   */
      for (int q = 0; q < n; ++q) E(M, m, row, i + q * n) += E(A, lda, j, q);  /* X A^T */
      r[row] = (i >= j) ? E(S, lds, i, j) : E(S, lds, j, i);
    }
  int st = orc_gepp(m, M, r);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) E(X, ldx, i, j) = r[i + j * n];
  return st;
}

/* ---- backward and forward error measures (all FP64, Frobenius norms) ---- */

/* General Sylvester: ||C - A X - X B||_F / ((||A||_F + ||B||_F) ||X||_F + ||C||_F),
 * A and B in full. */
double orc_eta_gesyl(int n, const double *A, int lda, const double *B, int ldb,
                     const double *C, int ldc, const double *X, int ldx) {
  double num = 0.0, na = 0.0, nb = 0.0, nx = 0.0, nc = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      double s = E(C, ldc, i, j);
      for (int k = 0; k < n; ++k) s -= E(A, lda, i, k) * E(X, ldx, k, j);
      for (int k = 0; k < n; ++k) s -= E(X, ldx, i, k) * E(B, ldb, k, j);
      num += s * s;
      na += E(A, lda, i, j) * E(A, lda, i, j);
      nb += E(B, ldb, i, j) * E(B, ldb, i, j);
      nx += E(X, ldx, i, j) * E(X, ldx, i, j);
      nc += E(C, ldc, i, j) * E(C, ldc, i, j);
    }
  return sqrt(num) / ((sqrt(na) + sqrt(nb)) * sqrt(nx) + sqrt(nc));
}

/* General Lyapunov: ||S - A X - X A^T||_F / (2 ||A||_F ||X||_F + ||S||_F),
 * A in full, S given by its lower triangle, X full. */
double orc_eta_gelyap(int n, const double *A, int lda, const double *S, int lds,
                      const double *X, int ldx) {
  double num = 0.0, na = 0.0, nx = 0.0, ns = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      double sv = (i >= j) ? E(S, lds, i, j) : E(S, lds, j, i);
      double s = sv;
      for (int k = 0; k < n; ++k) s -= E(A, lda, i, k) * E(X, ldx, k, j);
      for (int k = 0; k < n; ++k) s -= E(X, ldx, i, k) * E(A, lda, j, k);
      num += s * s;
      na += E(A, lda, i, j) * E(A, lda, i, j);
      nx += E(X, ldx, i, j) * E(X, ldx, i, j);
      ns += sv * sv;
    }
  return sqrt(num) / (2.0 * sqrt(na) * sqrt(nx) + sqrt(ns));
}


/* ||A - X^T X||_F / ||A||_F using the upper triangle of X and the full
 * symmetric A reconstructed from its upper triangle. */
double orc_eta_potrf(int n, const double *A, int lda, const double *X, int ldx) {
  double num = 0.0, den = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      int r = i < j ? i : j, c = i < j ? j : i;
      double a = E(A, lda, r, c);
      double s = 0.0;
      int kmax = (i < j ? i : j);
      for (int k = 0; k <= kmax; ++k) s += E(X, ldx, k, i) * E(X, ldx, k, j);
      num += (a - s) * (a - s);
      den += a * a;
    }
  return sqrt(num) / sqrt(den);
}

/* ||C - L X - X U||_F / ((||L||_F + ||U||_F) ||X||_F + ||C||_F) over the
 * referenced triangles of L and U. */
double orc_eta_trsyl(int n, const double *L, int ldl, const double *U, int ldu,
                     const double *C, int ldc, const double *X, int ldx) {
  double num = 0.0, nl = 0.0, nu = 0.0, nx = 0.0, nc = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      double s = E(C, ldc, i, j);
      for (int k = 0; k <= i; ++k) s -= E(L, ldl, i, k) * E(X, ldx, k, j);
      for (int k = 0; k <= j; ++k) s -= E(X, ldx, i, k) * E(U, ldu, k, j);
      num += s * s;
      if (i >= j) nl += E(L, ldl, i, j) * E(L, ldl, i, j);
      if (i <= j) nu += E(U, ldu, i, j) * E(U, ldu, i, j);
      nx += E(X, ldx, i, j) * E(X, ldx, i, j);
      nc += E(C, ldc, i, j) * E(C, ldc, i, j);
    }
  return sqrt(num) / ((sqrt(nl) + sqrt(nu)) * sqrt(nx) + sqrt(nc));
}

/* ||S - L X - X L^T||_F / (2 ||L||_F ||X||_F + ||S||_F), with S and L given by
 * their lower triangles and X full. */
double orc_eta_trlyap(int n, const double *L, int ldl, const double *S, int lds,
                      const double *X, int ldx) {
  double num = 0.0, nl = 0.0, nx = 0.0, ns = 0.0;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      double sv = (i >= j) ? E(S, lds, i, j) : E(S, lds, j, i);
      double s = sv;
      for (int k = 0; k <= i; ++k) s -= E(L, ldl, i, k) * E(X, ldx, k, j);
      for (int k = 0; k <= j; ++k) s -= E(X, ldx, i, k) * E(L, ldl, j, k);
      num += s * s;
      if (i >= j) nl += E(L, ldl, i, j) * E(L, ldl, i, j);
      nx += E(X, ldx, i, j) * E(X, ldx, i, j);
      ns += sv * sv;
    }
  return sqrt(num) / (2.0 * sqrt(nl) * sqrt(nx) + sqrt(ns));
}

/* ---- batched drivers over contiguous [batch, ld, n] column-major stacks ---- */

static void set_threads(int threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_potrf_batch(int batch, int n, const double *A, double *X, int *info, int threads) {
  set_threads(threads);
  size_t st = (size_t)n * n;
#pragma omp parallel for schedule(dynamic, 4)
  for (int b = 0; b < batch; ++b) info[b] = orc_potrf(n, A + b * st, n, X + b * st, n);
}

void orc_trsyl_batch(int batch, int n, const double *L, const double *U, const double *C,
                     double *X, int *info, int threads) {
  set_threads(threads);
  size_t st = (size_t)n * n;
#pragma omp parallel for schedule(dynamic, 4)
  for (int b = 0; b < batch; ++b)
    info[b] = orc_trsyl(n, L + b * st, n, U + b * st, n, C + b * st, n, X + b * st, n);
}

void orc_trlyap_batch(int batch, int n, const double *L, const double *S, double *X,
                      int *info, int threads) {
  set_threads(threads);
  size_t st = (size_t)n * n;
#pragma omp parallel for schedule(dynamic, 4)
  for (int b = 0; b < batch; ++b)
    info[b] = orc_trlyap(n, L + b * st, n, S + b * st, n, X + b * st, n);
}

void orc_potrs_batch(int batch, int n, int m, const double *X, double *B, int *info, int threads) {
  set_threads(threads);
  size_t sx = (size_t)n * n, sb = (size_t)n * m;
#pragma omp parallel for schedule(dynamic, 4)
  for (int b = 0; b < batch; ++b) info[b] = orc_potrs(n, m, X + b * sx, n, B + b * sb, n);
}

void orc_potri_batch(int batch, int n, const double *X, double *Y, int *info, int threads) {
  set_threads(threads);
  size_t st = (size_t)n * n;
#pragma omp parallel for schedule(dynamic, 4)
  for (int b = 0; b < batch; ++b) info[b] = orc_potri(n, X + b * st, n, Y + b * st, n);
}

void orc_eta_potrf_batch(int batch, int n, const double *A, const double *X, double *eta, int threads) {
  set_threads(threads);
  size_t st = (size_t)n * n;
#pragma omp parallel for schedule(dynamic, 4)
  for (int b = 0; b < batch; ++b) eta[b] = orc_eta_potrf(n, A + b * st, n, X + b * st, n);
}

void orc_eta_trsyl_batch(int batch, int n, const double *L, const double *U, const double *C,
                         const double *X, double *eta, int threads) {
  set_threads(threads);
  size_t st = (size_t)n * n;
#pragma omp parallel for schedule(dynamic, 4)
  for (int b = 0; b < batch; ++b)
    eta[b] = orc_eta_trsyl(n, L + b * st, n, U + b * st, n, C + b * st, n, X + b * st, n);
}

void orc_eta_trlyap_batch(int batch, int n, const double *L, const double *S, const double *X,
                          double *eta, int threads) {
  set_threads(threads);
  size_t st = (size_t)n * n;
#pragma omp parallel for schedule(dynamic, 4)
  for (int b = 0; b < batch; ++b)
    eta[b] = orc_eta_trlyap(n, L + b * st, n, S + b * st, n, X + b * st, n);
}

void orc_kron_gesyl_batch(int batch, int n, const double *A, const double *B, const double *C, double *X,
                          int *info, int threads) {
  set_threads(threads);
  size_t st = (size_t)n * n;
#pragma omp parallel
  {
    double *W = (double *)malloc(sizeof(double) * ((size_t)n * n * n * n + (size_t)n * n));
#pragma omp for schedule(dynamic, 1)
    for (int b = 0; b < batch; ++b)
      info[b] = W ? orc_kron_gesyl(n, A + b * st, n, B + b * st, n, C + b * st, n, X + b * st, n, W) : -99;
    free(W);
  }
}

void orc_kron_gelyap_batch(int batch, int n, const double *A, const double *S, double *X, int *info,
                           int threads) {
  set_threads(threads);
  size_t st = (size_t)n * n;
#pragma omp parallel
  {
    double *W = (double *)malloc(sizeof(double) * ((size_t)n * n * n * n + (size_t)n * n));
#pragma omp for schedule(dynamic, 1)
    for (int b = 0; b < batch; ++b)
      info[b] = W ? orc_kron_gelyap(n, A + b * st, n, S + b * st, n, X + b * st, n, W) : -99;
    free(W);
  }
}

void orc_eta_gesyl_batch(int batch, int n, const double *A, const double *B, const double *C,
                         const double *X, double *eta, int threads) {
  set_threads(threads);
  size_t st = (size_t)n * n;
#pragma omp parallel for schedule(dynamic, 4)
  for (int b = 0; b < batch; ++b)
    eta[b] = orc_eta_gesyl(n, A + b * st, n, B + b * st, n, C + b * st, n, X + b * st, n);
}

void orc_eta_gelyap_batch(int batch, int n, const double *A, const double *S, const double *X,
                          double *eta, int threads) {
  set_threads(threads);
  size_t st = (size_t)n * n;
#pragma omp parallel for schedule(dynamic, 4)
  for (int b = 0; b < batch; ++b)
    eta[b] = orc_eta_gelyap(n, A + b * st, n, S + b * st, n, X + b * st, n);
}

/* ------------------------------------------------------------------------
 * Mixed-precision model with FP64 refinement.  The paper computes in double
 * precision only (Preliminary performance results paragraph); this is the
 * textbook iterative refinement written out, used to check the decisions the
 * GPU path takes (iteration counts, fallback flags) on clear-cut inputs:
 *   - Sylvester / Lyapunov: classical refinement.  X = solve_lo(C); then
 *     repeat R = C - (L X + X U) in FP64, eta = backward error, stop when
 *     eta <= tau, D = solve_lo(R), X += D.
 *   - Cholesky: Newton correction of the factor.  Linearising
 *     (X+E)^T (X+E) = A gives X^T E + E^T X = R with R = A - X^T X.  Writing
 *     E = F X with F upper triangular gives F + F^T = X^{-T} R X^{-1} = M, so
 *     F = triu(M) with its diagonal halved.
 * solve_lo runs the same element recurrences as above in FP32.  Refinement
 * stops with flag FALLBACK when eta_k > 0.5 eta_{k-1} (stall) or max_iter
 * corrections did not reach tau, and with flag BREAKDOWN when the FP32
 * factorisation meets a zero/negative pivot or a zero denominator; in both
 * cases the result is recomputed by the FP64 recurrence.
 * ------------------------------------------------------------------------ */
enum { ORC_CONVERGED = 1, ORC_FALLBACK = 2, ORC_BREAKDOWN = 4, ORC_NONFINITE = 8 };

static int potrf_f32(int n, const float *A, float *X) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) X[i + j * n] = 0.0f;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j; ++i) {
      float s = A[i + j * n];
      for (int k = 0; k < i; ++k) s -= X[k + i * n] * X[k + j * n];
      if (i < j) X[i + j * n] = s / X[i + i * n];
      else { if (!(s > 0.0f)) return j + 1; X[j + j * n] = sqrtf(s); }
    }
  return 0;
}

static int sylv_f32(int n, const float *L, const float *U, const float *C, float *X) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      float d = L[i + i * n] + U[j + j * n];
      if (d == 0.0f) return 1 + i + j * n;
      float s = C[i + j * n];
      for (int k = 0; k < i; ++k) s -= L[i + k * n] * X[k + j * n];
      for (int k = 0; k < j; ++k) s -= X[i + k * n] * U[k + j * n];
      X[i + j * n] = s / d;
    }
  return 0;
}

static int all_finite(int m, const double *p) {
  for (int i = 0; i < m; ++i) if (!isfinite(p[i])) return 0;
  return 1;
}

/* op: 0 potrf (B = A), 1 trsyl (A = L, B = U, C), 2 trlyap (A = L, C = S).
 * All matrices n x n with ld = n; X receives the result (full matrix).
 * Returns info; writes iterations, flags and the final eta. */
int orc_refine(int op, int n, const double *A, const double *B, const double *C,
               double *X, int max_iter, double tau, int *iters, int *flags, double *eta_out) {
  size_t m = (size_t)n * n;
  float *lo_a = malloc(m * sizeof(float)), *lo_b = malloc(m * sizeof(float));
  float *lo_r = malloc(m * sizeof(float)), *lo_x = malloc(m * sizeof(float));
  double *R = malloc(m * sizeof(double));
  int info = 0, it = 0, fl = 0;
  double eta = INFINITY, prev = INFINITY;
  *iters = 0;
  if (!all_finite((int)m, A) || (op == 1 && !all_finite((int)m, B)) || (op != 0 && !all_finite((int)m, C)))
    fl |= ORC_NONFINITE;
  /* low-precision copies; for Lyapunov U = L^T and S is mirrored to full */
  for (size_t t = 0; t < m; ++t) lo_a[t] = (float)A[t];
  if (op == 1) for (size_t t = 0; t < m; ++t) lo_b[t] = (float)B[t];
  if (op == 2)
    for (int j = 0; j < n; ++j) for (int i = 0; i < n; ++i) lo_b[i + j * n] = (float)A[j + i * n];
  int lo_info;
  if (op == 0) lo_info = potrf_f32(n, lo_a, lo_x);
  else {
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        lo_r[i + j * n] = (float)((op == 2 && i < j) ? C[j + i * n] : C[i + j * n]);
    lo_info = sylv_f32(n, lo_a, lo_b, lo_r, lo_x);
  }
  if (lo_info != 0) fl |= ORC_BREAKDOWN;
  if (!(fl & (ORC_BREAKDOWN | ORC_NONFINITE))) {
    for (size_t t = 0; t < m; ++t) X[t] = (double)lo_x[t];
    for (;;) {
      if (op == 0) eta = orc_eta_potrf(n, A, n, X, n);
      else if (op == 1) eta = orc_eta_trsyl(n, A, n, B, n, C, n, X, n);
      else eta = orc_eta_trlyap(n, A, n, C, n, X, n);
      if (eta <= tau) { fl |= ORC_CONVERGED; break; }
      if (it >= max_iter || !(eta <= 0.5 * prev)) { fl |= ORC_FALLBACK; break; }
      prev = eta;
      ++it;
      if (op == 0) {
        /* R = A - X^T X (upper), M = X^{-T} R X^{-1}, F = triu(M), diag/2, E = F X */
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            int r = i < j ? i : j, c = i < j ? j : i;
            double s = A[r + c * n];
            int kmax = i < j ? i : j;
            for (int k = 0; k <= kmax; ++k) s -= X[k + i * n] * X[k + j * n];
            lo_r[i + j * n] = (float)s;
          }
        /* lo_x <- X in FP32; W = X^{-T} R (forward substitution, X^T lower) */
        for (size_t t = 0; t < m; ++t) lo_x[t] = (float)X[t];
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            float s = lo_r[i + j * n];
            for (int k = 0; k < i; ++k) s -= lo_x[k + i * n] * lo_a[k + j * n];
            lo_a[i + j * n] = s / lo_x[i + i * n];
          }
        /* M = W X^{-1}: solve M X = W row by row (X upper) */
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) {
            float s = lo_a[i + j * n];
            for (int k = 0; k < j; ++k) s -= lo_b[i + k * n] * lo_x[k + j * n];
            lo_b[i + j * n] = s / lo_x[j + j * n];
          }
        /* F = triu(M) with halved diagonal, then X += F X */
        for (int j = 0; j < n; ++j)
          for (int i = 0; i <= j; ++i) {
            float s = 0.0f;
            for (int k = i; k <= j; ++k) {
              float f = (k == i) ? 0.5f * lo_b[i + i * n] : lo_b[i + k * n];
              s += f * lo_x[k + j * n];
            }
            R[i + j * n] = (double)s;
          }
        for (int j = 0; j < n; ++j)
          for (int i = 0; i <= j; ++i) X[i + j * n] += R[i + j * n];
      } else {
        for (int j = 0; j < n; ++j)
          for (int i = 0; i < n; ++i) {
            double s = (op == 2 && i < j) ? C[j + i * n] : C[i + j * n];
            for (int k = 0; k <= i; ++k) s -= A[i + k * n] * X[k + j * n];
            if (op == 1) for (int k = 0; k <= j; ++k) s -= X[i + k * n] * B[k + j * n];
            else for (int k = 0; k <= j; ++k) s -= X[i + k * n] * A[j + k * n];
            lo_r[i + j * n] = (float)s;
          }
        if (sylv_f32(n, lo_a, lo_b, lo_r, lo_x) != 0) { fl |= ORC_BREAKDOWN; break; }
        for (size_t t = 0; t < m; ++t) X[t] += (double)lo_x[t];
      }
    }
  }
  if (!(fl & ORC_CONVERGED)) {
    if (op == 0) info = orc_potrf(n, A, n, X, n);
    else if (op == 1) info = orc_trsyl(n, A, n, B, n, C, n, X, n);
    else info = orc_trlyap(n, A, n, C, n, X, n);
    if (info == 0) {
      if (op == 0) eta = orc_eta_potrf(n, A, n, X, n);
      else if (op == 1) eta = orc_eta_trsyl(n, A, n, B, n, C, n, X, n);
      else eta = orc_eta_trlyap(n, A, n, C, n, X, n);
    }
  }
  *iters = it;
  *flags = fl;
  *eta_out = eta;
  free(lo_a); free(lo_b); free(lo_r); free(lo_x); free(R);
  return info;
}

/*
 * Plain CPU FP64 oracle for the dense SPD (Gaussian-process) solver path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path: it is written from the definitions in the paper (Fundamentals section,
 * "The Cholesky decomposition": L lower triangular with L L^T = A, solved by
 * forward and back substitution) and from textbook definitions of the
 * surrounding pieces.
 *
 * Deliberately slow and obvious: unblocked loops, sums taken in index order,
 * no fusion and no reordering beyond what each definition states.  The only
 * parallelism is OpenMP over independent output rows, which does not change
 * any summation order.
 *
 * Storage: every matrix is column-major, element (i, j) at M[i + j*ld].
 * Every right-hand-side block is column-major n x k with leading dimension n.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(M, ld, i, j) ((M)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

/* Threads the oracle's parallel loops use (1 without OpenMP). */
int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* O1: squared-exponential GP covariance (stand-in for the paper's kernel     */
/* matrices, Experimental Setup).  A_ij = var * exp(-sum_k (x_ik - x_jk)^2 /  */
/* (2 ls^2)) for i != j, and A_ii = var + noise exactly.  Differences are     */
/* taken directly (no |x|^2 + |y|^2 - 2 x.y expansion).  Full n x n output.   */
/* X is row-major n x d.                                                      */
/* ------------------------------------------------------------------------ */
/* One entry of O1. */
double oracle_gp_entry(const double *X, int64_t d, int64_t i, int64_t j,
                       double ls, double var, double noise) {
  if (i == j) return var + noise;
  double s = 0.0;
  for (int64_t k = 0; k < d; ++k) {
    double diff = X[i * d + k] - X[j * d + k];
    s += diff * diff;
  }
  return var * exp(-s / (2.0 * ls * ls));
}

void oracle_gp_assemble(const double *X, int64_t n, int64_t d, double ls,
                        double var, double noise, double *A) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i)
      AT(A, n, i, j) = oracle_gp_entry(X, d, i, j, ls, var, noise);
}

/* ------------------------------------------------------------------------ */
/* O2: Cholesky factor by its defining equations (Cholesky-Crout order).     */
/* For j = 0..n-1:                                                            */
/*   s     = A_jj - sum_{k<j} L_jk^2            (must be > 0, else info=j+1)  */
/*   L_jj  = sqrt(s)                                                          */
/*   L_ij  = (A_ij - sum_{k<j} L_ik L_jk) / L_jj     for i > j                */
/* Only the lower triangle of A is read.  L is written full n x n with the   */
/* strict upper triangle set to zero.  Returns info (0 = success).           */
/* A row-major copy of L is kept so that each inner product runs over        */
/* contiguous memory; it changes no arithmetic.                              */
/* ------------------------------------------------------------------------ */
int64_t oracle_cholesky(const double *A, int64_t n, int64_t lda, double *L,
                        int64_t ldl) {
  double *R = (double *)calloc((size_t)n * (size_t)n, sizeof(double));
  if (!R) return -1;
  int64_t info = 0;
  for (int64_t j = 0; j < n && info == 0; ++j) {
    const double *rj = R + (size_t)j * n;
    double s = AT(A, lda, j, j);
    for (int64_t k = 0; k < j; ++k) s -= rj[k] * rj[k];
    if (!(s > 0.0)) {  /* also catches NaN */
      info = j + 1;
      break;
    }
    const double ljj = sqrt(s);
    R[(size_t)j * n + j] = ljj;
#pragma omp parallel for schedule(static)
    for (int64_t i = j + 1; i < n; ++i) {
      const double *ri = R + (size_t)i * n;
      double t = AT(A, lda, i, j);
      for (int64_t k = 0; k < j; ++k) t -= ri[k] * rj[k];
      R[(size_t)i * n + j] = t / ljj;
    }
  }
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i)
      AT(L, ldl, i, j) = (i >= j) ? R[(size_t)i * n + j] : 0.0;
  free(R);
  return info;
}

/* ------------------------------------------------------------------------ */
/* O3: forward substitution  L y = b   y_i = (b_i - sum_{k<i} L_ik y_k)/L_ii  */
/*     back substitution     L^T x = y x_i = (y_i - sum_{k>i} L_ki x_k)/L_ii  */
/* In place on B (n x k, leading dimension ldb); each column independent.    */
/* ------------------------------------------------------------------------ */
void oracle_forward(const double *L, int64_t n, int64_t ldl, double *B,
                    int64_t k, int64_t ldb) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < k; ++c) {
    double *b = B + (size_t)c * ldb;
    for (int64_t i = 0; i < n; ++i) {
      double t = b[i];
      for (int64_t m = 0; m < i; ++m) t -= AT(L, ldl, i, m) * b[m];
      b[i] = t / AT(L, ldl, i, i);
    }
  }
}

void oracle_backward(const double *L, int64_t n, int64_t ldl, double *B,
                     int64_t k, int64_t ldb) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < k; ++c) {
    double *b = B + (size_t)c * ldb;
    for (int64_t i = n - 1; i >= 0; --i) {
      double t = b[i];
      for (int64_t m = i + 1; m < n; ++m) t -= AT(L, ldl, m, i) * b[m];
      b[i] = t / AT(L, ldl, i, i);
    }
  }
}

/* O4: x = A^{-1} b through the factor: forward then back substitution.      */
void oracle_solve(const double *L, int64_t n, int64_t ldl, double *B,
                  int64_t k, int64_t ldb) {
  oracle_forward(L, n, ldl, B, k, ldb);
  oracle_backward(L, n, ldl, B, k, ldb);
}

/* ------------------------------------------------------------------------ */
/* Residual R = B - A X with long-double accumulation.  A full (n x n, lda). */
/* ------------------------------------------------------------------------ */
void oracle_residual(const double *A, int64_t n, int64_t lda, const double *X,
                     const double *B, int64_t k, double *R) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t c = 0; c < k; ++c) {
      long double t = B[(size_t)c * n + i];
      for (int64_t j = 0; j < n; ++j)
        t -= (long double)AT(A, lda, i, j) * (long double)X[(size_t)c * n + j];
      R[(size_t)c * n + i] = (double)t;
    }
  }
}

/* Matrix-free residual R = B - (K(X,X) + noise I) Xs, entries of K from O1. */
void oracle_gp_residual(const double *F, int64_t n, int64_t d, double ls,
                        double var, double noise, const double *Xs,
                        const double *B, int64_t k, double *R) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t c = 0; c < k; ++c) {
      long double t = B[(size_t)c * n + i];
      for (int64_t j = 0; j < n; ++j)
        t -= (long double)oracle_gp_entry(F, d, i, j, ls, var, noise) *
             (long double)Xs[(size_t)c * n + j];
      R[(size_t)c * n + i] = (double)t;
    }
  }
}

static double nrm2_col(const double *v, int64_t n) {
  long double s = 0.0L;
  for (int64_t i = 0; i < n; ++i) s += (long double)v[i] * v[i];
  return (double)sqrtl(s);
}

static double dot_col(const double *a, const double *b, int64_t n) {
  long double s = 0.0L;
  for (int64_t i = 0; i < n; ++i) s += (long double)a[i] * b[i];
  return (double)s;
}

/* ------------------------------------------------------------------------ */
/* O5: iterative refinement with a (possibly low-precision) factor F         */
/* (Wilkinson/Moler; the three-precision form of Carson & Higham, 2018):     */
/*   x = F^-T F^-1 b;  repeat { r = b - A x;  stop if certified;             */
/*                              d = F^-T F^-1 r;  x += d }                   */
/* Stopping: with lam > 0 a lower bound on lambda_min(A) (the GP noise       */
/* variance), ||x - x*|| <= ||r|| / lam, so cert = ||r|| / (lam ||x||) is a  */
/* rigorous bound on the relative error; stop once cert <= tol/2.  With      */
/* lam <= 0 stop once ||d|| <= tol ||x||.  Per right-hand side.              */
/* iters[c] receives the number of corrections applied, cert[c] the final   */
/* certificate (or ||d||/||x||).  Returns the number of columns that did not */
/* converge within max_iter.                                                 */
/* ------------------------------------------------------------------------ */
int64_t oracle_refine(const double *F, int64_t ldf, const double *A,
                      int64_t lda, int64_t n, const double *B, double *X,
                      int64_t k, double lam, double tol, int64_t max_iter,
                      int64_t *iters, double *cert) {
  double *r = (double *)malloc((size_t)n * sizeof(double));
  int64_t failed = 0;
  for (int64_t c = 0; c < k; ++c) {
    double *x = X + (size_t)c * n;
    const double *b = B + (size_t)c * n;
    memcpy(x, b, (size_t)n * sizeof(double));
    oracle_solve(F, n, ldf, x, 1, n);
    int64_t it = 0;
    double cc = INFINITY;
    for (;;) {
      oracle_residual(A, n, lda, x, b, 1, r);
      if (lam > 0.0) {
        cc = nrm2_col(r, n) / (lam * nrm2_col(x, n));
        if (cc <= 0.5 * tol) break;
      }
      if (it >= max_iter) break;
      oracle_solve(F, n, ldf, r, 1, n);
      for (int64_t i = 0; i < n; ++i) x[i] += r[i];
      ++it;
      if (lam <= 0.0) {
        cc = nrm2_col(r, n) / nrm2_col(x, n);
        if (cc <= tol) break;
      }
    }
    if (!(cc <= (lam > 0.0 ? 0.5 * tol : tol))) ++failed;
    if (iters) iters[c] = it;
    if (cert) cert[c] = cc;
  }
  free(r);
  return failed;
}

/* ------------------------------------------------------------------------ */
/* O6: conjugate gradients preconditioned with M = F F^T (Shewchuk's         */
/* preconditioned CG; the paper's CG with z = M^-1 r in place of r in the    */
/* search direction).  Starting point x0 = M^-1 b.                           */
/*   r = b - A x; z = M^-1 r; p = z; rho = r.z                               */
/*   loop: q = A p; alpha = rho / p.q; x += alpha p; r -= alpha q;           */
/*         every `recompute` iterations r = b - A x (the paper's periodic    */
/*         true-residual recomputation);                                     */
/*         z = M^-1 r; rho' = r.z; p = z + (rho'/rho) p; rho = rho'          */
/* Convergence is decided on the true residual: whenever the recurrence      */
/* residual certifies, the true residual is recomputed and certified.        */
/* ------------------------------------------------------------------------ */
int64_t oracle_pcg(const double *F, int64_t ldf, const double *A, int64_t lda,
                   int64_t n, const double *B, double *X, int64_t k,
                   double lam, double tol, int64_t max_iter, int64_t recompute,
                   int64_t *iters, double *cert) {
  double *r = (double *)malloc((size_t)n * sizeof(double));
  double *z = (double *)malloc((size_t)n * sizeof(double));
  double *p = (double *)malloc((size_t)n * sizeof(double));
  double *q = (double *)malloc((size_t)n * sizeof(double));
  int64_t failed = 0;
  for (int64_t c = 0; c < k; ++c) {
    double *x = X + (size_t)c * n;
    const double *b = B + (size_t)c * n;
    memcpy(x, b, (size_t)n * sizeof(double));
    oracle_solve(F, n, ldf, x, 1, n);
    oracle_residual(A, n, lda, x, b, 1, r);
    double cc = nrm2_col(r, n) / (lam * nrm2_col(x, n));
    int64_t it = 0;
    if (!(cc <= 0.5 * tol)) {
      memcpy(z, r, (size_t)n * sizeof(double));
      oracle_solve(F, n, ldf, z, 1, n);
      memcpy(p, z, (size_t)n * sizeof(double));
      double rho = dot_col(r, z, n);
      while (it < max_iter) {
        /* q = A p (plain FP64 product, long-double accumulation) */
        for (int64_t i = 0; i < n; ++i) q[i] = 0.0;
        for (int64_t i = 0; i < n; ++i) {
          long double t = 0.0L;
          for (int64_t j = 0; j < n; ++j)
            t += (long double)AT(A, lda, i, j) * p[j];
          q[i] = (double)t;
        }
        const double alpha = rho / dot_col(p, q, n);
        for (int64_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (int64_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        ++it;
        if (recompute > 0 && it % recompute == 0)
          oracle_residual(A, n, lda, x, b, 1, r);
        cc = nrm2_col(r, n) / (lam * nrm2_col(x, n));
        if (cc <= 0.5 * tol) {
          oracle_residual(A, n, lda, x, b, 1, r);
          cc = nrm2_col(r, n) / (lam * nrm2_col(x, n));
          if (cc <= 0.5 * tol) break;
        }
        memcpy(z, r, (size_t)n * sizeof(double));
        oracle_solve(F, n, ldf, z, 1, n);
        const double rho_new = dot_col(r, z, n);
        const double beta = rho_new / rho;
        rho = rho_new;
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
      }
    }
    if (!(cc <= 0.5 * tol)) ++failed;
    if (iters) iters[c] = it;
    if (cert) cert[c] = cc;
  }
  free(r);
  free(z);
  free(p);
  free(q);
  return failed;
}

/* ------------------------------------------------------------------------ */
/* The paper's conjugate gradient method (Fundamentals section, "The         */
/* Conjugate Gradient method", left column of its CG / Cholesky algorithm    */
/* figure, after Shewchuk), one right-hand side at a time, x holding the     */
/* starting guess on entry:                                                  */
/*   s = r = b - A x;  u = u0 = r.r                                          */
/*   while u > eps^2 u0 (and fewer than max_iter iterations):                */
/*     t = A s;  alpha = u / s.t;  x += alpha s;                             */
/*     r -= alpha t, except that every `recompute`-th iteration takes the    */
/*       true residual r = b - A x instead (the paper's periodic             */
/*       recomputation; recompute <= 0 never does);                          */
/*     v = u;  u = r.r;  beta = u / v;  s = r + beta s                       */
/* A full (n x n, lda).  Products and dots accumulate in long double.        */
/* iters[c] = iterations taken, relres[c] = sqrt(u / u0) at exit (0 when     */
/* b - A x0 = 0).  Returns the number of columns stopped by max_iter.        */
/* ------------------------------------------------------------------------ */
static void matvec(const double *A, int64_t lda, int64_t n, const double *v,
                   double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    long double t = 0.0L;
    for (int64_t j = 0; j < n; ++j) t += (long double)AT(A, lda, i, j) * v[j];
    out[i] = (double)t;
  }
}

int64_t oracle_cg(const double *A, int64_t lda, int64_t n, const double *B,
                  double *X, int64_t k, double eps, int64_t max_iter,
                  int64_t recompute, int64_t *iters, double *relres) {
  double *r = (double *)malloc((size_t)n * sizeof(double));
  double *s = (double *)malloc((size_t)n * sizeof(double));
  double *t = (double *)malloc((size_t)n * sizeof(double));
  int64_t stopped = 0;
  for (int64_t c = 0; c < k; ++c) {
    double *x = X + (size_t)c * n;
    const double *b = B + (size_t)c * n;
    matvec(A, lda, n, x, t);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
    memcpy(s, r, (size_t)n * sizeof(double));
    double u = dot_col(r, r, n);
    const double u0 = u;
    int64_t it = 0;
    while (u > eps * eps * u0 && it < max_iter) {
      matvec(A, lda, n, s, t);
      const double alpha = u / dot_col(s, t, n);
      for (int64_t i = 0; i < n; ++i) x[i] += alpha * s[i];
      ++it;
      if (recompute > 0 && it % recompute == 0) {
        matvec(A, lda, n, x, t);
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
      } else {
        for (int64_t i = 0; i < n; ++i) r[i] -= alpha * t[i];
      }
      const double v = u;
      u = dot_col(r, r, n);
      const double beta = u / v;
      for (int64_t i = 0; i < n; ++i) s[i] = r[i] + beta * s[i];
    }
    if (u > eps * eps * u0) ++stopped;
    if (iters) iters[c] = it;
    if (relres) relres[c] = u0 > 0.0 ? sqrt(u / u0) : 0.0;
  }
  free(r);
  free(s);
  free(t);
  return stopped;
}

/* ------------------------------------------------------------------------ */
/* Checkers.                                                                 */
/* backward error ||A - L L^T||_F / ||A||_F over the full symmetric matrix,  */
/* with L lower (upper triangle ignored) and A's lower triangle mirrored.    */
/* ------------------------------------------------------------------------ */
double oracle_backward_error(const double *A, int64_t lda, const double *L,
                             int64_t ldl, int64_t n) {
  long double num = 0.0L, den = 0.0L;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : num, den)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = 0; j <= i; ++j) {
      long double s = 0.0L;
      for (int64_t k = 0; k <= j; ++k)
        s += (long double)AT(L, ldl, i, k) * AT(L, ldl, j, k);
      const long double a = AT(A, lda, i, j);
      const long double e = a - s;
      const long double w = (i == j) ? 1.0L : 2.0L;
      num += w * e * e;
      den += w * a * a;
    }
  }
  return (double)sqrtl(num / den);
}

/* Randomized backward-error estimate for orders where the exact checker is */
/* too slow (Hutchinson's trace estimator): for probe vectors z ~ N(0, I),  */
/* E[||E z||^2] = ||E||_F^2 with E = A - L L^T.  For the k probes Z (n x k, */
/* column-major) this returns num = sum_p ||A z_p - L (L^T z_p)||^2 and     */
/* den = sum_p ||A z_p||^2, so sqrt(num / den) estimates ||E||_F / ||A||_F.  */
/* A is dense (lda) or, with A == NULL, the GP matrix of O1 from features F */
/* (n x d row-major), each entry computed once for all probes.  L lower,    */
/* column-major (ldl), upper triangle ignored.  Long-double accumulation.   */
void oracle_backward_error_probes(const double *A, int64_t lda, const double *F,
                                  int64_t d, double ls, double var, double noise,
                                  const double *L, int64_t ldl, int64_t n,
                                  const double *Z, int64_t k, double *num,
                                  double *den) {
  long double *W = (long double *)calloc((size_t)n * k, sizeof(long double));
  long double *Y = (long double *)calloc((size_t)n * k, sizeof(long double));
  long double *AZ = (long double *)calloc((size_t)n * k, sizeof(long double));
  /* W = L^T Z: W_j = sum_{i >= j} L_ij z_i */
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t j = 0; j < n; ++j)
    for (int64_t p = 0; p < k; ++p) {
      long double t = 0.0L;
      for (int64_t i = j; i < n; ++i)
        t += (long double)AT(L, ldl, i, j) * Z[(size_t)p * n + i];
      W[(size_t)p * n + j] = t;
    }
  /* Y = L W: Y_i = sum_{j <= i} L_ij W_j, by row blocks walking columns */
  const int64_t RB = 64;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t r0 = 0; r0 < n; r0 += RB) {
    const int64_t r1 = r0 + RB < n ? r0 + RB : n;
    for (int64_t j = 0; j < r1; ++j)
      for (int64_t i = (j > r0 ? j : r0); i < r1; ++i)
        for (int64_t p = 0; p < k; ++p)
          Y[(size_t)p * n + i] += (long double)AT(L, ldl, i, j) * W[(size_t)p * n + j];
  }
  /* A Z, each A_ij used for every probe */
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) {
      const long double a = A ? (long double)AT(A, lda, (i > j ? i : j), (i > j ? j : i))
                              : (long double)oracle_gp_entry(F, d, i, j, ls, var, noise);
      for (int64_t p = 0; p < k; ++p) AZ[(size_t)p * n + i] += a * Z[(size_t)p * n + j];
    }
  long double nu = 0.0L, de = 0.0L;
  for (size_t e = 0; e < (size_t)n * k; ++e) {
    const long double r = AZ[e] - Y[e];
    nu += r * r;
    de += AZ[e] * AZ[e];
  }
  *num = (double)nu;
  *den = (double)de;
  free(W);
  free(Y);
  free(AZ);
}

/* Certificate cert = ||b - A x||_2 / (lam ||x||_2) for one column, given    */
/* its residual; lam a lower bound on lambda_min(A).                         */
double oracle_certificate(const double *r, const double *x, int64_t n,
                          double lam) {
  return nrm2_col(r, n) / (lam * nrm2_col(x, n));
}

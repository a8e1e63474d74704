/*
 * ORACLE -- test infrastructure only.  Nothing in the library's product path
 * may link, load or call this file; it exists so that the tests, the smoke
 * check and the CPU baseline of the benchmark have an independent answer.
 *
 * What it computes: the solution X = P^{-1} F of the block-tridiagonal system
 * of eq. (main-eq) of Terekhov, "A fast parallel algorithm for solving
 * block-tridiagonal systems of linear equations including the domain
 * decomposition method" (Sec. 1):
 *
 *     -A_j X_{j-1} + C_j X_j - B_j X_{j+1} = F_j ,   j = 1..N,
 *
 * with M x M blocks and A_1, B_N absent.  Because the method of the paper
 * (Algorithms 1 and 2) is a direct method, its result is this X up to
 * rounding, and the oracle is the plain definition: a sequential block
 * Gaussian elimination ("matrix sweep", the pre-factorized block solver the
 * paper refers to in Sec. 2.2, cost O(M^3 N)) over the whole system, with no
 * subdomains, no dichotomy and no reordering:
 *
 *     D_1 = C_1,               D_j = C_j - A_j alpha_{j-1},
 *     alpha_j = D_j^{-1} B_j,
 *     beta_1 = D_1^{-1} F_1,   beta_j = D_j^{-1} (F_j + A_j beta_{j-1}),
 *     X_N = beta_N,            X_j = alpha_j X_{j+1} + beta_j.
 *
 * D_j^{-1} is applied through an LU factorization with partial pivoting (row
 * interchanges inside the block), written out here without BLAS.  All
 * arithmetic is float64.  OpenMP runs independent right-hand-side columns
 * (and the independent columns of alpha_j) in parallel; every column is
 * computed by the same sequential loop, so the result does not depend on the
 * thread count.
 *
 * Block formats: A and B are DENSE (M x M column-major per block) or DIAG
 * (diagonal only, [N][M]); C is DENSE or TRIDIAG ([N][3][M]: sub, diag,
 * super).  Right-hand sides are column-major (N*M) x K with leading
 * dimension ldf.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_DENSE 0
#define OR_DIAG 1
#define OR_TRIDIAG 2

/* status codes */
#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2
#define OR_ESINGULAR 3

/* relative pivot threshold: a pivot |u_kk| <= OR_PIVTOL * ||D_j||_inf means singular */
#define OR_PIVTOL 1e-14

/* Planted-mistake switch for the oracle's self-tests: a build with
 * -DORACLE_MUTANT=n (n > 0) carries one deliberate error, and the pin tests
 * must reject every such build.  The default build (0) has none. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

static void expand(int fmt, const double* src, int64_t j, int64_t M, double* out) {
  const int64_t MM = M * M;
  if (fmt == OR_DENSE) {
    memcpy(out, src + j * MM, (size_t)MM * sizeof(double));
    return;
  }
  memset(out, 0, (size_t)MM * sizeof(double));
  if (fmt == OR_DIAG) {
    for (int64_t i = 0; i < M; ++i) out[i + i * M] = src[j * M + i];
  } else { /* TRIDIAG */
    const double* t = src + j * 3 * M;
    for (int64_t i = 0; i < M; ++i) {
      if (i > 0) out[i + (i - 1) * M] = t[i];
      out[i + i * M] = t[M + i];
      if (i < M - 1) out[i + (i + 1) * M] = t[2 * M + i];
    }
  }
}

/* LU with partial pivoting, in place, column-major a (M x M).  piv[k] = row swapped with k. */
static int lu_factor(double* a, int64_t M, int32_t* piv) {
  double norm = 0.0;
  for (int64_t r = 0; r < M; ++r) {
    double s = 0.0;
    for (int64_t c = 0; c < M; ++c) s += fabs(a[r + c * M]);
    if (s > norm) norm = s;
  }
  for (int64_t k = 0; k < M; ++k) {
    int64_t p = k;
    double best = fabs(a[k + k * M]);
    for (int64_t i = k + 1; i < M; ++i) {
      double v = fabs(a[i + k * M]);
      if (v > best) { best = v; p = i; }
    }
    if (!(best > OR_PIVTOL * norm)) return OR_ESINGULAR; /* also catches NaN */
    if (ORACLE_MUTANT == 5) p = k;
    piv[k] = (int32_t)p;
    if (p != k)
      for (int64_t c = 0; c < M; ++c) {
        double t = a[k + c * M]; a[k + c * M] = a[p + c * M]; a[p + c * M] = t;
      }
    const double inv = 1.0 / a[k + k * M];
    for (int64_t i = k + 1; i < M; ++i) a[i + k * M] *= inv;
    for (int64_t c = k + 1; c < M; ++c) {
      const double u = a[k + c * M];
      if (u != 0.0)
        for (int64_t i = k + 1; i < M; ++i) a[i + c * M] -= a[i + k * M] * u;
    }
  }
  return OR_OK;
}

/* solve (LU) x = b in place for one column b */
static void lu_solve_col(const double* lu, const int32_t* piv, int64_t M, double* b) {
  for (int64_t k = 0; k < M; ++k) {
    int64_t p = piv[k];
    if (p != k) { double t = b[k]; b[k] = b[p]; b[p] = t; }
  }
  for (int64_t k = 0; k < M; ++k) { /* unit lower */
    const double bk = b[k];
    if (bk != 0.0)
      for (int64_t i = k + 1; i < M; ++i) b[i] -= lu[i + k * M] * bk;
  }
  for (int64_t k = M - 1; k >= 0; --k) { /* upper */
    b[k] /= lu[k + k * M];
    const double bk = b[k];
    if (bk != 0.0)
      for (int64_t i = 0; i < k; ++i) b[i] -= lu[i + k * M] * bk;
  }
}

/* y += G x  with G a dense M x M column-major block (one column x) */
static void gemv_acc(const double* G, int64_t M, const double* x, double* y) {
  for (int64_t c = 0; c < M; ++c) {
    const double xc = x[c];
    if (xc != 0.0)
      for (int64_t i = 0; i < M; ++i) y[i] += G[i + c * M] * xc;
  }
}

/* Factored system: LU of every D_j and alpha_j = D_j^{-1} B_j. */
typedef struct {
  int64_t N, M;
  int fmt_A;
  const double* A; /* caller keeps A alive while the factor is used */
  double* lu;      /* N * M * M */
  int32_t* piv;    /* N * M */
  double* alpha;   /* N * M * M (alpha_N unused) */
  int64_t bad_block;
} or_factor;

void oracle_free(or_factor* f) {
  if (!f) return;
  free(f->lu); free(f->piv); free(f->alpha); free(f);
}

int64_t oracle_bad_block(const or_factor* f) { return f ? f->bad_block : -1; }

/* Forward elimination of the matrix: D_j and alpha_j for j = 1..N. */
int oracle_factor(int64_t N, int64_t M, int fmt_A, int fmt_B, int fmt_C,
                  const double* A, const double* B, const double* C, int nthreads,
                  or_factor** out, int64_t* bad_block) {
  *out = NULL;
  if (bad_block) *bad_block = -1;
  if (N < 1 || M < 1) return OR_EINVAL;
  if (!(fmt_A == OR_DENSE || fmt_A == OR_DIAG) || !(fmt_B == OR_DENSE || fmt_B == OR_DIAG) ||
      !(fmt_C == OR_DENSE || fmt_C == OR_TRIDIAG))
    return OR_EINVAL;
  const int64_t MM = M * M;
  or_factor* f = (or_factor*)calloc(1, sizeof(or_factor));
  double* Aj = (double*)malloc((size_t)MM * sizeof(double));
  double* Bj = (double*)malloc((size_t)MM * sizeof(double));
  if (!f || !Aj || !Bj) { free(f); free(Aj); free(Bj); return OR_ENOMEM; }
  f->N = N; f->M = M; f->fmt_A = fmt_A; f->A = A; f->bad_block = -1;
  f->lu = (double*)malloc((size_t)(N * MM) * sizeof(double));
  f->piv = (int32_t*)malloc((size_t)(N * M) * sizeof(int32_t));
  f->alpha = (double*)malloc((size_t)(N * MM) * sizeof(double));
  if (!f->lu || !f->piv || !f->alpha) { oracle_free(f); free(Aj); free(Bj); return OR_ENOMEM; }
  (void)nthreads;
  for (int64_t j = 0; j < N; ++j) {
    double* D = f->lu + j * MM;
    expand(fmt_C, C, j, M, D);                 /* D_j = C_j */
    if (j > 0) {                               /* D_j -= A_j alpha_{j-1} */
      expand(fmt_A, A, j, M, Aj);
      const double* al = f->alpha + (j - 1) * MM;
#pragma omp parallel for schedule(static) num_threads(nthreads)
      for (int64_t c = 0; c < M; ++c) {
        double* col = (double*)malloc((size_t)M * sizeof(double));
        memset(col, 0, (size_t)M * sizeof(double));
        gemv_acc(Aj, M, al + c * M, col);
        for (int64_t i = 0; i < M; ++i) D[i + c * M] += (ORACLE_MUTANT == 3 ? 1.0 : -1.0) * col[i];
        free(col);
      }
    }
    if (lu_factor(D, M, f->piv + j * M) != OR_OK) {
      f->bad_block = j;
      if (bad_block) *bad_block = j;
      oracle_free(f); free(Aj); free(Bj);
      return OR_ESINGULAR;
    }
    if (j < N - 1) {                           /* alpha_j = D_j^{-1} B_j */
      expand(fmt_B, B, j, M, Bj);
      if (ORACLE_MUTANT == 2)
        for (int64_t r = 0; r < M; ++r)
          for (int64_t c = r + 1; c < M; ++c) { double t = Bj[r + c * M]; Bj[r + c * M] = Bj[c + r * M]; Bj[c + r * M] = t; }
      double* al = f->alpha + j * MM;
      memcpy(al, Bj, (size_t)MM * sizeof(double));
#pragma omp parallel for schedule(static) num_threads(nthreads)
      for (int64_t c = 0; c < M; ++c) lu_solve_col(D, f->piv + j * M, M, al + c * M);
    }
  }
  free(Aj); free(Bj);
  *out = f;
  return OR_OK;
}

/* Forward and backward sweeps for K right-hand sides with the factored matrix. */
int oracle_solve(const or_factor* f, const double* F, int64_t ldf, double* X, int64_t ldx,
                 int64_t K, int nthreads) {
  if (!f || K < 0) return OR_EINVAL;
  const int64_t N = f->N, M = f->M, MM = M * M;
  if (ldf < N * M || ldx < N * M) return OR_EINVAL;
  int status = OR_OK;
#pragma omp parallel num_threads(nthreads)
  {
    double* Aj = (double*)malloc((size_t)MM * sizeof(double));
    double* tmp = (double*)malloc((size_t)M * sizeof(double));
    if (!Aj || !tmp) {
#pragma omp atomic write
      status = OR_ENOMEM;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t k = 0; k < K; ++k) {
        const double* Fk = F + k * ldf;
        double* Xk = X + k * ldx; /* beta_j is kept in X_j until the backward sweep */
        for (int64_t j = 0; j < N; ++j) {
          double* bj = Xk + j * M;
          memcpy(bj, Fk + j * M, (size_t)M * sizeof(double));       /* F_j */
          if (j > 0 && ORACLE_MUTANT != 6) {                          /* + A_j beta_{j-1} */
            expand(f->fmt_A, f->A, j, M, Aj);
            if (ORACLE_MUTANT == 1)
              for (int64_t i = 0; i < MM; ++i) Aj[i] = -Aj[i];
            gemv_acc(Aj, M, Xk + (j - 1) * M, bj);
          }
          lu_solve_col(f->lu + j * MM, f->piv + j * M, M, bj);        /* D_j^{-1} ( . ) */
        }
        for (int64_t j = N - 2; j >= 0; --j) {                        /* X_j = alpha_j X_{j+1} + beta_j */
          memset(tmp, 0, (size_t)M * sizeof(double));
          gemv_acc(f->alpha + (ORACLE_MUTANT == 4 && j + 1 < N - 1 ? j + 1 : j) * MM, M, Xk + (j + 1) * M, tmp);
          for (int64_t i = 0; i < M; ++i) Xk[j * M + i] += tmp[i];
        }
      }
    }
    free(Aj); free(tmp);
  }
  return status;
}

/* Factor, solve and free in one call. */
int oracle_solve_system(int64_t N, int64_t M, int fmt_A, int fmt_B, int fmt_C,
                        const double* A, const double* B, const double* C,
                        const double* F, int64_t ldf, double* X, int64_t ldx, int64_t K,
                        int nthreads, int64_t* bad_block) {
  or_factor* f = NULL;
  int st = oracle_factor(N, M, fmt_A, fmt_B, fmt_C, A, B, C, nthreads, &f, bad_block);
  if (st != OR_OK) return st;
  st = oracle_solve(f, F, ldf, X, ldx, K, nthreads);
  oracle_free(f);
  return st;
}

/* Y = P X straight from eq. (main-eq): Y_j = -A_j X_{j-1} + C_j X_j - B_j X_{j+1}. */
int oracle_apply(int64_t N, int64_t M, int fmt_A, int fmt_B, int fmt_C,
                 const double* A, const double* B, const double* C,
                 const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t K, int nthreads) {
  if (N < 1 || M < 1 || ldx < N * M || ldy < N * M) return OR_EINVAL;
  const int64_t MM = M * M;
  int status = OR_OK;
#pragma omp parallel num_threads(nthreads)
  {
    double* blk = (double*)malloc((size_t)MM * sizeof(double));
    if (!blk) {
#pragma omp atomic write
      status = OR_ENOMEM;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t k = 0; k < K; ++k) {
        const double* Xk = X + k * ldx;
        double* Yk = Y + k * ldy;
        for (int64_t j = 0; j < N; ++j) {
          double* y = Yk + j * M;
          memset(y, 0, (size_t)M * sizeof(double));
          expand(fmt_C, C, j, M, blk);
          gemv_acc(blk, M, Xk + j * M, y);
          if (j > 0) {
            expand(fmt_A, A, j, M, blk);
            for (int64_t i = 0; i < MM; ++i) blk[i] = -blk[i];
            gemv_acc(blk, M, Xk + (j - 1) * M, y);
          }
          if (j < N - 1) {
            expand(fmt_B, B, j, M, blk);
            for (int64_t i = 0; i < MM; ++i) blk[i] = -blk[i];
            gemv_acc(blk, M, Xk + (j + 1) * M, y);
          }
        }
      }
    }
    free(blk);
  }
  return status;
}

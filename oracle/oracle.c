/*
 * CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Build: gcc -std=c11 -O2 -ffp-contract=off -fopenmp -fPIC -shared oracle.c -lm
 * (-ffp-contract=off: every multiply-add below is exactly the fma() call or
 * the separate multiply and add that is written, nothing is fused behind the
 * reader's back).  The row loops of X^2 and of the update run on OpenMP
 * threads: each output row depends only on the inputs, so the result does not
 * depend on the thread count.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int32_t orc_threads(int32_t n)
{
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* Empty rows (nnz 0, indices -1, values 0), written row by row in the static
 * schedule of the row loops below: with threads bound to cores, the pages of
 * a row land on the memory node of the thread that will fill it. */
void orc_rows_init(int32_t N, int32_t M, int32_t *nnz, int32_t *idx, void *val, int32_t val_size)
{
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < N; ++i) {
    nnz[i] = 0;
    for (int32_t s = 0; s < M; ++s) idx[(int64_t)i * M + s] = -1;
    memset((char *)val + (int64_t)i * M * val_size, 0, (size_t)M * (size_t)val_size);
  }
}

/* ------------------------------------------------------------------------ */
/* pairwise tree sum (the fixed summation order of every trace and norm)     */
/* ------------------------------------------------------------------------ */
double orc_pairwise(int64_t n, const double *d)
{
  if (n <= 0) return 0.0;
  double *w = (double *)malloc((size_t)n * sizeof(double));
  if (!w) return NAN;
  memcpy(w, d, (size_t)n * sizeof(double));
  while (n > 1) {
    int64_t h = n / 2;
    for (int64_t i = 0; i < h; ++i) w[i] = w[2 * i] + w[2 * i + 1];
    if (n & 1) w[h] = w[n - 1];
    n = h + (n & 1);
  }
  double s = w[0];
  free(w);
  return s;
}

/* ------------------------------------------------------------------------ */
/* checks                                                                   */
/* ------------------------------------------------------------------------ */
int orc_check_ell(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx)
{
  if (N <= 0 || M <= 0) return ORC_EINVAL;
  for (int32_t i = 0; i < N; ++i) {
    if (nnz[i] < 0 || nnz[i] > M) return ORC_EINVAL;
    const int32_t *c = idx + (int64_t)i * M;
    for (int32_t s = 0; s < nnz[i]; ++s) {
      if (c[s] < 0 || c[s] >= N) return ORC_EINVAL;
      if (s > 0 && c[s] <= c[s - 1]) return ORC_EINVAL;
    }
  }
  return ORC_OK;
}

int orc_check_finite_f64(int32_t N, int32_t M, const int32_t *nnz, const double *val)
{
  for (int32_t i = 0; i < N; ++i)
    for (int32_t s = 0; s < nnz[i]; ++s)
      if (!isfinite(val[(int64_t)i * M + s])) return ORC_ENONFINITE;
  return ORC_OK;
}

int64_t orc_x2_fma_count(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx)
{
  int64_t f = 0;
  for (int32_t i = 0; i < N; ++i)
    for (int32_t s = 0; s < nnz[i]; ++s) f += nnz[idx[(int64_t)i * M + s]];
  return f;
}

static int cmp_i32(const void *a, const void *b)
{
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* ------------------------------------------------------------------------ */
/* X^2 with threshold: Gustavson row-by-row product with a dense sparse      */
/* accumulator (SPA).  For row i, k runs over row i in ascending order, j    */
/* over row k in ascending order, acc[j] = fma(X_ik, X_kj, acc[j]).          */
/* ------------------------------------------------------------------------ */
/* Row i of prune(X.X, tau) in FP64 into (idx2r, val2r) (at most M2 entries):
 * returns the surviving count (which may exceed M2); *xii = X_ii, *dii = the
 * unpruned (X.X)_ii.  acc, mark: N zeros on entry and on return; touched: N. */
static int32_t x2_row_f64(int32_t i, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
                          double tau, int32_t M2, int32_t *idx2r, double *val2r, double *acc, char *mark,
                          int32_t *touched, double *xii, double *dii)
{
  const int32_t *ci = idx + (int64_t)i * M;
  const double *vi = val + (int64_t)i * M;
  int32_t nt = 0;
  *xii = 0.0;
  for (int32_t s = 0; s < nnz[i]; ++s) {
    int32_t k = ci[s];
    double a = vi[s];
    if (k == i) *xii = a;
    const int32_t *ck = idx + (int64_t)k * M;
    const double *vk = val + (int64_t)k * M;
    for (int32_t t = 0; t < nnz[k]; ++t) {
      int32_t j = ck[t];
      if (!mark[j]) { mark[j] = 1; touched[nt++] = j; }
      acc[j] = fma(a, vk[t], acc[j]);
    }
  }
  *dii = acc[i];
  qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
  int32_t c = 0;
  for (int32_t q = 0; q < nt; ++q) {
    int32_t j = touched[q];
    if (fabs(acc[j]) > tau) {
      if (c < M2) {
        idx2r[c] = j;
        val2r[c] = acc[j];
      }
      ++c;
    }
    acc[j] = 0.0;
    mark[j] = 0;
  }
  return c;
}

int orc_x2_f64(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
               double tau, int32_t M2, int32_t *nnz2, int32_t *idx2, double *val2,
               double *d1, double *d2, int32_t *maxw)
{
  int failed = 0, overflow = 0;
  int32_t widest = 0;
#pragma omp parallel reduction(| : failed, overflow) reduction(max : widest)
  {
    /* the dense accumulator of one row, its marks and touched columns */
    double *acc = (double *)calloc((size_t)N, sizeof(double));
    char *mark = (char *)calloc((size_t)N, 1);
    int32_t *touched = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    const int ok = acc && mark && touched;
    if (!ok) failed = 1;
#pragma omp for schedule(static)
    for (int32_t i = 0; i < N; ++i) {
      if (!ok) continue;
      double xii, dii;
      const int32_t c = x2_row_f64(i, M, nnz, idx, val, tau, M2, idx2 + (int64_t)i * M2, val2 + (int64_t)i * M2,
                                   acc, mark, touched, &xii, &dii);
      if (d1) d1[i] = xii;
      if (d2) d2[i] = dii;
      if (c > M2) { overflow = 1; nnz2[i] = M2; } else nnz2[i] = c;
      if (c > widest) widest = c;
    }
    free(acc); free(mark); free(touched);
  }
  if (failed) return ORC_ENOMEM;
  if (maxw) *maxw = widest;
  return overflow ? ORC_EOVERFLOW : ORC_OK;
}

int orc_x2_rows_f64(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
                    double tau, int32_t nr, const int32_t *rows, int32_t M2, int32_t *nnz2, int32_t *idx2,
                    double *val2, double *d2)
{
  for (int32_t q = 0; q < nr; ++q)
    if (rows[q] < 0 || rows[q] >= N) return ORC_EINVAL;
  int failed = 0, overflow = 0;
#pragma omp parallel reduction(| : failed, overflow)
  {
    double *acc = (double *)calloc((size_t)N, sizeof(double));
    char *mark = (char *)calloc((size_t)N, 1);
    int32_t *touched = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    const int ok = acc && mark && touched;
    if (!ok) failed = 1;
#pragma omp for schedule(dynamic)
    for (int32_t q = 0; q < nr; ++q) {
      if (!ok) continue;
      double xii, dii;
      const int32_t c = x2_row_f64(rows[q], M, nnz, idx, val, tau, M2, idx2 + (int64_t)q * M2,
                                   val2 + (int64_t)q * M2, acc, mark, touched, &xii, &dii);
      if (d2) d2[q] = dii;
      if (c > M2) { overflow = 1; nnz2[q] = M2; } else nnz2[q] = c;
    }
    free(acc); free(mark); free(touched);
  }
  if (failed) return ORC_ENOMEM;
  return overflow ? ORC_EOVERFLOW : ORC_OK;
}

int orc_x2_f32(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const float *val,
               float tau, int32_t M2, int32_t *nnz2, int32_t *idx2, float *val2,
               double *d1, double *d2, int32_t *maxw)
{
  int failed = 0, overflow = 0;
  int32_t widest = 0;
#pragma omp parallel reduction(| : failed, overflow) reduction(max : widest)
  {
    /* the dense accumulator of one row, its marks and touched columns */
    float *acc = (float *)calloc((size_t)N, sizeof(float));
    char *mark = (char *)calloc((size_t)N, 1);
    int32_t *touched = (int32_t *)malloc((size_t)N * sizeof(int32_t));
    const int ok = acc && mark && touched;
    if (!ok) failed = 1;
#pragma omp for schedule(static)
    for (int32_t i = 0; i < N; ++i) {
      if (!ok) continue;
      const int32_t *ci = idx + (int64_t)i * M;
      const float *vi = val + (int64_t)i * M;
      int32_t nt = 0;
      float xii = 0.0f;
      for (int32_t s = 0; s < nnz[i]; ++s) {
        int32_t k = ci[s];
        float a = vi[s];
        if (k == i) xii = a;
        const int32_t *ck = idx + (int64_t)k * M;
        const float *vk = val + (int64_t)k * M;
        for (int32_t t = 0; t < nnz[k]; ++t) {
          int32_t j = ck[t];
          if (!mark[j]) { mark[j] = 1; touched[nt++] = j; }
          acc[j] = fmaf(a, vk[t], acc[j]);
        }
      }
      if (d1) d1[i] = (double)xii;
      if (d2) d2[i] = (double)acc[i];
      qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
      int32_t c = 0;
      for (int32_t q = 0; q < nt; ++q) {
        int32_t j = touched[q];
        if (fabsf(acc[j]) > tau) {
          if (c < M2) {
            idx2[(int64_t)i * M2 + c] = j;
            val2[(int64_t)i * M2 + c] = acc[j];
          }
          ++c;
        }
        acc[j] = 0.0f;
        mark[j] = 0;
      }
      if (c > M2) { overflow = 1; nnz2[i] = M2; } else nnz2[i] = c;
      if (c > widest) widest = c;
    }
    free(acc); free(mark); free(touched);
  }
  if (failed) return ORC_ENOMEM;
  if (maxw) *maxw = widest;
  return overflow ? ORC_EOVERFLOW : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* trace and idempotency norm                                               */
/* ------------------------------------------------------------------------ */
double orc_trace_f64(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val)
{
  double *d = (double *)malloc((size_t)N * sizeof(double));
  if (!d) return NAN;
  for (int32_t i = 0; i < N; ++i) {
    d[i] = 0.0;
    for (int32_t s = 0; s < nnz[i]; ++s)
      if (idx[(int64_t)i * M + s] == i) d[i] = val[(int64_t)i * M + s];
  }
  double t = orc_pairwise(N, d);
  free(d);
  return t;
}

/* Tr(AB) = sum_i sum_j A_ij B_ji (the energy Tr(DH) of the ExaSP2 output, in
 * the paper's "ExaSP2 Application" section).  Row term t_i: fused
 * multiply-adds t = fma(A_ij, B_ji, t) over the stored entries of row i of A
 * in ascending column j, B_ji taken from row j of B (skipped where B stores no
 * (j, i) entry); Tr(AB) = pairwise tree of the t_i. */
double orc_trace_product_f64(int32_t N, int32_t MA, const int32_t *nnzA, const int32_t *idxA, const double *valA,
                             int32_t MB, const int32_t *nnzB, const int32_t *idxB, const double *valB)
{
  double *t = (double *)malloc((size_t)N * sizeof(double));
  if (!t) return NAN;
  for (int32_t i = 0; i < N; ++i) {
    double acc = 0.0;
    for (int32_t s = 0; s < nnzA[i]; ++s) {
      const int32_t j = idxA[(int64_t)i * MA + s];
      for (int32_t u = 0; u < nnzB[j]; ++u)
        if (idxB[(int64_t)j * MB + u] == i) {
          acc = fma(valA[(int64_t)i * MA + s], valB[(int64_t)j * MB + u], acc);
          break;
        }
    }
    t[i] = acc;
  }
  const double r = orc_pairwise(N, t);
  free(t);
  return r;
}

/* Row term e_i: the pairwise tree over the row's N column positions of
 * q_j = d*d with d = X2_ij - X_ij (absent entries are 0, so q_j = +0 wherever
 * neither matrix stores column j); eta^2 = pairwise tree of the e_i.  The tree
 * over N leaves is the perfect tree over the next power of two with +0 leaves
 * past N (an odd element passing a level unchanged is the same as adding +0).
 * A subtree whose leaves are all +0 sums to +0 and adding +0 changes nothing,
 * so only the stored columns need visiting: tree_sum() walks the aligned
 * subtrees that contain one. */
static double tree_sum(const int32_t *col, const double *q, int32_t n, int64_t lo, int64_t size)
{
  /* entries with lo <= col < lo + size, col ascending */
  int32_t a = 0, b = n;
  while (a < b && col[a] < lo) ++a;
  int32_t e = a;
  while (e < b && col[e] < lo + size) ++e;
  if (a == e) return 0.0;
  if (size == 1) return q[a];
  const int64_t h = size / 2;
  return tree_sum(col + a, q + a, e - a, lo, h) + tree_sum(col + a, q + a, e - a, lo + h, h);
}

static int64_t pow2_at_least(int64_t n)
{
  int64_t p = 1;
  while (p < n) p *= 2;
  return p;
}

double orc_norm2_f64(int32_t N, int32_t MX, const int32_t *nnzX, const int32_t *idxX, const double *valX,
                     int32_t M2, const int32_t *nnz2, const int32_t *idx2, const double *val2, double *e)
{
  double *row = (double *)malloc((size_t)N * sizeof(double));
  double *q = (double *)malloc((size_t)(MX + M2 + 1) * sizeof(double));
  int32_t *c = (int32_t *)malloc((size_t)(MX + M2 + 1) * sizeof(int32_t));
  if (!row || !q || !c) { free(row); free(q); free(c); return NAN; }
  const int64_t P = pow2_at_least(N);
  for (int32_t i = 0; i < N; ++i) {
    const int32_t *cx = idxX + (int64_t)i * MX, *cy = idx2 + (int64_t)i * M2;
    const double *vx = valX + (int64_t)i * MX, *vy = val2 + (int64_t)i * M2;
    int32_t p = 0, r = 0, n = 0;
    while (p < nnzX[i] || r < nnz2[i]) {
      int32_t jx = p < nnzX[i] ? cx[p] : N;
      int32_t jy = r < nnz2[i] ? cy[r] : N;
      double x = 0.0, y = 0.0;
      c[n] = jx < jy ? jx : jy;
      if (jx <= jy) x = vx[p++];
      if (jy <= jx) y = vy[r++];
      double d = y - x;
      q[n++] = d * d;
    }
    row[i] = tree_sum(c, q, n, 0, P);
  }
  if (e) memcpy(e, row, (size_t)N * sizeof(double));
  double s = orc_pairwise(N, row);
  free(row);
  free(q);
  free(c);
  return s;
}

double orc_norm2_f32(int32_t N, int32_t MX, const int32_t *nnzX, const int32_t *idxX, const float *valX,
                     int32_t M2, const int32_t *nnz2, const int32_t *idx2, const float *val2, double *e)
{
  double *row = (double *)malloc((size_t)N * sizeof(double));
  double *q = (double *)malloc((size_t)(MX + M2 + 1) * sizeof(double));
  int32_t *c = (int32_t *)malloc((size_t)(MX + M2 + 1) * sizeof(int32_t));
  if (!row || !q || !c) { free(row); free(q); free(c); return NAN; }
  const int64_t P = pow2_at_least(N);
  for (int32_t i = 0; i < N; ++i) {
    const int32_t *cx = idxX + (int64_t)i * MX, *cy = idx2 + (int64_t)i * M2;
    const float *vx = valX + (int64_t)i * MX, *vy = val2 + (int64_t)i * M2;
    int32_t p = 0, r = 0, n = 0;
    while (p < nnzX[i] || r < nnz2[i]) {
      int32_t jx = p < nnzX[i] ? cx[p] : N;
      int32_t jy = r < nnz2[i] ? cy[r] : N;
      double x = 0.0, y = 0.0;
      c[n] = jx < jy ? jx : jy;
      if (jx <= jy) x = (double)vx[p++];
      if (jy <= jx) y = (double)vy[r++];
      double d = y - x;
      q[n++] = d * d;
    }
    row[i] = tree_sum(c, q, n, 0, P);
  }
  if (e) memcpy(e, row, (size_t)N * sizeof(double));
  double s = orc_pairwise(N, row);
  free(row);
  free(q);
  free(c);
  return s;
}

/* ------------------------------------------------------------------------ */
/* update X <- prune(2X - X^2)                                              */
/* ------------------------------------------------------------------------ */
int orc_update_f64(int32_t N, int32_t MX, const int32_t *nnzX, const int32_t *idxX, const double *valX,
                   int32_t M2, const int32_t *nnz2, const int32_t *idx2, const double *val2, double tau,
                   int32_t Mo, int32_t *nnzo, int32_t *idxo, double *valo, int32_t *maxw)
{
  int overflow = 0;
  int32_t widest = 0;
#pragma omp parallel for schedule(static) reduction(| : overflow) reduction(max : widest)
  for (int32_t i = 0; i < N; ++i) {
    const int32_t *cx = idxX + (int64_t)i * MX, *cy = idx2 + (int64_t)i * M2;
    const double *vx = valX + (int64_t)i * MX, *vy = val2 + (int64_t)i * M2;
    int32_t p = 0, q = 0, c = 0;
    while (p < nnzX[i] || q < nnz2[i]) {
      int32_t jx = p < nnzX[i] ? cx[p] : N;
      int32_t jy = q < nnz2[i] ? cy[q] : N;
      int32_t j = jx < jy ? jx : jy;
      double x = 0.0, y = 0.0;
      if (jx == j) x = vx[p++];
      if (jy == j) y = vy[q++];
      double v = 2.0 * x - y;
      if (fabs(v) > tau) {
        if (c < Mo) { idxo[(int64_t)i * Mo + c] = j; valo[(int64_t)i * Mo + c] = v; }
        ++c;
      }
    }
    if (c > Mo) { overflow = 1; nnzo[i] = Mo; } else nnzo[i] = c;
    if (c > widest) widest = c;
  }
  if (maxw) *maxw = widest;
  return overflow ? ORC_EOVERFLOW : ORC_OK;
}

int orc_update_f32(int32_t N, int32_t MX, const int32_t *nnzX, const int32_t *idxX, const float *valX,
                   int32_t M2, const int32_t *nnz2, const int32_t *idx2, const float *val2, float tau,
                   int32_t Mo, int32_t *nnzo, int32_t *idxo, float *valo, int32_t *maxw)
{
  int overflow = 0;
  int32_t widest = 0;
#pragma omp parallel for schedule(static) reduction(| : overflow) reduction(max : widest)
  for (int32_t i = 0; i < N; ++i) {
    const int32_t *cx = idxX + (int64_t)i * MX, *cy = idx2 + (int64_t)i * M2;
    const float *vx = valX + (int64_t)i * MX, *vy = val2 + (int64_t)i * M2;
    int32_t p = 0, q = 0, c = 0;
    while (p < nnzX[i] || q < nnz2[i]) {
      int32_t jx = p < nnzX[i] ? cx[p] : N;
      int32_t jy = q < nnz2[i] ? cy[q] : N;
      int32_t j = jx < jy ? jx : jy;
      float x = 0.0f, y = 0.0f;
      if (jx == j) x = vx[p++];
      if (jy == j) y = vy[q++];
      float v = 2.0f * x - y;
      if (fabsf(v) > tau) {
        if (c < Mo) { idxo[(int64_t)i * Mo + c] = j; valo[(int64_t)i * Mo + c] = v; }
        ++c;
      }
    }
    if (c > Mo) { overflow = 1; nnzo[i] = Mo; } else nnzo[i] = c;
    if (c > widest) widest = c;
  }
  if (maxw) *maxw = widest;
  return overflow ? ORC_EOVERFLOW : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* prune: keep |v| > tau (the single pruning of the one-pruning SP2 mode)    */
/* ------------------------------------------------------------------------ */
int orc_prune_f64(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val, double tau,
                  int32_t Mo, int32_t *nnzo, int32_t *idxo, double *valo, int32_t *maxw)
{
  int overflow = 0;
  int32_t widest = 0;
  for (int32_t i = 0; i < N; ++i) {
    int32_t c = 0;
    for (int32_t s = 0; s < nnz[i]; ++s) {
      const double v = val[(int64_t)i * M + s];
      if (fabs(v) > tau) {
        if (c < Mo) { idxo[(int64_t)i * Mo + c] = idx[(int64_t)i * M + s]; valo[(int64_t)i * Mo + c] = v; }
        ++c;
      }
    }
    if (c > Mo) { overflow = 1; nnzo[i] = Mo; } else nnzo[i] = c;
    if (c > widest) widest = c;
  }
  if (maxw) *maxw = widest;
  return overflow ? ORC_EOVERFLOW : ORC_OK;
}

int orc_prune_f32(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const float *val, float tau,
                  int32_t Mo, int32_t *nnzo, int32_t *idxo, float *valo, int32_t *maxw)
{
  int overflow = 0;
  int32_t widest = 0;
  for (int32_t i = 0; i < N; ++i) {
    int32_t c = 0;
    for (int32_t s = 0; s < nnz[i]; ++s) {
      const float v = val[(int64_t)i * M + s];
      if (fabsf(v) > tau) {
        if (c < Mo) { idxo[(int64_t)i * Mo + c] = idx[(int64_t)i * M + s]; valo[(int64_t)i * Mo + c] = v; }
        ++c;
      }
    }
    if (c > Mo) { overflow = 1; nnzo[i] = Mo; } else nnzo[i] = c;
    if (c > widest) widest = c;
  }
  if (maxw) *maxw = widest;
  return overflow ? ORC_EOVERFLOW : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Gershgorin bounds and the initial guess X0                               */
/* ------------------------------------------------------------------------ */
int orc_gershgorin(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
                   double *emin, double *emax)
{
  double lo = INFINITY, hi = -INFINITY;
  for (int32_t i = 0; i < N; ++i) {
    double r = 0.0, hii = 0.0;
    for (int32_t s = 0; s < nnz[i]; ++s) {
      int32_t j = idx[(int64_t)i * M + s];
      double h = val[(int64_t)i * M + s];
      if (!isfinite(h)) return ORC_ENONFINITE;
      if (j == i) hii = h; else r = r + fabs(h);
    }
    double a = hii - r, b = hii + r;
    if (a < lo) lo = a;
    if (b > hi) hi = b;
  }
  *emin = lo;
  *emax = hi;
  return ORC_OK;
}

/* one row of X0 in FP64, diagonal inserted if absent; returns the surviving count */
static int32_t x0_row(int32_t i, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
                      double emax, double inv, int32_t *cols, double *vals)
{
  const int32_t *ci = idx + (int64_t)i * M;
  const double *vi = val + (int64_t)i * M;
  int32_t c = 0, s = 0, diag_done = 0;
  while (s < nnz[i] || !diag_done) {
    int32_t j;
    double h;
    if (s < nnz[i] && (diag_done || ci[s] <= i)) {
      j = ci[s];
      h = vi[s];
      ++s;
    } else {
      j = i;
      h = 0.0;
    }
    if (j == i) diag_done = 1;
    double x = (j == i) ? (emax - h) * inv : (-h) * inv;
    cols[c] = j;
    vals[c] = x;
    ++c;
  }
  return c;
}

int orc_x0_f64(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
               double emin, double emax, double tau,
               int32_t Mo, int32_t *nnzo, int32_t *idxo, double *valo, int32_t *maxw)
{
  double inv = 1.0 / (emax - emin);
  int32_t *cols = (int32_t *)malloc((size_t)(M + 1) * sizeof(int32_t));
  double *vals = (double *)malloc((size_t)(M + 1) * sizeof(double));
  if (!cols || !vals) { free(cols); free(vals); return ORC_ENOMEM; }
  int status = ORC_OK;
  int32_t widest = 0;
  for (int32_t i = 0; i < N; ++i) {
    int32_t n = x0_row(i, M, nnz, idx, val, emax, inv, cols, vals);
    int32_t c = 0;
    for (int32_t q = 0; q < n; ++q) {
      if (fabs(vals[q]) > tau) {
        if (c < Mo) { idxo[(int64_t)i * Mo + c] = cols[q]; valo[(int64_t)i * Mo + c] = vals[q]; }
        ++c;
      }
    }
    if (c > Mo) { status = ORC_EOVERFLOW; nnzo[i] = Mo; } else nnzo[i] = c;
    if (c > widest) widest = c;
  }
  if (maxw) *maxw = widest;
  free(cols); free(vals);
  return status;
}

int orc_x0_f32(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
               double emin, double emax, float tau,
               int32_t Mo, int32_t *nnzo, int32_t *idxo, float *valo, int32_t *maxw)
{
  double inv = 1.0 / (emax - emin);
  int32_t *cols = (int32_t *)malloc((size_t)(M + 1) * sizeof(int32_t));
  double *vals = (double *)malloc((size_t)(M + 1) * sizeof(double));
  if (!cols || !vals) { free(cols); free(vals); return ORC_ENOMEM; }
  int status = ORC_OK;
  int32_t widest = 0;
  for (int32_t i = 0; i < N; ++i) {
    int32_t n = x0_row(i, M, nnz, idx, val, emax, inv, cols, vals);
    int32_t c = 0;
    for (int32_t q = 0; q < n; ++q) {
      float xf = (float)vals[q];
      if (fabsf(xf) > tau) {
        if (c < Mo) { idxo[(int64_t)i * Mo + c] = cols[q]; valo[(int64_t)i * Mo + c] = xf; }
        ++c;
      }
    }
    if (c > Mo) { status = ORC_EOVERFLOW; nnzo[i] = Mo; } else nnzo[i] = c;
    if (c > widest) widest = c;
  }
  if (maxw) *maxw = widest;
  free(cols); free(vals);
  return status;
}

/* ------------------------------------------------------------------------ */
/* SP2 driver                                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t N, M;
  int32_t *nnz, *idx;
  double *v;  /* FP64 values, or NULL */
  float *f;   /* FP32 values, or NULL */
} omat;

static void omat_free(omat *a)
{
  free(a->nnz); free(a->idx); free(a->v); free(a->f);
  memset(a, 0, sizeof(*a));
}

static int omat_alloc(omat *a, int32_t N, int32_t M, int fp32)
{
  omat_free(a);
  a->N = N;
  a->M = M;
  a->nnz = (int32_t *)calloc((size_t)N, sizeof(int32_t));
  a->idx = (int32_t *)calloc((size_t)N * M, sizeof(int32_t));
  if (fp32) a->f = (float *)calloc((size_t)N * M, sizeof(float));
  else a->v = (double *)calloc((size_t)N * M, sizeof(double));
  if (!a->nnz || !a->idx || (!a->f && !a->v)) { omat_free(a); return ORC_ENOMEM; }
  return ORC_OK;
}

static int32_t roundup32(int32_t x) { return (x + 31) / 32 * 32; }

/* Stall rule on the phase-local eta^2 history h[0..n]: once eta has gone below
 * 1e-2, stop when the best of the last two steps is no better than the best of
 * the two steps before them. */
static int stalled(const double *h, int32_t n)
{
  if (n < 3) return 0;
  if (!(h[n - 3] < 1e-4)) return 0;
  double now = h[n] < h[n - 1] ? h[n] : h[n - 1];
  double before = h[n - 2] < h[n - 3] ? h[n - 2] : h[n - 3];
  return now >= before;
}

static int sp2_x2_grow(omat *X, omat *Y, double tau, float tau32, double *d1, double *d2, int32_t *maxw)
{
  for (;;) {
    int rc;
    if (X->f)
      rc = orc_x2_f32(X->N, X->M, X->nnz, X->idx, X->f, tau32, Y->M, Y->nnz, Y->idx, Y->f, d1, d2, maxw);
    else
      rc = orc_x2_f64(X->N, X->M, X->nnz, X->idx, X->v, tau, Y->M, Y->nnz, Y->idx, Y->v, d1, d2, maxw);
    if (rc != ORC_EOVERFLOW) return rc;
    rc = omat_alloc(Y, X->N, roundup32(*maxw), X->f != NULL);
    if (rc) return rc;
  }
}

static int sp2_update_grow(omat *X, const omat *Y, omat *T, double tau, float tau32)
{
  for (;;) {
    int32_t w = 0;
    int rc;
    if (X->f)
      rc = orc_update_f32(X->N, X->M, X->nnz, X->idx, X->f, Y->M, Y->nnz, Y->idx, Y->f, tau32,
                          T->M, T->nnz, T->idx, T->f, &w);
    else
      rc = orc_update_f64(X->N, X->M, X->nnz, X->idx, X->v, Y->M, Y->nnz, Y->idx, Y->v, tau,
                          T->M, T->nnz, T->idx, T->v, &w);
    if (rc != ORC_EOVERFLOW) return rc;
    rc = omat_alloc(T, X->N, roundup32(w), X->f != NULL);
    if (rc) return rc;
  }
}

static int sp2_prune_grow(const omat *Y, omat *P, double tau, float tau32, int32_t *maxw)
{
  for (;;) {
    int rc;
    if (Y->f)
      rc = orc_prune_f32(Y->N, Y->M, Y->nnz, Y->idx, Y->f, tau32, P->M, P->nnz, P->idx, P->f, maxw);
    else
      rc = orc_prune_f64(Y->N, Y->M, Y->nnz, Y->idx, Y->v, tau, P->M, P->nnz, P->idx, P->v, maxw);
    if (rc != ORC_EOVERFLOW) return rc;
    rc = omat_alloc(P, Y->N, roundup32(*maxw), Y->f != NULL);
    if (rc) return rc;
  }
}

static void omat_swap(omat *a, omat *b) { omat t = *a; *a = *b; *b = t; }

/* widen an FP32 matrix to FP64 (exact) */
static int omat_widen(omat *X)
{
  double *v = (double *)calloc((size_t)X->N * X->M, sizeof(double));
  if (!v) return ORC_ENOMEM;
  for (int64_t q = 0; q < (int64_t)X->N * X->M; ++q) v[q] = (double)X->f[q];
  free(X->f);
  X->f = NULL;
  X->v = v;
  return ORC_OK;
}

int orc_sp2(int32_t N, int32_t M, const int32_t *nnz, const int32_t *idx, const double *val,
            const orc_sp2_params *p, int32_t Mo, int32_t *nnzD, int32_t *idxD, double *valD,
            orc_sp2_report *r)
{
  int rc = orc_check_ell(N, M, nnz, idx);
  if (rc) return rc;
  if (!(p->tau >= 0.0) || p->max_iter <= 0 || !(p->idem_target >= 0.0)) return ORC_EINVAL;
  if (p->precision == ORC_PREC_MIXED && !(p->tau_fp32 >= 0.0)) return ORC_EINVAL;
  rc = orc_check_finite_f64(N, M, nnz, val);
  if (rc) return rc;
  double emin, emax;
  rc = orc_gershgorin(N, M, nnz, idx, val, &emin, &emax);
  if (rc) return rc;
  r->emin = emin;
  r->emax = emax;
  if (!(emax > emin)) return ORC_EDEGENERATE;
  if (!(p->n_occ > 0.0 && p->n_occ < (double)N)) return ORC_EDEGENERATE;

  int mixed = p->precision == ORC_PREC_MIXED;
  float tau32 = (float)p->tau_fp32;
  double target2 = p->idem_target * p->idem_target;
  double switch2 = p->switch_eta * p->switch_eta;

  const int once = p->prune_once != 0;
  omat X = {0}, Y = {0}, T = {0}, P = {0};
  double *d1 = (double *)malloc((size_t)N * sizeof(double));
  double *d2 = (double *)malloc((size_t)N * sizeof(double));
  double *hist = (double *)malloc((size_t)p->max_iter * sizeof(double));
  if (!d1 || !d2 || !hist) { rc = ORC_ENOMEM; goto done; }

  /* X0 */
  {
    int32_t cap = M + 1, w = 0;
    for (;;) {
      rc = omat_alloc(&X, N, cap, mixed);
      if (rc) goto done;
      if (mixed)
        rc = orc_x0_f32(N, M, nnz, idx, val, emin, emax, tau32, X.M, X.nnz, X.idx, X.f, &w);
      else
        rc = orc_x0_f64(N, M, nnz, idx, val, emin, emax, p->tau, X.M, X.nnz, X.idx, X.v, &w);
      if (rc != ORC_EOVERFLOW) break;
      cap = roundup32(w);
    }
    if (rc) goto done;
  }
  rc = omat_alloc(&Y, N, X.M, mixed);
  if (rc) goto done;
  rc = omat_alloc(&T, N, X.M, mixed);
  if (rc) goto done;

  int32_t phase_start = 0, fp32_iters = 0, fp64_updates = 0;
  int32_t n;
  int final_status = ORC_ENOCONV;
  double eta2 = NAN, trx = NAN;
  for (n = 0; n < p->max_iter; ++n) {
    int32_t maxw = 0;
    int in32 = X.f != NULL;
    if (once) {
      /* Y = X.X unpruned (every nonzero entry); P = prune(Y), the X^2 branch's iterate */
      rc = sp2_x2_grow(&X, &Y, 0.0, 0.0f, d1, d2, &maxw);
      if (rc) goto done;
      if (P.M == 0 || (P.f != NULL) != in32) {
        omat_free(&P);
        rc = omat_alloc(&P, N, X.M, in32);
        if (rc) goto done;
      }
      rc = sp2_prune_grow(&Y, &P, p->tau, tau32, &maxw);
    } else {
      rc = sp2_x2_grow(&X, &Y, p->tau, tau32, d1, d2, &maxw);
    }
    if (rc) goto done;
    trx = orc_pairwise(N, d1);
    double trx2 = orc_pairwise(N, d2);
    if (in32)
      eta2 = orc_norm2_f32(N, X.M, X.nnz, X.idx, X.f, Y.M, Y.nnz, Y.idx, Y.f, NULL);
    else
      eta2 = orc_norm2_f64(N, X.M, X.nnz, X.idx, X.v, Y.M, Y.nnz, Y.idx, Y.v, NULL);
    hist[n] = eta2;
    if (r->hist_trx) r->hist_trx[n] = trx;
    if (r->hist_trx2) r->hist_trx2[n] = trx2;
    if (r->hist_eta2) r->hist_eta2[n] = eta2;
    if (r->hist_maxw) r->hist_maxw[n] = maxw;
    if (r->hist_prec) r->hist_prec[n] = (int8_t)in32;
    if (r->hist_up) r->hist_up[n] = -1;
    if (in32) ++fp32_iters;

    int stall = p->stall_stop && stalled(hist + phase_start, n - phase_start);
    if (in32) {
      if (eta2 < switch2 || stall) {
        /* switch: widen X, then continue in FP64 from this same X */
        rc = omat_widen(&X);
        if (rc) goto done;
        omat_free(&Y);
        omat_free(&T);
        rc = omat_alloc(&Y, N, X.M, 0);
        if (!rc) rc = omat_alloc(&T, N, X.M, 0);
        if (rc) goto done;
        phase_start = n + 1;
        if (n + 1 == p->max_iter) { final_status = ORC_ENOCONV; ++n; break; }
        continue; /* the FP64 phase recomputes X^2 of the widened X */
      }
    } else {
      if (eta2 < target2 && fp64_updates >= (mixed ? p->fp64_tail_steps : 0)) {
        final_status = ORC_OK;
        ++n;
        break;
      }
      if (stall) { final_status = ORC_ENOCONV; ++n; break; }
    }
    if (n + 1 == p->max_iter) { final_status = ORC_ENOCONV; ++n; break; }

    double a = fabs(2.0 * trx - trx2 - p->n_occ);
    double b = fabs(trx2 - p->n_occ);
    int up = a < b;
    if (r->hist_up) r->hist_up[n] = (int8_t)up;
    if (up) {
      rc = sp2_update_grow(&X, &Y, &T, p->tau, tau32);  /* once: Y unpruned, one pruning */
      if (rc) goto done;
      omat_swap(&X, &T);
    } else {
      omat_swap(&X, once ? &P : &Y);
    }
    if (!in32) ++fp64_updates;
    /* keep the scratch matrices at least as wide as X */
    if (Y.M < X.M) { rc = omat_alloc(&Y, N, X.M, X.f != NULL); if (rc) goto done; }
    if (T.M < X.M) { rc = omat_alloc(&T, N, X.M, X.f != NULL); if (rc) goto done; }
  }

  r->iterations = n;
  r->fp32_iterations = fp32_iters;
  r->eta = sqrt(eta2);
  r->trace_x = trx;
  if (X.f) { rc = omat_widen(&X); if (rc) goto done; }
  {
    int32_t w = 0;
    for (int32_t i = 0; i < N; ++i) if (X.nnz[i] > w) w = X.nnz[i];
    r->final_M = w;
    if (w > Mo) { rc = ORC_EOVERFLOW; goto done; }
    for (int32_t i = 0; i < N; ++i) {
      nnzD[i] = X.nnz[i];
      for (int32_t s = 0; s < X.nnz[i]; ++s) {
        idxD[(int64_t)i * Mo + s] = X.idx[(int64_t)i * X.M + s];
        valD[(int64_t)i * Mo + s] = X.v[(int64_t)i * X.M + s];
      }
    }
  }
  rc = final_status;
done:
  r->status = rc;
  omat_free(&X); omat_free(&Y); omat_free(&T); omat_free(&P);
  free(d1); free(d2); free(hist);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* dense variant                                                            */
/* ------------------------------------------------------------------------ */
void orc_dense_x2_f64(int32_t N, const double *A, double *C)
{
  for (int64_t q = 0; q < (int64_t)N * N; ++q) C[q] = 0.0;
  for (int32_t i = 0; i < N; ++i)
    for (int32_t k = 0; k < N; ++k) {
      double a = A[(int64_t)i * N + k];
      const double *bk = A + (int64_t)k * N;
      double *ci = C + (int64_t)i * N;
      for (int32_t j = 0; j < N; ++j) ci[j] = fma(a, bk[j], ci[j]);
    }
}

float orc_bf16_rne(float x)
{
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) {          /* inf / nan: truncate, keep nan quiet */
    if (u & 0x007fffffu) u |= 0x00400000u;
    u &= 0xffff0000u;
  } else {
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
  }
  float y;
  memcpy(&y, &u, 4);
  return y;
}

void orc_dense_x2_bf16x3(int32_t N, const float *A, float *C)
{
  int64_t nn = (int64_t)N * N;
  float *hi = (float *)malloc((size_t)nn * sizeof(float));
  float *lo = (float *)malloc((size_t)nn * sizeof(float));
  if (!hi || !lo) { free(hi); free(lo); return; }
  for (int64_t q = 0; q < nn; ++q) {
    hi[q] = orc_bf16_rne(A[q]);
    lo[q] = orc_bf16_rne(A[q] - hi[q]);
  }
  for (int64_t q = 0; q < nn; ++q) C[q] = 0.0f;
  for (int32_t i = 0; i < N; ++i)
    for (int32_t k = 0; k < N; ++k) {
      float ah = hi[(int64_t)i * N + k], al = lo[(int64_t)i * N + k];
      const float *bh = hi + (int64_t)k * N, *bl = lo + (int64_t)k * N;
      float *ci = C + (int64_t)i * N;
      for (int32_t j = 0; j < N; ++j) {
        float c = ci[j];
        c = fmaf(ah, bh[j], c);
        c = fmaf(ah, bl[j], c);
        c = fmaf(al, bh[j], c);
        ci[j] = c;
      }
    }
  free(hi); free(lo);
}

/* dense traces: diagonal by pairwise tree */
static double dense_trace(int32_t N, const double *A, double *scratch)
{
  for (int32_t i = 0; i < N; ++i) scratch[i] = A[(int64_t)i * N + i];
  return orc_pairwise(N, scratch);
}

/* dense norm: every entry of the row is in the pattern; same trees as the sparse norm */
static double dense_norm2(int32_t N, const double *X, const double *Y, double *scratch, double *q)
{
  for (int32_t i = 0; i < N; ++i) {
    for (int32_t j = 0; j < N; ++j) {
      double d = Y[(int64_t)i * N + j] - X[(int64_t)i * N + j];
      q[j] = d * d;
    }
    scratch[i] = orc_pairwise(N, q);
  }
  return orc_pairwise(N, scratch);
}

int orc_dense_sp2(int32_t N, const double *H, int32_t mode, const orc_sp2_params *p,
                  double *D, orc_sp2_report *r)
{
  if (N <= 0 || p->max_iter <= 0) return ORC_EINVAL;
  int64_t nn = (int64_t)N * N;
  for (int64_t q = 0; q < nn; ++q) if (!isfinite(H[q])) return ORC_ENONFINITE;
  /* Gershgorin on the dense matrix, row sums in ascending j */
  double emin = INFINITY, emax = -INFINITY;
  for (int32_t i = 0; i < N; ++i) {
    double rsum = 0.0;
    for (int32_t j = 0; j < N; ++j) if (j != i) rsum = rsum + fabs(H[(int64_t)i * N + j]);
    double hii = H[(int64_t)i * N + i];
    if (hii - rsum < emin) emin = hii - rsum;
    if (hii + rsum > emax) emax = hii + rsum;
  }
  r->emin = emin;
  r->emax = emax;
  if (!(emax > emin)) return ORC_EDEGENERATE;
  if (!(p->n_occ > 0.0 && p->n_occ < (double)N)) return ORC_EDEGENERATE;
  double inv = 1.0 / (emax - emin);

  int lowp = mode == ORC_DENSE_BF16X3;
  double *X = (double *)malloc((size_t)nn * sizeof(double));
  double *Y = (double *)malloc((size_t)nn * sizeof(double));
  float *Xf = (float *)malloc((size_t)nn * sizeof(float));
  float *Yf = (float *)malloc((size_t)nn * sizeof(float));
  double *scr = (double *)malloc((size_t)N * sizeof(double));
  double *qrow = (double *)malloc((size_t)N * sizeof(double));
  double *hist = (double *)malloc((size_t)p->max_iter * sizeof(double));
  int rc = ORC_OK;
  if (!X || !Y || !Xf || !Yf || !scr || !qrow || !hist) { rc = ORC_ENOMEM; goto done; }
  for (int32_t i = 0; i < N; ++i)
    for (int32_t j = 0; j < N; ++j) {
      double h = H[(int64_t)i * N + j];
      X[(int64_t)i * N + j] = (j == i) ? (emax - h) * inv : (-h) * inv;
    }
  if (lowp) for (int64_t q = 0; q < nn; ++q) Xf[q] = (float)X[q];

  double target2 = p->idem_target * p->idem_target;
  double switch2 = p->switch_eta * p->switch_eta;
  int32_t phase_start = 0, lp_iters = 0, fp64_updates = 0, n;
  int final_status = ORC_ENOCONV;
  double eta2 = NAN, trx = NAN;
  for (n = 0; n < p->max_iter; ++n) {
    int inlp = lowp;
    if (inlp) {
      orc_dense_x2_bf16x3(N, Xf, Yf);
      for (int64_t q = 0; q < nn; ++q) { X[q] = (double)Xf[q]; Y[q] = (double)Yf[q]; }
      ++lp_iters;
    } else {
      orc_dense_x2_f64(N, X, Y);
    }
    trx = dense_trace(N, X, scr);
    double trx2 = dense_trace(N, Y, scr);
    eta2 = dense_norm2(N, X, Y, scr, qrow);
    hist[n] = eta2;
    if (r->hist_trx) r->hist_trx[n] = trx;
    if (r->hist_trx2) r->hist_trx2[n] = trx2;
    if (r->hist_eta2) r->hist_eta2[n] = eta2;
    if (r->hist_maxw) r->hist_maxw[n] = N;
    if (r->hist_prec) r->hist_prec[n] = (int8_t)inlp;
    if (r->hist_up) r->hist_up[n] = -1;
    int stall = p->stall_stop && stalled(hist + phase_start, n - phase_start);
    if (inlp) {
      if (eta2 < switch2 || stall) {
        lowp = 0;           /* X already holds the widened values */
        phase_start = n + 1;
        if (n + 1 == p->max_iter) { ++n; break; }
        continue;
      }
    } else {
      if (eta2 < target2 && fp64_updates >= (mode == ORC_DENSE_BF16X3 ? p->fp64_tail_steps : 0)) {
        final_status = ORC_OK;
        ++n;
        break;
      }
      if (stall) { ++n; break; }
    }
    if (n + 1 == p->max_iter) { ++n; break; }
    double a = fabs(2.0 * trx - trx2 - p->n_occ);
    double b = fabs(trx2 - p->n_occ);
    int up = a < b;
    if (r->hist_up) r->hist_up[n] = (int8_t)up;
    if (inlp) {
      for (int64_t q = 0; q < nn; ++q) Xf[q] = up ? 2.0f * Xf[q] - Yf[q] : Yf[q];
    } else {
      for (int64_t q = 0; q < nn; ++q) X[q] = up ? 2.0 * X[q] - Y[q] : Y[q];
      ++fp64_updates;
    }
  }
  r->iterations = n;
  r->fp32_iterations = lp_iters;
  r->final_M = N;
  r->eta = sqrt(eta2);
  r->trace_x = trx;
  memcpy(D, X, (size_t)nn * sizeof(double));
  rc = final_status;
done:
  r->status = rc;
  free(X); free(Y); free(Xf); free(Yf); free(scr); free(qrow); free(hist);
  return rc;
}

/* Test program (CPU only): runs every entry point of the C oracle on small
 * matrices -- m = 0, nnz = 0, ragged rows with empty ones, a dense row --
 * with 1 and 3 threads, under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built by tests/test_oracle_sanitize.py).  Integer-valued inputs, so the
 * four functions must agree exactly.  Prints "ok" and returns 0. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_spmv_dot2(int64_t, const int32_t *, const int32_t *, const double *, const double *, double *, int);
int oracle_spmv_naive(int64_t, const int32_t *, const int32_t *, const double *, const double *, double *);
int oracle_spmv_rowblock(int64_t, const int32_t *, const int32_t *, const double *, const double *, double *, int);
int oracle_abs_spmv(int64_t, const int32_t *, const int32_t *, const double *, const double *, double *, int);

static int check(int64_t m, int64_t n, const int32_t *rp, const int32_t *col, const double *val, const double *x) {
  /* exact arrays of the sizes the definition reads, so any overrun is caught */
  double *y1 = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  double *y2 = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  double *y3 = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  double *ya = malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  int bad = 0;
  for (int t = 1; t <= 3; t += 2) {
    if (oracle_spmv_dot2(m, rp, col, val, x, y1, t) || oracle_spmv_naive(m, rp, col, val, x, y2) ||
        oracle_spmv_rowblock(m, rp, col, val, x, y3, t) || oracle_abs_spmv(m, rp, col, val, x, ya, t))
      bad = 1;
    for (int64_t i = 0; i < m; ++i) {
      double s = 0.0, a = 0.0;
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
        s += val[k] * x[col[k]];
        a += fabs(val[k] * x[col[k]]);
      }
      if (y1[i] != s || y2[i] != s || y3[i] != s || ya[i] != a) bad = 1;
    }
  }
  (void)n;
  free(y1); free(y2); free(y3); free(ya);
  return bad;
}

int main(void) {
  int bad = 0;
  /* m = 0 */
  int32_t rp0[1] = {0};
  bad |= check(0, 3, rp0, NULL, NULL, NULL);
  /* nnz = 0, five empty rows */
  int32_t rp1[6] = {0, 0, 0, 0, 0, 0};
  double x1[2] = {1.0, 2.0};
  bad |= check(5, 2, rp1, NULL, NULL, x1);
  /* ragged rows with empty ones, and a dense row */
  enum { M = 2000, N = 300 };
  int32_t *rp = malloc(sizeof(int32_t) * (M + 1));
  rp[0] = 0;
  for (int i = 0; i < M; ++i) rp[i + 1] = rp[i] + (i == 777 ? N : (i % 3 == 0 ? 0 : (i * 7) % 13));
  const int32_t nnz = rp[M];
  int32_t *col = malloc(sizeof(int32_t) * (size_t)nnz);
  double *val = malloc(sizeof(double) * (size_t)nnz);
  double *x = malloc(sizeof(double) * N);
  for (int i = 0; i < M; ++i)
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      col[k] = (int32_t)((k - rp[i]) * 7 % N);
      val[k] = (double)((k * 5) % 7 - 3);
    }
  for (int j = 0; j < N; ++j) x[j] = (double)(j % 7 - 3);
  bad |= check(M, N, rp, col, val, x);
  /* invalid sizes are rejected */
  double y[1];
  if (oracle_spmv_dot2(-1, rp, col, val, x, y, 1) != -1) bad = 1;
  if (oracle_spmv_dot2(3, NULL, col, val, x, y, 1) != -1) bad = 1;
  free(rp); free(col); free(val); free(x);
  if (bad) {
    printf("mismatch\n");
    return 1;
  }
  printf("ok\n");
  return 0;
}

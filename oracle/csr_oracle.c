/*
 * CPU oracle for CSR sparse matrix-vector multiply, y = A x.
 *
 * TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the CPU-baseline leg of
 * the benchmark call this; the GPU library never links or calls it, and it
 * shares no code with the GPU path.
 *
 * What it computes is the plain definition of SpMV over CSR (Section 1 states
 * the problem; Section 2.1 defines the three CSR arrays and works the 6x6
 * example): for every row i,
 *     y[i] = sum_{k = row_ptr[i]}^{row_ptr[i+1]-1} val[k] * x[col[k]],
 * with an empty row giving 0.
 *
 * oracle_spmv_dot2 evaluates each row with the compensated dot product "Dot2"
 * of Ogita, Rump and Oishi (Accurate sum and dot product, SIAM J. Sci. Comput.
 * 26(6), 2005): error-free TwoProduct (via fma) and TwoSum (Knuth) transforms,
 * accumulating the rounding errors separately.  The result is as accurate as
 * if computed in twice the working precision and then rounded, so it serves as
 * the reference for every floating-point comparison.
 *
 * oracle_spmv_naive (single thread) and oracle_spmv_rowblock (OpenMP row
 * blocks) are the paper's CPU comparators (Section 4.3): a single-threaded
 * naive loop and the OpenMP-parallel basic row block method.
 *
 * oracle_abs_spmv computes (|A| |x|)_i = sum |val[k] * x[col[k]]|, the scale of
 * the rounding-error bound used for tolerances.
 *
 * Build with -ffp-contract=off: the error-free transforms must not be fused.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline void two_sum(double a, double b, double *s, double *e) {
  double x = a + b;
  double z = x - a;
  *e = (a - (x - z)) + (b - z);
  *s = x;
}

static inline void two_prod(double a, double b, double *p, double *e) {
  double x = a * b;
  *e = fma(a, b, -x);
  *p = x;
}

static double dot2_row(int64_t lo, int64_t hi, const int32_t *col,
                       const double *val, const double *x) {
  if (lo >= hi) return 0.0;
  double p, s;
  two_prod(val[lo], x[col[lo]], &p, &s);
  for (int64_t k = lo + 1; k < hi; ++k) {
    double h, r, q;
    two_prod(val[k], x[col[k]], &h, &r);
    two_sum(p, h, &p, &q);
    s = s + (q + r);
  }
  return p + s;
}

/* Returns 0 on success, -1 on invalid arguments. */
int oracle_spmv_dot2(int64_t m, const int32_t *row_ptr, const int32_t *col,
                     const double *val, const double *x, double *y,
                     int nthreads) {
  if (m < 0) return -1;
  if (m == 0) return 0;
  if (!row_ptr || !y) return -1;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1024) num_threads(nthreads)
#endif
  for (int64_t i = 0; i < m; ++i)
    y[i] = dot2_row(row_ptr[i], row_ptr[i + 1], col, val, x);
  return 0;
}

int oracle_spmv_naive(int64_t m, const int32_t *row_ptr, const int32_t *col,
                      const double *val, const double *x, double *y) {
  if (m < 0) return -1;
  for (int64_t i = 0; i < m; ++i) {
    double s = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += val[k] * x[col[k]];
    y[i] = s;
  }
  return 0;
}

int oracle_spmv_rowblock(int64_t m, const int32_t *row_ptr, const int32_t *col,
                         const double *val, const double *x, double *y,
                         int nthreads) {
  if (m < 0) return -1;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
  for (int64_t i = 0; i < m; ++i) {
    double s = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += val[k] * x[col[k]];
    y[i] = s;
  }
  return 0;
}

int oracle_abs_spmv(int64_t m, const int32_t *row_ptr, const int32_t *col,
                    const double *val, const double *x, double *y,
                    int nthreads) {
  if (m < 0) return -1;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1024) num_threads(nthreads)
#endif
  for (int64_t i = 0; i < m; ++i) {
    double s = 0.0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) s += fabs(val[k] * x[col[k]]);
    y[i] = s;
  }
  return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

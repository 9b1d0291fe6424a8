/*
 * CPU oracle for C = A * B on CSR matrices.  TEST INFRASTRUCTURE ONLY: the
 * tests, the smoke check and the CPU-baseline leg of the benchmark may call
 * it; the product path never does.  It shares no code with the GPU library.
 *
 * It is the plain definition of the product, written out: Gustavson's
 * row-wise formulation (paper, Section III-A): row i of C is the sum over the
 * nonzeros A[i,k] of A[i,k] times row k of B.  Accumulation is in FP64 with a
 * dense accumulator per thread; the product of two FP32 numbers is exact in
 * FP64.  Next to every value it returns the bound sum |A[i,k]| |B[k,j]|,
 * which the parity tests scale by the FP32 tolerance.
 *
 * Structure is the boolean product of the stored patterns: a column appears
 * in row i of C as soon as one product lands there, whatever its value, so
 * entries that cancel to zero are kept.  Rows are emitted in ascending column
 * order, the order compressed-row storage requires (paper, Section III-D,
 * column index sorting).
 *
 * The intermediate-product count of a row (paper, Algorithm 1) is the sum of
 * the lengths of the rows of B named by the columns of row i of A.
 *
 * Plain C99 + OpenMP; rows are independent, so threads take rows
 * dynamically.  Pinned by the pytest suite against dense FP64 products,
 * scipy's boolean product, identity / permutation special cases and the
 * closed form sum_k indeg_A(k) * len_B(k).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Algorithm 1: intermediate products per row, rows 0 .. m-1. */
int oracle_ip(int64_t m, const int64_t *rptA, const int32_t *colA,
              const int64_t *rptB, int64_t *ip_out)
{
    int64_t i;
#pragma omp parallel for schedule(dynamic, 1024)
    for (i = 0; i < m; ++i) {
        int64_t count = 0;
        for (int64_t j = rptA[i]; j < rptA[i + 1]; ++j) {
            int32_t col = colA[j];
            count += rptB[col + 1] - rptB[col];
        }
        ip_out[i] = count;
    }
    return 0;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Number of distinct columns in each selected row of C (the row's output
 * length).  rows == NULL selects rows 0 .. nsel-1.
 */
int oracle_row_counts(int64_t n, const int64_t *rptA, const int32_t *colA,
                      const int64_t *rptB, const int32_t *colB,
                      int64_t nsel, const int64_t *rows, int64_t *count_out)
{
    int failed = 0;
#pragma omp parallel
    {
        int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
        if (!mark) {
#pragma omp atomic write
            failed = 1;
        } else {
            for (int64_t c = 0; c < n; ++c) mark[c] = -1;
            int64_t s;
#pragma omp for schedule(dynamic, 64)
            for (s = 0; s < nsel; ++s) {
                int64_t i = rows ? rows[s] : s;
                int64_t distinct = 0;
                for (int64_t j = rptA[i]; j < rptA[i + 1]; ++j) {
                    int32_t k = colA[j];
                    for (int64_t t = rptB[k]; t < rptB[k + 1]; ++t) {
                        int32_t c = colB[t];
                        if (mark[c] != s) { mark[c] = s; ++distinct; }
                    }
                }
                count_out[s] = distinct;
            }
            free(mark);
        }
    }
    return failed ? -1 : 0;
}

/*
 * Values of the selected rows.  out_rpt[s] .. out_rpt[s+1] is where row s
 * goes (the caller sizes it from oracle_row_counts).  Writes sorted columns,
 * the FP64 sum and the FP64 absolute bound.  Returns -2 if a row's distinct
 * count disagrees with the space given to it.
 */
int oracle_row_values(int64_t n, const int64_t *rptA, const int32_t *colA,
                      const float *valA, const int64_t *rptB,
                      const int32_t *colB, const float *valB,
                      int64_t nsel, const int64_t *rows, const int64_t *out_rpt,
                      int32_t *out_col, double *out_val, double *out_abs)
{
    int failed = 0;
#pragma omp parallel
    {
        size_t nn = (size_t)(n > 0 ? n : 1);
        int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * nn);
        double *acc = (double *)malloc(sizeof(double) * nn);
        double *absacc = (double *)malloc(sizeof(double) * nn);
        int32_t *list = (int32_t *)malloc(sizeof(int32_t) * nn);
        if (!mark || !acc || !absacc || !list) {
#pragma omp atomic write
            failed = -1;
        } else {
            for (int64_t c = 0; c < n; ++c) mark[c] = -1;
            int64_t s;
#pragma omp for schedule(dynamic, 64)
            for (s = 0; s < nsel; ++s) {
                int64_t i = rows ? rows[s] : s;
                int64_t len = 0;
                for (int64_t j = rptA[i]; j < rptA[i + 1]; ++j) {
                    int32_t k = colA[j];
                    double a = (double)valA[j];
                    for (int64_t t = rptB[k]; t < rptB[k + 1]; ++t) {
                        int32_t c = colB[t];
                        double b = (double)valB[t];
                        if (mark[c] != s) {
                            mark[c] = s;
                            acc[c] = 0.0;
                            absacc[c] = 0.0;
                            list[len++] = c;
                        }
                        acc[c] += a * b;
                        absacc[c] += fabs(a) * fabs(b);
                    }
                }
                if (len != out_rpt[s + 1] - out_rpt[s]) {
#pragma omp atomic write
                    failed = -2;
                    continue;
                }
                qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);
                int64_t base = out_rpt[s];
                for (int64_t q = 0; q < len; ++q) {
                    int32_t c = list[q];
                    out_col[base + q] = c;
                    out_val[base + q] = acc[c];
                    out_abs[base + q] = absacc[c];
                }
            }
        }
        free(mark);
        free(acc);
        free(absacc);
        free(list);
    }
    return failed;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

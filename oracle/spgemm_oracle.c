/*
 * CPU oracle for sparse general matrix-matrix multiplication C = A * B.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * loads this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP path.
 *
 * What it computes (FSpGEMM, Sec. II-B "SpGEMM Algorithms", row-wise
 * Gustavson's method, Fig. 1): row i of C is the sum over the nonzeros
 * A(i,k) of the scaled sparse rows A(i,k) * B(k,:).  Adding sparse partial
 * rows is a sort by column index plus a merge that adds values with equal
 * column index (same section, "sort and merge"); the merge adds without any
 * zero test, so an entry whose terms cancel to 0.0 stays in the structure
 * (reading of Algorithm 1: the SM unit emits every merged element).
 *
 * The accumulator is Gustavson's dense sparse accumulator in FP64: a value
 * array and a marker array of length ncols(B), a list of the touched
 * columns, and a final sort of that list.  Terms are added in ascending k
 * (the order of A's row), then ascending j (the order of B's row).  FP32
 * inputs are promoted to FP64; the product of two FP32 numbers is exact in
 * FP64.  Alongside each value the oracle accumulates the error-bound scale
 * sum_k |a_ik| |b_kj|.
 *
 * Build with -O2 -ffp-contract=off so that every a*b is rounded before the
 * add (this makes the transpose identity (AB)^T = B^T A^T bit-exact between
 * two oracle runs, a pin the tests rely on).
 *
 * Rows are independent, so row ranges run in parallel with OpenMP, each
 * thread holding its own accumulator.
 *
 * Also here: per-row statistics (intermediate products, min/mean/max B-row
 * length, column span), written as plain loops over the same definitions.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline double load_val(const void* v, int is_f32, int64_t p)
{
    return is_f32 ? (double)((const float*)v)[p] : ((const double*)v)[p];
}

static int cmp_i32(const void* x, const void* y)
{
    int32_t a = *(const int32_t*)x, b = *(const int32_t*)y;
    return (a > b) - (a < b);
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Number of structural nonzeros of each row of C in [r0, r1): the size of
 * the union of the column sets of the B rows named by row i of A.
 * row_nnz has r1 - r0 entries.  Returns 0, or -1 on allocation failure.
 */
int oracle_row_nnz(int64_t r0, int64_t r1, int64_t ncols_b,
                   const int64_t* a_ptr, const int32_t* a_col,
                   const int64_t* b_ptr, const int32_t* b_col,
                   int64_t* row_nnz)
{
    int failed = 0;
#pragma omp parallel
    {
        int64_t* mark = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ncols_b > 0 ? ncols_b : 1));
        if (!mark) {
#pragma omp atomic write
            failed = 1;
        } else {
            for (int64_t j = 0; j < ncols_b; ++j) mark[j] = -1;
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = r0; i < r1; ++i) {
                int64_t count = 0;
                for (int64_t p = a_ptr[i]; p < a_ptr[i + 1]; ++p) {
                    int32_t k = a_col[p];
                    for (int64_t q = b_ptr[k]; q < b_ptr[k + 1]; ++q) {
                        int32_t j = b_col[q];
                        if (mark[j] != i) {
                            mark[j] = i;
                            ++count;
                        }
                    }
                }
                row_nnz[i - r0] = count;
            }
            free(mark);
        }
    }
    return failed ? -1 : 0;
}

/*
 * Rows [r0, r1) of C = A*B.  out_ptr holds r1 - r0 + 1 offsets into the
 * output arrays (out_ptr[0] need not be 0; it is the offset of row r0), as
 * produced by a prefix sum of oracle_row_nnz.  Writes sorted column indices,
 * FP64 values and FP64 bound scales sum |a||b|.  Returns 0, -1 on allocation
 * failure, -2 if a row's count disagrees with out_ptr.
 */
int oracle_spgemm_rows(int64_t r0, int64_t r1, int64_t ncols_b,
                       const int64_t* a_ptr, const int32_t* a_col, const void* a_val,
                       const int64_t* b_ptr, const int32_t* b_col, const void* b_val,
                       int is_f32, const int64_t* out_ptr,
                       int32_t* out_col, double* out_val, double* out_bnd)
{
    int failed = 0;
#pragma omp parallel
    {
        size_t n = (size_t)(ncols_b > 0 ? ncols_b : 1);
        double* acc = (double*)malloc(sizeof(double) * n);
        double* bnd = (double*)malloc(sizeof(double) * n);
        int64_t* mark = (int64_t*)malloc(sizeof(int64_t) * n);
        int32_t* list = (int32_t*)malloc(sizeof(int32_t) * n);
        if (!acc || !bnd || !mark || !list) {
#pragma omp atomic write
            failed = -1;
        } else {
            for (int64_t j = 0; j < ncols_b; ++j) mark[j] = -1;
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = r0; i < r1; ++i) {
                int64_t len = 0;
                for (int64_t p = a_ptr[i]; p < a_ptr[i + 1]; ++p) {
                    int32_t k = a_col[p];
                    double a = load_val(a_val, is_f32, p);
                    for (int64_t q = b_ptr[k]; q < b_ptr[k + 1]; ++q) {
                        int32_t j = b_col[q];
                        double b = load_val(b_val, is_f32, q);
                        if (mark[j] != i) {
                            mark[j] = i;
                            acc[j] = 0.0;
                            bnd[j] = 0.0;
                            list[len++] = j;
                        }
                        double t = a * b;
                        acc[j] = acc[j] + t;
                        bnd[j] = bnd[j] + fabs(t);
                    }
                }
                int64_t base = out_ptr[i - r0];
                if (out_ptr[i - r0 + 1] - base != len) {
#pragma omp atomic write
                    failed = -2;
                    continue;
                }
                qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);
                for (int64_t e = 0; e < len; ++e) {
                    int32_t j = list[e];
                    out_col[base + e] = j;
                    out_val[base + e] = acc[j];
                    out_bnd[base + e] = bnd[j];
                }
            }
        }
        free(acc);
        free(bnd);
        free(mark);
        free(list);
    }
    return failed;
}

/*
 * Per-row statistics of row i of A against B, for i in [r0, r1):
 *   nnz_a[i]   number of nonzeros in A(i,:)
 *   prod[i]    sum over k in A(i,:) of nnz(B(k,:)): the intermediate
 *              products of row i under Gustavson's method
 *   min_b/max_b  the smallest and largest nnz(B(k,:)) over k in A(i,:)
 *              (0 for an empty row)
 *   span[i]    largest minus smallest column index over the nonempty B
 *              rows named by A(i,:) (0 if there are none)
 * All arrays hold r1 - r0 entries.
 */
void oracle_row_stats(int64_t r0, int64_t r1,
                      const int64_t* a_ptr, const int32_t* a_col,
                      const int64_t* b_ptr, const int32_t* b_col,
                      int64_t* nnz_a, int64_t* prod, int64_t* min_b,
                      int64_t* max_b, int64_t* span)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = r0; i < r1; ++i) {
        int64_t s = 0, mn = -1, mx = 0, lo = -1, hi = -1;
        for (int64_t p = a_ptr[i]; p < a_ptr[i + 1]; ++p) {
            int32_t k = a_col[p];
            int64_t len = b_ptr[k + 1] - b_ptr[k];
            s += len;
            if (mn < 0 || len < mn) mn = len;
            if (len > mx) mx = len;
            if (len > 0) {
                int64_t first = b_col[b_ptr[k]];
                int64_t last = b_col[b_ptr[k + 1] - 1];
                if (lo < 0 || first < lo) lo = first;
                if (hi < 0 || last > hi) hi = last;
            }
        }
        nnz_a[i - r0] = a_ptr[i + 1] - a_ptr[i];
        prod[i - r0] = s;
        min_b[i - r0] = mn < 0 ? 0 : mn;
        max_b[i - r0] = mx;
        span[i - r0] = lo < 0 ? 0 : hi - lo;
    }
}

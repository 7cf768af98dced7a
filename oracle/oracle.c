/*
 * oracle.c - plain, slow, obviously correct CPU reference for the CSR SpMV +
 * dot hot path and the loops that call it.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this file; it shares no header, helper, table or constant with
 * the HIP path.  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.
 *
 * Built with `gcc -O2 -ffp-contract=off` (no FMA contraction, no reordering)
 * so every sum is taken exactly in the order written here, in IEEE binary64
 * with round-to-nearest-even.
 *
 * Paper: Ginsbach, Collie, O'Boyle, "Automatically Harnessing Sparse
 * Acceleration", CC 2020.  Section names below refer to that paper.
 */
#include <omp.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Validation outcome codes (first failing check wins). */
#define OR_OK 0
#define OR_BAD_ROWS (-1)   /* rows < 0 */
#define OR_BAD_FIRST (-2)  /* row_ptr[0] != 0 */
#define OR_BAD_MONO (-3)   /* row_ptr decreases somewhere */
#define OR_BAD_COL (-4)    /* a column index < 0 or >= cols */

/*
 * CSR well-formedness, following the format's definition (section "Sparse
 * Matrix Variations in LiLAC-What", CSR paragraph): row_ptr[i] is where row i
 * begins in col_idx/vals, so row_ptr starts at 0 and never decreases; rows =
 * len(row_ptr)-1; nnz = row_ptr[rows].  With cols >= 0 every column index
 * must lie in [0, cols).  cols < 0 means "not given": only col >= 0 is
 * required (the column count is then derived, see oracle_csr_cols).
 */
int oracle_csr_validate(int32_t rows, const int32_t *row_ptr,
                        const int32_t *col_idx, int32_t cols)
{
    if (rows < 0)
        return OR_BAD_ROWS;
    if (row_ptr[0] != 0)
        return OR_BAD_FIRST;
    for (int32_t i = 0; i < rows; ++i)
        if (row_ptr[i + 1] < row_ptr[i])
            return OR_BAD_MONO;
    int64_t nnz = row_ptr[rows];
    for (int64_t k = 0; k < nnz; ++k) {
        if (col_idx[k] < 0)
            return OR_BAD_COL;
        if (cols >= 0 && col_idx[k] >= cols)
            return OR_BAD_COL;
    }
    return OR_OK;
}

/*
 * The column count is not stored in CSR; the paper's MKL harness computes it
 * as the largest column index plus one and caches it as a data-dependent
 * invariant (section "LiLAC-How", the MKL example and the marshaled
 * "cols" computation).  An empty matrix has 0 columns.
 */
int32_t oracle_csr_cols(int64_t nnz, const int32_t *col_idx)
{
    int32_t m = -1;
    for (int64_t k = 0; k < nnz; ++k)
        if (col_idx[k] > m)
            m = col_idx[k];
    return m + 1;
}

/*
 * CSR sparse matrix-vector product y = A x (section "Sparse Matrix Variations
 * in LiLAC-What", CSR; the spmv_csr computation that the harness replaces).
 * The harness call replaces the loop together with its result store (section
 * "Code Replacement"), so y is overwritten: an empty row gives exactly 0.
 *   y[i] = sum_{k = row_ptr[i]}^{row_ptr[i+1]-1} vals[k] * x[col_idx[k]]
 * Summed in CSR order.  Repeated column indices simply add.
 */
void oracle_spmv_csr_f64(int32_t rows, const int32_t *row_ptr,
                         const int32_t *col_idx, const double *vals,
                         const double *x, double *y)
{
    for (int32_t i = 0; i < rows; ++i) {
        double s = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            s += vals[k] * x[col_idx[k]];
        y[i] = s;
    }
}

/* The same product with the rows shared among host threads (OpenMP): each
 * row is formed exactly as above, so the result equals the serial one bit
 * for bit.  Only used to time the host baseline on all of its cores. */
void oracle_spmv_csr_f64_par(int32_t rows, const int32_t *row_ptr,
                             const int32_t *col_idx, const double *vals,
                             const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < rows; ++i) {
        double s = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            s += vals[k] * x[col_idx[k]];
        y[i] = s;
    }
}

/* Threads the parallel product uses. */
int oracle_threads(void)
{
    return omp_get_max_threads();
}

/* Same product for float32 storage: every operand is widened to binary64
 * first, so the result is the float64 value of the float32 data. */
void oracle_spmv_csr_f32(int32_t rows, const int32_t *row_ptr,
                         const int32_t *col_idx, const float *vals,
                         const float *x, double *y)
{
    for (int32_t i = 0; i < rows; ++i) {
        double s = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            s += (double)vals[k] * (double)x[col_idx[k]];
        y[i] = s;
    }
}

/* Per-row magnitude sum_k |vals[k]| |x[col_idx[k]]|: the scale against
 * which a floating-point SpMV result is judged. */
void oracle_spmv_abs_f64(int32_t rows, const int32_t *row_ptr,
                         const int32_t *col_idx, const double *vals,
                         const double *x, double *out)
{
    for (int32_t i = 0; i < rows; ++i) {
        double s = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            s += fabs(vals[k]) * fabs(x[col_idx[k]]);
        out[i] = s;
    }
}

void oracle_spmv_abs_f32(int32_t rows, const int32_t *row_ptr,
                         const int32_t *col_idx, const float *vals,
                         const float *x, double *out)
{
    for (int32_t i = 0; i < rows; ++i) {
        double s = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            s += fabs((double)vals[k]) * fabs((double)x[col_idx[k]]);
        out[i] = s;
    }
}

/*
 * Dot product, the paper's dotproduct computation (section "Backtracking
 * Search Algorithm", the dotproduct specification):
 *   result = sum_{0 <= i < length} a[i] * b[i]
 * Each product is rounded once; the running sum is kept with Neumaier's
 * compensated summation (Neumaier 1974) so that the oracle's own error is
 * about 2u * sum |a_i b_i| even at n ~ 1e5..1e8, far inside the tolerance the
 * GPU result is judged by.  An empty sum is 0.
 */
double oracle_dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double p = a[i] * b[i];
        double t = s + p;
        if (fabs(s) >= fabs(p))
            c += (s - t) + p;
        else
            c += (p - t) + s;
        s = t;
    }
    return s + c;
}

/* sum |a_i| |b_i|, the scale for judging a dot result. */
double oracle_dot_abs(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += fabs(a[i]) * fabs(b[i]);
    return s;
}

/*
 * Unpreconditioned conjugate gradient (Hestenes-Stiefel), the solver loop of
 * the paper's NPB-CG motivating example (sections "Introduction" and
 * "Overview"), whose sparse matrix-vector product and dot products are the
 * library calls.  Starting from x = 0, r = b, p = r, rho = r.r, each
 * iteration does
 *     q = A p;  alpha = rho / (p.q);  x += alpha p;  r -= alpha q;
 *     rho' = r.r;  beta = rho' / rho;  p = r + beta p;  rho = rho'
 * for exactly `iters` iterations, stopping early (and keeping x) only when
 * rho == 0 or p.q == 0.  Returns the number of completed iterations;
 * rho_hist (iters+1 entries, may be NULL) receives rho before each iteration
 * and after the last.
 */
int oracle_cg(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
              const double *vals, const double *b, double *x, int iters,
              double *rho_hist)
{
    double *r = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *p = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *q = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) {
        x[i] = 0.0;
        r[i] = b[i];
        p[i] = b[i];
    }
    double rho = oracle_dot(n, r, r);
    int it = 0;
    if (rho_hist)
        for (int k = 0; k <= iters; ++k)
            rho_hist[k] = NAN;
    for (; it < iters; ++it) {
        if (rho_hist)
            rho_hist[it] = rho;
        if (rho == 0.0)
            break;
        oracle_spmv_csr_f64(n, row_ptr, col_idx, vals, p, q);
        double pq = oracle_dot(n, p, q);
        if (pq == 0.0)
            break;
        double alpha = rho / pq;
        for (int32_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        double rho_new = oracle_dot(n, r, r);
        double beta = rho_new / rho;
        for (int32_t i = 0; i < n; ++i)
            p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }
    if (rho_hist)
        rho_hist[it] = rho;
    free(r);
    free(p);
    free(q);
    return it;
}

/*
 * One PageRank step over a pull-direction CSR (rows are destinations,
 * vals[k] = 1/outdeg(source)), the repeated SpMV of the paper's PageRank
 * graph kernel (section "Results", graph kernels):
 *     y[i] = d * sum_k vals[k] * x[col_idx[k]] + (1 - d) / rows
 * Mass of vertices without out-edges is not redistributed.  float32 matrix
 * and vector, binary64 arithmetic.
 */
void oracle_pagerank_step_f32(int32_t rows, const int32_t *row_ptr,
                              const int32_t *col_idx, const float *vals,
                              const float *x, double d, double *y)
{
    double tele = (1.0 - d) / (double)rows;
    for (int32_t i = 0; i < rows; ++i) {
        double s = 0.0;
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
            s += (double)vals[k] * (double)x[col_idx[k]];
        y[i] = d * s + tele;
    }
}

/* `iters` PageRank steps from x_inout, carried entirely in binary64. */
void oracle_pagerank_f64(int32_t rows, const int32_t *row_ptr,
                         const int32_t *col_idx, const float *vals, double d,
                         int iters, double *x_inout)
{
    double *y = malloc(sizeof(double) * (size_t)(rows > 0 ? rows : 1));
    double tele = (1.0 - d) / (double)rows;
    for (int it = 0; it < iters; ++it) {
        for (int32_t i = 0; i < rows; ++i) {
            double s = 0.0;
            for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
                s += (double)vals[k] * x_inout[col_idx[k]];
            y[i] = d * s + tele;
        }
        memcpy(x_inout, y, sizeof(double) * (size_t)rows);
    }
    free(y);
}

/*
 * Row-length binning (the analysis step a sparse library runs once per
 * matrix and then amortises, like the tuning phase the paper measures in
 * section "Effectiveness of Data Marshaling").  Definitions:
 *   len_i = row_ptr[i+1] - row_ptr[i]
 *   bin(i) = the first b in [0, nbins) with len_i <= upper[b]
 *            (upper is ascending; rows longer than every bound get bin nbins-1)
 *   bin_off[b] = number of rows whose bin is < b   (bin_off[nbins] = rows)
 *   bin_rows lists the rows of bin 0, then bin 1, ..., each in ascending order.
 */
void oracle_bins(int32_t rows, const int32_t *row_ptr, int32_t nbins,
                 const int32_t *upper, int32_t *bin_of_row, int32_t *bin_off,
                 int32_t *bin_rows)
{
    for (int32_t b = 0; b <= nbins; ++b)
        bin_off[b] = 0;
    for (int32_t i = 0; i < rows; ++i) {
        int32_t len = row_ptr[i + 1] - row_ptr[i];
        int32_t b = 0;
        while (b < nbins - 1 && len > upper[b])
            ++b;
        bin_of_row[i] = b;
    }
    /* counts, then exclusive prefix sum */
    for (int32_t i = 0; i < rows; ++i)
        bin_off[bin_of_row[i] + 1] += 1;
    for (int32_t b = 0; b < nbins; ++b)
        bin_off[b + 1] += bin_off[b];
    /* stable placement: walk the bins, and inside each the rows in order */
    int32_t pos = 0;
    for (int32_t b = 0; b < nbins; ++b)
        for (int32_t i = 0; i < rows; ++i)
            if (bin_of_row[i] == b)
                bin_rows[pos++] = i;
}

/*
 * Chunk table for long rows: every row with len > t_split, in ascending row
 * order, is cut into consecutive pieces of `chunk` non-zeros (the last piece
 * may be shorter).  Entry j is (row, k0, k1) = the half-open range
 * [k0, k1) of the row's non-zeros.  Returns the number of entries; with NULL
 * outputs it only counts.
 */
int64_t oracle_split_chunks(int32_t rows, const int32_t *row_ptr,
                            int32_t t_split, int32_t chunk, int32_t *c_row,
                            int32_t *c_k0, int32_t *c_k1)
{
    int64_t m = 0;
    for (int32_t i = 0; i < rows; ++i) {
        int32_t a = row_ptr[i], e = row_ptr[i + 1];
        if (e - a <= t_split)
            continue;
        for (int32_t k = a; k < e; k += chunk) {
            if (c_row) {
                c_row[m] = i;
                c_k0[m] = k;
                c_k1[m] = (e - k > chunk) ? k + chunk : e;
            }
            ++m;
        }
    }
    return m;
}

/*
 * Jagged Diagonal Storage (section "Sparse Matrix Variations in LiLAC-What",
 * JDS paragraph, and the JDS figure): rows are reordered by decreasing
 * non-zero count (ties keep their original order); perm[i] is the new
 * position of original row i; nzcnt[p] is the count of the row at new
 * position p; diagonal j holds the j-th non-zero of every row that has one,
 * in new-row order, starting at jd_ptr[j].  jd_ptr has max_len+1 entries.
 * Returns max_len.
 */
int32_t oracle_csr_to_jds(int32_t rows, const int32_t *row_ptr,
                          const int32_t *col_idx, const double *vals,
                          int32_t *perm, int32_t *nzcnt, int32_t *jd_ptr,
                          int32_t *jd_col, double *jd_val)
{
    int32_t *order = malloc(sizeof(int32_t) * (size_t)(rows > 0 ? rows : 1));
    int32_t max_len = 0;
    for (int32_t i = 0; i < rows; ++i) {
        int32_t len = row_ptr[i + 1] - row_ptr[i];
        if (len > max_len)
            max_len = len;
    }
    /* stable order by decreasing length: scan lengths from longest down */
    int32_t pos = 0;
    for (int32_t len = max_len; len >= 0; --len)
        for (int32_t i = 0; i < rows; ++i)
            if (row_ptr[i + 1] - row_ptr[i] == len)
                order[pos++] = i;
    for (int32_t p = 0; p < rows; ++p) {
        perm[order[p]] = p;
        nzcnt[p] = row_ptr[order[p] + 1] - row_ptr[order[p]];
    }
    int32_t k = 0;
    for (int32_t j = 0; j < max_len; ++j) {
        jd_ptr[j] = k;
        for (int32_t p = 0; p < rows && nzcnt[p] > j; ++p) {
            int32_t src = row_ptr[order[p]] + j;
            jd_col[k] = col_idx[src];
            jd_val[k] = vals[src];
            ++k;
        }
    }
    jd_ptr[max_len] = k;
    free(order);
    return max_len;
}

/* y = A x from JDS: the row at new position p accumulates its diagonals in
 * order j = 0, 1, ..., and the result goes to original row order via perm. */
void oracle_spmv_jds_f64(int32_t rows, int32_t max_len, const int32_t *perm,
                         const int32_t *nzcnt, const int32_t *jd_ptr,
                         const int32_t *jd_col, const double *jd_val,
                         const double *x, double *y)
{
    for (int32_t i = 0; i < rows; ++i) {
        int32_t p = perm[i];
        double s = 0.0;
        for (int32_t j = 0; j < max_len && j < nzcnt[p]; ++j) {
            int32_t k = jd_ptr[j] + p;
            s += jd_val[k] * x[jd_col[k]];
        }
        y[i] = s;
    }
}

/*
 * Breadth-first search levels by repeated sparse matrix-vector products over
 * the Boolean (or, and) semiring, the SpMV-based BFS graph kernel the paper
 * accelerates (section "Results", graph kernels).  Pull CSR: row v lists the
 * sources u of edges u -> v.  level[src] = 0; a vertex joins level L+1 if it
 * has no level yet and some source in its row is in level L.  Unreached
 * vertices keep -1.  Returns the number of levels.
 */
int32_t oracle_bfs_levels(int32_t rows, const int32_t *row_ptr,
                          const int32_t *col_idx, int32_t source,
                          int32_t *level)
{
    for (int32_t i = 0; i < rows; ++i)
        level[i] = -1;
    if (rows <= 0)
        return 0;
    level[source] = 0;
    int32_t depth = 0;
    for (;;) {
        int changed = 0;
        for (int32_t v = 0; v < rows; ++v) {
            if (level[v] != -1)
                continue;
            for (int32_t k = row_ptr[v]; k < row_ptr[v + 1]; ++k)
                if (level[col_idx[k]] == depth) {
                    level[v] = depth + 1;
                    changed = 1;
                    break;
                }
        }
        if (!changed)
            break;
        ++depth;
    }
    return depth + 1;
}

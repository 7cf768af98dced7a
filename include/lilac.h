/*
 * lilac.h - C ABI of liblilac.so, an AMD Instinct MI355X (gfx950) library for
 * the computations that the LiLAC compiler (Ginsbach, Collie, O'Boyle,
 * "Automatically Harnessing Sparse Acceleration", CC 2020) offloads to
 * sparse libraries: the CSR sparse matrix-vector product and the dense dot
 * product, plus the solver and graph loops built from them.
 *
 * General conventions (apply to every call unless its comment says otherwise)
 *  - Indices are 0-based int32 (`int`).  CSR is (row_ptr[rows+1], col_idx[nnz],
 *    vals[nnz]) as defined in the paper's section "Sparse Matrix Variations in
 *    LiLAC-What" (CSR paragraph): row_ptr[i] is where row i starts, rows is
 *    len(row_ptr)-1, the column count is not part of the format.
 *  - Every call returns a status (LILAC_OK = 0, negative on error) except
 *    lilac_dot / lilac_version / lilac_last_error, which return their value.
 *    On error lilac_last_error() gives a thread-local message.  No C++
 *    exception ever crosses this interface.
 *  - The caller owns every pointer it passes; the library never frees caller
 *    memory.  "host or device" pointers are classified with
 *    hipPointerGetAttributes; "device" pointers must be device memory of the
 *    current HIP device.
 *  - `stream` is a hipStream_t passed as void*; NULL is HIP's default (null)
 *    stream.  Calls marked "async" only enqueue work on `stream` and return;
 *    the caller orders them against its own work through that stream.
 *    Blocking calls that read device memory first wait for the whole device
 *    (hipDeviceSynchronize), since the data may come from any stream.
 *  - Floating-point results are not bitwise reproducible against a serial
 *    loop (sums are reordered and contracted to FMA), but every call is
 *    deterministic: the same inputs and the same matrix handle give bitwise
 *    identical outputs on every run, alone or in a batch.
 *  - Entry points are thread-safe (one library lock serialises them).
 */
#ifndef LILAC_H
#define LILAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define LILAC_OK 0
#define LILAC_ERR_ARG (-1)         /* bad argument (NULL, negative size ...) */
#define LILAC_ERR_CSR (-2)         /* matrix is not well-formed CSR */
#define LILAC_ERR_OOM (-3)         /* device allocation failed */
#define LILAC_ERR_BUDGET (-4)      /* would exceed the HBM byte budget */
#define LILAC_ERR_DEVICE (-5)      /* a HIP call failed / no device */
#define LILAC_ERR_STATE (-6)       /* call not valid in the object's state */
#define LILAC_ERR_UNSUPPORTED (-7) /* combination not implemented */

typedef enum { LILAC_F64 = 0, LILAC_F32 = 1 } lilac_dtype;

typedef struct lilac_csr_s *lilac_csr_t;

/* ---- library lifetime ------------------------------------------------ */
/*
 * Persistent state shared by all calls (the paper's PersistentVariables,
 * with BeforeFirstExecution / AfterLastExecution set-up and tear-down,
 * section "LiLAC-How", paragraph "Persistence").  lilac_init is optional: the
 * first call of any entry point initialises the library on the current
 * device.  lilac_finalize releases every device copy the library made
 * (including the raw-call cache) and is also run at process exit.
 * Returns LILAC_ERR_DEVICE if no HIP device is usable.
 */
int lilac_init(int device);
int lilac_finalize(void);
const char *lilac_last_error(void);
int lilac_version(void); /* major*10000 + minor*100 + patch */

/* ---- paper-shaped calls ---------------------------------------------- */
/*
 * y = A x over CSR, the spmv_csr computation whose loop the paper's compiler
 * replaces by a harness call (sections "Overview" and "Code Replacement");
 * y is overwritten (an empty row gives 0):
 *     y[i] = sum_{k=row_ptr[i]}^{row_ptr[i+1]-1} vals[k] * x[col_idx[k]]
 * Every pointer may be host or device.  x must hold cols = max(col_idx)+1
 * entries, y holds rows entries.  Blocking: returns when y is written.
 * Marshaling (section "Data Marshaling", and the ReadObject rules of section
 * "Implementation", LiLAC-How): the three matrix arrays are copied to the
 * device on the first call and cached, keyed by their addresses and sizes;
 * later calls with the same arrays reuse the device copy and the analysis
 * (including cols) until lilac_invalidate names one of the arrays or
 * lilac_release_all / lilac_finalize runs.  The environment variable
 * LILAC_MARSHAL=naive turns caching off (every call re-uploads, for the
 * paper's naive-transfer comparison); LILAC_MARSHAL=protect tracks host
 * writes to cached host arrays with page protection and re-uploads them
 * automatically.  Host x is uploaded and host y copied back on every call.
 * Errors: LILAC_ERR_ARG (rows < 0, NULL), LILAC_ERR_CSR (validation failed:
 * row_ptr[0] != 0, row_ptr decreasing, a column index < 0).
 */
int lilac_spmv_csr(int rows, const int *row_ptr, const int *col_idx,
                   const double *vals, const double *x, double *y);
/* Same with float32 values and vectors; products are accumulated in
 * binary64 and rounded once to float32 when stored. */
int lilac_spmv_csr_f32(int rows, const int *row_ptr, const int *col_idx,
                       const float *vals, const float *x, float *y);

/*
 * result = sum_{0 <= i < n} a[i] * b[i], the dotproduct computation (section
 * "Backtracking Search Algorithm", the dotproduct specification).  a and b
 * may be host or device; the sum is taken on the device in a fixed two-level
 * order.  n == 0 gives 0.  On error returns NaN and sets lilac_last_error.
 */
double lilac_dot(int64_t n, const double *a, const double *b);
/* The same for float32 arrays: products and sums in binary64 (the float32
 * values widened exactly), the total rounded once to float32. */
float lilac_dot_f32(int64_t n, const float *a, const float *b);

/* Marshaling control for the raw calls: the next call that uses the array
 * containing `ptr` re-uploads it (values only when ptr is a vals array,
 * full re-analysis when it is row_ptr or col_idx).  Unknown pointers are
 * ignored.  lilac_release_all frees every cached device copy. */
int lilac_invalidate(const void *ptr);
int lilac_release_all(void);

/* ---- device-resident matrix handle ----------------------------------- */
#define LILAC_KEEP_HOST 1u /* remember the host pointers for invalidate */
/*
 * Creates a device copy of a CSR matrix (the ReadObject "construct" +
 * "update" of the paper's section "Implementation", LiLAC-How): validates
 * it, uploads it, derives cols = max(col_idx)+1 when cols < 0 (the cached
 * invariant of section "LiLAC-How", the MKL example), and runs the one-time
 * row-length analysis (bins of rows by length, chunk table for long rows)
 * that every later product reuses.  Input pointers may be host or device;
 * vals is double* for LILAC_F64, float* for LILAC_F32.  nnz must equal
 * row_ptr[rows].  The handle owns its device memory.  Blocking.
 * Errors: LILAC_ERR_ARG, LILAC_ERR_CSR, LILAC_ERR_OOM, LILAC_ERR_BUDGET.
 */
int lilac_csr_create(lilac_csr_t *h, int rows, int cols, int64_t nnz,
                     const int *row_ptr, const int *col_idx, const void *vals,
                     lilac_dtype dt, unsigned flags);
/* New values for the same structure ("update"); vals host or device. */
int lilac_csr_update_values(lilac_csr_t h, const void *vals);
/* With LILAC_KEEP_HOST: re-upload and re-analyse from the remembered host
 * pointers before the next use.  LILAC_ERR_STATE without it. */
int lilac_csr_invalidate(lilac_csr_t h);
/* Waits for the library's work on the handle, then frees it ("destruct"). */
int lilac_csr_destroy(lilac_csr_t h);

typedef struct {
    int rows, cols;
    int64_t nnz;
    int64_t device_bytes;   /* bytes the handle holds on the device */
    int dtype;              /* lilac_dtype */
    int nbins;              /* number of row-length classes (9) */
    int bin_upper[16];      /* inclusive upper row length of each class */
    int bin_count[16];      /* rows in each class */
    int chunk;              /* non-zeros per chunk of a split row */
    int64_t nchunks;        /* entries of the chunk table */
    int ntiles;             /* work tiles of one product */
    int layout;             /* LILAC_LAYOUT_ROWS, _PANELS, _HOT or _BAND in use */
    int npanels;            /* column panels (panel layout), else 0 */
} lilac_csr_info_t;
int lilac_csr_info(lilac_csr_t h, lilac_csr_info_t *out);

/*
 * Copies the handle's analysis to host arrays (for inspection and tests):
 * bin_off[nbins+1] (row offsets of each class in bin_rows), bin_rows[rows]
 * (rows grouped by class, ascending inside each class), and the chunk table
 * c_row/c_k0/c_k1[nchunks] (row and half-open non-zero range of each chunk
 * of the rows longer than the split threshold).  Any output may be NULL.
 * Blocking.
 */
int lilac_csr_analysis(lilac_csr_t h, int *bin_off, int *bin_rows, int *c_row,
                       int *c_k0, int *c_k1);

/*
 * Row-class thresholds: upper[c] is the largest row length handled by class
 * c (classes use 1, 2, 4, 8, 16, 32, 64 lanes per row, then a whole
 * workgroup per row, then split rows cut into `chunk`-non-zero pieces);
 * rows_per_group[c] is how many rows one lane group handles per tile.  Any
 * change re-runs the analysis.  NULL arguments keep the current values.
 */
int lilac_csr_set_plan(lilac_csr_t h, const int *upper /* [8] */,
                       const int *rows_per_group /* [9] */, int chunk);

/*
 * Device layout used by the product.  LILAC_LAYOUT_ROWS: the CSR arrays with
 * the row-class tiles above.  LILAC_LAYOUT_PANELS: a second, column-panel
 * copy of the matrix in which the columns are cut into panels that fit the
 * LDS and the rows into blocks; each workgroup stages one panel of x in LDS
 * at a time and gathers from there, with 16-bit column offsets.  Row
 * blocks hold at most 4096 rows, enough blocks for every CU but at least
 * the rows that weigh as much as one copy of x; the block's row sums and
 * one panel share the LDS.  It suits matrices whose
 * non-zeros scatter over x; it is built only for at most 64 panels (else
 * the rows layout is used).  LILAC_LAYOUT_AUTO (the default) picks it for
 * gather-heavy matrices (sampled distinct 128-byte x lines per non-zero at
 * least 0.3, at least 16384 non-zeros) with no row longer than 1024 and
 * copies of x at most four times the matrix bytes.  Batched calls run all
 * column-panel matrices of a batch in one launch, with the same results.  LILAC_LAYOUT_HOT: a second copy for
 * matrices whose most referenced columns have the lowest indices (a graph
 * relabelled by decreasing out-degree, as lilac_pagerank does by itself for
 * graphs of at least 65536 vertices): the first 34560 (float32) or 17280
 * (float64) columns of x stay in LDS, the others are read from x in device
 * memory; rows are cut into blocks of at most 1536 non-empty rows (24576
 * rows in all) and about equal non-zeros, and empty rows take no row sum.  Built only on request and only for matrices with non-zeros;
 * otherwise the rows layout is used (lilac_csr_info reports which).  Every
 * layout gives deterministic results.  LILAC_LAYOUT_BAND: the CSR order and
 * values with one extra 32-bit word per non-zero packing the row inside a
 * block of at most 2048 rows and the column offset from the block's first
 * column; possible when no block has to span 65536 columns or more (banded
 * and stencil matrices, small matrices).  The wavefronts stream the
 * entries and add up each row's run with a segmented scan.  LILAC_LAYOUT_AUTO
 * picks it for matrices with at least 16384 non-zeros whose columns are
 * local (sampled distinct 128-byte x lines per non-zero below 0.3) when it
 * is possible and its blocks average at least 1024 non-zeros (rows whose
 * columns are local within each row but not between neighbouring rows cut
 * a block at nearly every row: those stay on the rows layout).  Re-runs
 * the analysis.
 */
#define LILAC_LAYOUT_AUTO (-1)
#define LILAC_LAYOUT_ROWS 0
#define LILAC_LAYOUT_PANELS 1
#define LILAC_LAYOUT_HOT 2
#define LILAC_LAYOUT_BAND 3
int lilac_csr_set_layout(lilac_csr_t h, int layout);

/*
 * y = A x with x (cols entries) and y (rows entries) in device memory, of the
 * handle's dtype.  Async on `stream`.
 */
int lilac_spmv(lilac_csr_t h, const void *x, void *y, void *stream);

/* y = A x and out = sum_i w[i] * y[i] (the fused product + dot a CG step
 * needs); w, x, y device arrays of the handle's dtype (F64 only), out a
 * device double.  Async. */
int lilac_spmv_dot(lilac_csr_t h, const void *x, void *y, const void *w,
                   double *out, void *stream);

/*
 * out = sum a[i] b[i] (the dotproduct computation of section "Backtracking
 * Search Algorithm") with device a, b of n elements of `dtype` (lilac_dtype)
 * and a device result of the same dtype.  Products and the fixed two-level
 * sum are binary64 (float32 data widened exactly); a float32 result is that
 * total rounded once.  n == 0 stores 0.  The partial sums live in the
 * library's scratch, so calls on different streams must not overlap.
 * Async.  Errors: LILAC_ERR_ARG (n < 0, NULL, unknown dtype).
 */
int lilac_dot_dev(int64_t n, const void *a, const void *b, void *out, lilac_dtype dtype,
                  void *stream);

/*
 * Conjugate gradient on an SPD handle (F64), the solver loop of the paper's
 * NPB-CG example (sections "Introduction" and "Overview"): from x = 0,
 * `iters` iterations of
 *   q = A p; alpha = rho/(p.q); x += alpha p; r -= alpha q;
 *   rho' = r.r; beta = rho'/rho; p = r + beta p
 * stopping early (x kept) only if rho or p.q becomes exactly 0 (p.q as
 * the recurrence below gives it).  The
 * iterations are computed in the arrangement of Chronopoulos and Gear
 * (1989), the same iterates in exact arithmetic: the product is w = A r and
 * s = A p is updated alongside p, so both inner products of an iteration
 * are known together and an iteration is one product (with r.w fused into
 * it) and one vector kernel.  b and x are device arrays of rows doubles.
 * With LILAC_CG_GRAPH the whole solve runs as one captured HIP graph
 * (scalars stay on the device, no host round trip); the graph is cached per
 * (handle, b, x, iters).  rho_out / iters_done are host pointers (may be
 * NULL; if given the call waits for the result): r.r of the final residual
 * (or at the early stop) and the iterations done.  Async otherwise.
 */
#define LILAC_CG_GRAPH 1u
int lilac_cg(lilac_csr_t h, const double *b, double *x, int iters,
             unsigned flags, void *stream, double *rho_out, int *iters_done);

/*
 * The same conjugate gradient as lilac_cg (eager, identical kernels and
 * reduction shapes, so x is bitwise what lilac_cg without LILAC_CG_GRAPH
 * gives), for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  It
 * allocates nothing: the solver state (r, p, s, w, partial sums, scalars)
 * lives in one fixed device array of the library, 32 MiB per GPU, held from
 * the library's set-up until the process ends, which limits the matrix to
 * at most 1048576 rows (LILAC_ERR_ARG beyond).  The handle must be up to
 * date: after lilac_csr_invalidate it is refused with LILAC_ERR_STATE until
 * a call that may allocate (lilac_spmv, lilac_cg ...) has re-uploaded the
 * matrix (lilac_csr_update_values uploads at once).  b and x are device arrays of
 * rows doubles.  Every call on one GPU shares that array, so calls that
 * overlap on one GPU (other streams, other threads, other handles) race and
 * must be ordered by the caller; each call initialises all of the state it
 * reads.  Async on `stream` (NULL: HIP's null stream).
 */
int lilac_cg_noalloc(lilac_csr_t h, const double *b, double *x, int iters, void *stream);

/*
 * PageRank power iteration on a pull-direction F32 handle (rows are
 * destinations, vals[k] = 1/outdeg of the source), the repeated product of
 * the paper's PageRank graph kernel (section "Results", graph kernels):
 *   x <- d * (A x) + (1 - d) / rows      repeated `iters` times
 * x_inout is a device float array of rows entries holding the start vector
 * and receiving the result.  Runs as a cached HIP graph.  Async.
 */
int lilac_pagerank(lilac_csr_t h, float damping, int iters, float *x_inout,
                   void *stream);

/*
 * Many independent products y_j = A_j x_j in one grouped persistent launch
 * (plus one finaliser launch if any matrix has split rows).  Each y_j is
 * bitwise equal to what lilac_spmv(h_j, x_j, y_j) gives.  All handles must
 * share one dtype.  The grouped work list is cached per (handles, x, y)
 * pointer set.  Async.
 */
int lilac_spmv_batched(int count, const lilac_csr_t *hs, const void *const *xs,
                       void *const *ys, void *stream);

/*
 * Autotuner: times candidate row-class thresholds and tile shapes on the
 * handle's own matrix (a few products into scratch vectors), keeps the
 * fastest, and records it in the tuning cache under a key made of the
 * matrix's shape class, so later handles of the same class start from it.
 * The cache is read from and written to the JSON file named by
 * LILAC_TUNE_CACHE when set.  Blocking.  best_us (may be NULL) receives the
 * time of one product with the chosen plan.
 */
int lilac_csr_tune(lilac_csr_t h, double *best_us);
/*
 * Autotuner for a batch (the choice of storage per matrix of section
 * "Necessity of Flexible Backends", made by timing): the handles are
 * grouped by shape class (lilac_csr_tune_class); class by class, most
 * non-zeros first, each layout a grouped launch takes (row-class tiles,
 * column panels, band) is tried on all matrices of the class and kept when
 * the whole lilac_spmv_batched call on (hs, xs, ys) gets at least 1%
 * faster.  The handles keep the chosen plans, and each class's plan goes
 * to the tuning cache (and the LILAC_TUNE_CACHE file), so handles created
 * later start from it.  The vectors are overwritten by the trial calls.
 * best_ms (may be NULL) receives the time of one batched call with the
 * chosen plans.  Blocking.  Errors: LILAC_ERR_ARG.
 */
int lilac_spmv_batched_tune(int count, const lilac_csr_t *hs, const void *const *xs,
                            void *const *ys, double *best_ms);
/* The shape class under which lilac_csr_tune records and looks up plans
 * (dtype, log2 of rows, twice log2 of the mean row length, row class of
 * the longest row), as a NUL-terminated string into buf[cap].
 * LILAC_ERR_ARG if it does not fit. */
int lilac_csr_tune_class(lilac_csr_t h, char *buf, int cap);
/* Forgets every tuned plan held in memory (including those read from the
 * LILAC_TUNE_CACHE file; the file itself is left as it is): handles created
 * afterwards start from the default plan and the automatic layout choice;
 * existing handles keep their plans.  Never fails. */
int lilac_tune_clear(void);

/* ---- measurement -------------------------------------------------------- */
/*
 * The device's streaming ceiling, written for this library rather than
 * borrowed: reads `bytes` of src once with non-temporal 16-byte loads (eight
 * per thread in flight), and with dst != NULL also stores them there (a
 * copy).  groups_per_cu workgroups of 256 threads per compute unit, each
 * streaming one contiguous range.  Benchmarks time it beside the products
 * to quote their bandwidth against what the part delivers as well as
 * against its nominal peak.  src, dst: device, 16-byte aligned; bytes a
 * multiple of 16.  Async on `stream` (NULL: HIP's null stream).
 * Errors: LILAC_ERR_ARG.
 */
int lilac_hbm_stream(const void *src, void *dst, int64_t bytes, int groups_per_cu,
                     void *stream);

/* ---- 64-bit row offsets ------------------------------------------------ */

/*
 * Matrices with 2^31 - 8192 or more non-zeros (the CSR arrays of the CSR
 * paragraph of section "Sparse Matrix Variations in LiLAC-What", with
 * int64 row offsets; column indices stay int32).  The rows are cut into
 * consecutive parts of at most 2^31 - 2^20 non-zeros each (the environment
 * variable LILAC_PART_NNZ, read when a matrix is created, lowers that bound
 * so that small matrices can be split for tests); each part is an ordinary
 * handle over its rows with its row offsets rebased to 32 bits, and a
 * product runs all parts as one batched call (lilac_spmv_batched) with the
 * shared x and y offset by each part's first row.
 *
 * lilac_csr64_create: row_ptr int64[rows+1], col_idx int32[nnz] and vals
 * (F64 or F32)[nnz], host or device, owned by the caller and read only
 * during the call (the parts keep their own device copies).  cols < 0:
 * max(col_idx)+1 per part.  Validation as lilac_csr_create, over all parts
 * (row_ptr[0] == 0, non-decreasing, row_ptr[rows] == nnz; LILAC_ERR_CSR
 * otherwise); LILAC_ERR_UNSUPPORTED if one row alone exceeds the part
 * bound.  Blocking.
 */
typedef struct lilac_csr64_s *lilac_csr64_t;
int lilac_csr64_create(lilac_csr64_t *h, int rows, int cols, int64_t nnz,
                       const int64_t *row_ptr, const int *col_idx, const void *vals,
                       lilac_dtype dt);
/* y = A x for device x[cols] and y[rows] of the handle's dtype; y is
 * overwritten.  Async on `stream` (NULL: the library's stream). */
int lilac_csr64_spmv(lilac_csr64_t h, const void *x, void *y, void *stream);
/* Sizes and the number of parts; any output may be NULL. */
int lilac_csr64_info(lilac_csr64_t h, int *rows, int *cols, int64_t *nnz, int *nparts);
/* Waits for the library's work on the parts, then frees them. */
int lilac_csr64_destroy(lilac_csr64_t h);

/* ---- second format and graph traversal -------------------------------- */
/*
 * y = A x with A in Jagged Diagonal Storage (section "Sparse Matrix
 * Variations in LiLAC-What", JDS paragraph and the JDS figure): rows are
 * ordered by decreasing non-zero count, perm[i] is the position of original
 * row i in that order, nzcnt[p] the count of the row at position p, diagonal
 * j (j < max_len) holds the j-th entry of every row that has one, in
 * position order, starting at jd_ptr[j]; jd_ptr has max_len+1 entries and
 * jd_ptr[max_len] is the number of entries.  Each row's sum is taken in
 * diagonal order without fused multiply-add, so y equals the sequential
 * definition bitwise.  Pointers host or device; host arrays are copied for
 * the call (JDS inputs are not cached).  Blocking.  Errors: LILAC_ERR_ARG,
 * LILAC_ERR_CSR (negative column index).
 */
int lilac_spmv_jds(int rows, int max_len, const int *perm, const int *nzcnt,
                   const int *jd_ptr, const int *jd_col, const double *jd_val,
                   const double *x, double *y);

/*
 * CSR -> JDS of a handle's matrix, on the device (section "Sparse Matrix
 * Variations in LiLAC-What", JDS paragraph and the JDS figure): rows in
 * order of decreasing non-zero count, equal counts in ascending original
 * order; perm[i] = new position of original row i; nzcnt[p] = count of the
 * row at position p; diagonal j holds the j-th entry of every row that has
 * one, in position order, from jd_ptr[j]; jd_ptr[max_len] = nnz.  The
 * arrays are exactly what lilac_spmv_jds takes.
 * *max_len (host) receives the longest row.  With jd_ptr == NULL only
 * *max_len is computed (a size query).  Otherwise every output is device
 * memory owned by the caller: perm[rows], nzcnt[rows] int, jd_ptr int with
 * jd_ptr_len >= max_len + 1 entries, jd_col[nnz] int, jd_val[nnz] of the
 * handle's dtype.  Integer work and copies only, so the result is exact.
 * Runs on `stream` (NULL: the library's stream) and returns when done.
 * Errors: LILAC_ERR_ARG (NULL, host outputs, jd_ptr too short).
 */
int lilac_csr_to_jds(lilac_csr_t h, int *perm, int *nzcnt, int *jd_ptr, int jd_ptr_len,
                     int *jd_col, void *jd_val, int *max_len, void *stream);

/*
 * Breadth-first search levels from `source` by repeated Boolean sparse
 * products over the handle's pull-direction CSR (row v lists the sources u
 * of edges u -> v), the SpMV-based BFS graph kernel of the paper's
 * evaluation (section "Results", graph kernels): level[v] = 0 for the
 * source, depth+1 for a vertex first reached from a vertex of level depth,
 * -1 if unreachable.  level is a device int array of rows entries; nlevels
 * (host, may be NULL) receives the number of levels.  Needs cols <= rows.
 * Blocking (one host check per level).
 */
int lilac_bfs(lilac_csr_t h, int source, int *level, int *nlevels, void *stream);

/* ---- request server (continuous batching) ----------------------------- */
/*
 * A server keeps a pool of matrices resident on the device and runs SpMV and
 * CG-solve requests as they arrive: a scheduler thread admits requests whose
 * matrix is resident while request slots and the HBM budget allow, and
 * advances all admitted requests together, one grouped product plus one CG
 * iteration per request per step (the Chronopoulos-Gear arrangement of
 * lilac_cg), so requests that arrive while others run join the next step;
 * matrices of 2^23 or more non-zeros step in a lane of their own.  Matrices
 * not resident are uploaded by two upload threads (overlapping the steps);
 * idle ones are evicted (LRU-2: the oldest second-to-last use first) when
 * the pool or the budget is full.  A request's result does not depend
 * on what it was batched with.  This is the persistent-state, upload-once
 * marshaling of the paper (section "LiLAC-How", "Data Marshaling") applied
 * to a stream of independent calls.  Thread-safe.
 */
typedef struct lilac_server_s *lilac_server_t;

typedef struct {
    int64_t hbm_budget;  /* device bytes for matrices + request state; <= 0: 200 GiB */
    int max_active;      /* requests admitted at once (slots); <= 0: 256 */
    int pool_capacity;   /* resident matrices before eviction; <= 0: no count
                            limit (2^20), the budget alone decides */
    int fifo;            /* 1: no batching, one request at a time with the
                            single-matrix calls (the plain path, for comparison) */
} lilac_server_config;

#define LILAC_REQ_SPMV 0
#define LILAC_REQ_CG 1

typedef struct {
    int kind;            /* LILAC_REQ_SPMV or LILAC_REQ_CG */
    int matrix;          /* id from lilac_server_add_matrix */
    int iters;           /* CG iterations (CG only) */
    const double *in;    /* device: x (SpMV, cols entries) or b (CG, rows) */
    double *out;         /* device: y (SpMV, rows entries) or x (CG, rows) */
    int64_t arrival_ns;  /* arrival time on lilac_server_now's clock; 0 = now */
} lilac_request;

typedef struct {
    int64_t completed, spmv_done, cg_done, failed;
    double p50_us, p99_us, mean_us, max_us;  /* arrival -> completion */
    double wall_s;       /* first arrival -> last completion */
    double req_per_s, solves_per_s;
    double gbytes_per_s; /* credited algorithmic bytes of the work done / wall */
    int64_t uploads, evictions, ticks;
    int64_t peak_device_bytes;    /* highest device bytes the server held (its
                                     allocator account: matrices, slots,
                                     tables), since creation or the last reset */
    int64_t device_bytes;         /* device bytes it holds now */
    int64_t planned_peak_bytes;   /* highest planned bytes (resident charges +
                                     upload reserves + slots + tables) */
    double mean_wait_us;          /* arrival -> admission (upload, slot, queue) */
    double mean_run_us;           /* admission -> completion */
    int64_t waited_upload;        /* requests whose matrix was not resident
                                     when they arrived */
} lilac_server_stats;

int lilac_server_create(lilac_server_t *s, const lilac_server_config *cfg);
/* Registers a float64 CSR matrix given by host arrays: the server copies
 * them into pinned host memory (so the caller may free or change its arrays
 * after the call) and uploads the matrix when a request first needs it, and
 * again after an eviction.  cols < 0 means cols = rows.  Must be called
 * before the first request is submitted. */
int lilac_server_add_matrix(lilac_server_t s, int rows, int cols, int64_t nnz,
                            const int *row_ptr, const int *col_idx,
                            const double *vals, int *id);
/* Queues a request (non-blocking); the device vectors must stay valid until
 * it completes.  ticket (may be NULL) identifies it. */
int lilac_server_submit(lilac_server_t s, const lilac_request *r,
                        uint64_t *ticket);
/* done: 0 pending, 1 completed, -1 failed (e.g. matrix beyond the budget). */
int lilac_server_poll(lilac_server_t s, uint64_t ticket, int *done);
/* Blocks until the request completed; LILAC_ERR_STATE if it failed. */
int lilac_server_wait(lilac_server_t s, uint64_t ticket);
int lilac_server_now(lilac_server_t s, int64_t *ns);
/* Latency and throughput of the requests completed since the last reset. */
int lilac_server_stats_get(lilac_server_t s, lilac_server_stats *out);
int lilac_server_reset_stats(lilac_server_t s);
/* Open-loop replay: request i (kind[i], matrix[i]) arrives arrival_ns[i]
 * after the start; CG requests run cg_iters iterations.  Operands are the
 * server's own per-matrix vectors (x = b = 1).  Blocks until every request
 * completed, then fills *out. */
int lilac_server_run_trace(lilac_server_t s, int n, const int64_t *arrival_ns,
                           const int *kind, const int *matrix, int cg_iters,
                           lilac_server_stats *out);
/* Finishes the requests already running, fails the queued ones, frees all. */
int lilac_server_destroy(lilac_server_t s);

#ifdef __cplusplus
}
#endif
#endif /* LILAC_H */

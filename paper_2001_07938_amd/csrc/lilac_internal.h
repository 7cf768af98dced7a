// Internal declarations shared by the HIP sources of liblilac.so.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <mutex>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "lilac.h"

namespace lilac {

// Row classes by row length.  C_W<n>: n lanes of a wavefront share one row
// (n = 1 is one lane per row, n = 64 a whole wavefront per row).  C_WG: one
// 256-lane workgroup per row.  C_SPLIT: the row is cut into chunks of
// `chunk` non-zeros, one workgroup per chunk, partial sums combined by a
// finaliser in chunk order.
enum RowClass : int32_t {
    C_W1 = 0, C_W2, C_W4, C_W8, C_W16, C_W32, C_W64, C_WG, C_SPLIT, NCLASS
};

constexpr int kBlock = 256;       // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kPad = 64;          // device arrays of nnz are padded to this
constexpr int kDotParts = 1024;   // partials of a standalone dot

// One unit of work of a product: `count` rows of class `cls`, taken from the
// class-ordered row list at `first` (for C_SPLIT: chunk index `first`).
// When the tile's rows are consecutive matrix rows, cls carries
// kTileContig and `first` is the first row itself.
constexpr int32_t kTileClassMask = 0xFF;
constexpr int32_t kTileContig = 0x100;
struct Tile {
    int32_t cls;
    int32_t mat;
    int32_t first;
    int32_t count;
};

// Everything a kernel needs to know about one matrix of a product.
struct MatDesc {
    const int32_t *row_ptr;
    const int32_t *col;
    const void *vals;
    const int32_t *bin_rows;  // rows ordered by class, ascending per class
    const int32_t *c_k0;      // chunk table: first non-zero of each chunk
    const int32_t *c_k1;      //              one past the last
    const int32_t *s_first;   // per split row: first chunk (nsplit+1 entries)
    const int32_t *c_row;     // chunk table: row of each chunk
    const void *x;
    void *y;
    const void *w;            // second operand of the fused dot (or null)
    double *chunk_part;       // one partial sum per chunk
    int32_t split_begin;      // position of the first split row in bin_rows
    int32_t nsplit;
    const Tile *tiles;        // the matrix's own tile list (segment launches)
    int32_t ntiles;
    int32_t pad;
};

enum EpiMode : int32_t { EPI_NONE = 0, EPI_PAGERANK = 1 };

// Epilogue applied when a row's sum s is stored:
//   EPI_NONE:      y = s
//   EPI_PAGERANK:  y = d * s + tele
struct Epi {
    int32_t mode;
    int32_t pad;
    double d;
    double tele;
};

struct Thresholds {
    int32_t upper[NCLASS];  // inclusive upper row length per class
};

// Per-matrix launch plan (row classes and tile shapes).
struct Plan {
    int32_t upper[NCLASS];
    int32_t rpg[NCLASS];    // rows per lane group per tile
    int32_t chunk;          // non-zeros per split-row chunk
    int32_t grid_per_cu;    // persistent workgroups per compute unit
    int32_t layout;         // LAYOUT_AUTO, _ROWS, _PANELS, _HOT or _BAND
};

// Device layouts of a matrix for the product: the row-class tiles over the
// CSR arrays, or column panels (x staged in LDS one panel at a time).
enum : int32_t { LAYOUT_AUTO = -1, LAYOUT_ROWS = 0, LAYOUT_PANELS = 1, LAYOUT_HOT = 2,
                 LAYOUT_BAND = 3 };

// Column-panel layout: the columns are cut into panels of `pw` (a panel of
// x fits the LDS), the rows into blocks of `rb`.  Within row block b and
// panel p the entries are stored row by row (each row's entries in their
// CSR order), with the row inside the block and the column inside the panel
// packed into 32 bits, (row << 16) | col.  Each of the sixteen wavefronts of
// a workgroup owns `rw` consecutive rows of the block; wptr[(b*np + p)*17 + w]
// is where wavefront w's entries of panel p start (entry 16: the end).
struct PanelDesc {
    const void *vals;
    const uint32_t *rc;
    const int32_t *wptr;
    int32_t rows, cols;
    int32_t pw, np, rb, nblk, rw;
    int32_t pad;
};
// Vectors of one matrix in a grouped panel launch.
// dot: when set (float64 only), the blocks also write the partial sums of
// x_i * y_i over their rows (square matrices), one per row block, the
// product's fused dot of the single-matrix launch.
struct PanelIO {
    const void *x;
    void *y;
    double *dot = nullptr;
};
constexpr int kPanelThreads = 1024;            // 16 wave64: one workgroup per CU
constexpr int kPanelWaves = kPanelThreads / 64;
constexpr int kPanelMaxRb = 4096;              // rows per block (sums in LDS)
constexpr int kPanelLds = 160 * 1024;          // LDS of one workgroup
constexpr int kPanelChunks = 2;                // 128-entry chunks in flight
constexpr int kPanelMaxPanels = 64;            // one lane per panel in the build
constexpr int kPanelRotateBlocks = 128;        // blocks from which panel order rotates
// LDS bytes of the row sums of a block of rb rows (the x panel follows)
constexpr int panel_sum_bytes(int rb)
{
    return (rb * 8 + 15) & ~15;
}
// widest panel (elements) for a value size and rb rows per block
constexpr int panel_width(int vsize, int rb)
{
    return (kPanelLds - panel_sum_bytes(rb)) / vsize;
}

// Hot-column layout, for matrices whose most referenced columns come first
// (a graph relabelled by decreasing out-degree).  Columns [0, hot) are
// copied into LDS once per workgroup; the others are read from x in global
// memory.  Rows are cut into blocks of at most kHotRows non-empty rows and
// about the same number of entries; block b holds rows [brow[b], brow[b+1])
// and the entries [bent[b], bent[b+1]), its hot entries first (up to
// bsplit[b]), then its cold ones, each part row by row.  A row's key is its
// number among the non-empty rows of its block (rmap[row]; kHotEmpty for an
// empty row), so empty rows take no row sum.  A hot entry's word packs the
// key and the column, (key << 16) | col; a cold entry's word is its column
// and key[] holds its key.
struct HotDesc {
    const void *vals;
    const uint32_t *rc;
    const uint16_t *key;
    const uint16_t *rmap;    // [rows]: key of the row, kHotEmpty if it has no entries
    const int32_t *brow;     // [nblk + 1]
    const int32_t *bent;     // [nblk + 1]
    const int32_t *bsplit;   // [nblk]
    const int32_t *gptr;     // [grid + 1]: workgroup g takes blocks gblk[gptr[g] .. gptr[g+1])
    const int32_t *gblk;     // [nblk]
    int32_t rows, cols, nblk, hot, grid, pad;
};
constexpr int kHotRows = 1536;                        // non-empty rows per block
constexpr uint16_t kHotEmpty = 0xFFFF;                // rmap of an empty row
constexpr int kHotSpan = 16 * kHotRows;               // rows per block, empty ones too
constexpr int kHotLdsHead = 2 * kHotRows * 8 + 1024;  // hot and cold row sums + carries
// hot columns (elements) for a value size
constexpr int hot_width(int vsize)
{
    return ((kPanelLds - kHotLdsHead) / vsize) & ~63;
}

// Band layout, for matrices whose rows reach only nearby columns: the CSR
// order and values are kept, and each entry gets a 32-bit word
// (row inside its block << 16) | (column - cbase[b]).  Rows are cut into
// blocks of at most kBandRows rows, about the same number of entries, and
// a column span below 65536; block b holds rows [brow[b], brow[b+1]) and
// the entries [bent[b], bent[b+1]).
struct BandDesc {
    const void *vals;        // the CSR values
    const uint32_t *rc;      // [nnz + pad]
    const int32_t *brow;     // [nblk + 1]
    const int32_t *bent;     // [nblk + 1]
    const int32_t *cbase;    // [nblk]
    int32_t rows, cols, nblk, pad;
};
constexpr int kBandThreads = 256;
constexpr int kBandWaves = kBandThreads / 64;
constexpr int kBandRows = 2048;                            // rows per block
constexpr int kBandLds = kBandRows * 8 + kBandWaves * 12 + 16;

Plan default_plan();

struct CgState;      // device buffers + graph cache of a CG solve
struct PrState;      // graph cache of PageRank

struct CsrHandle {
    int32_t rows = 0, cols = 0;
    int32_t cols_given = -1;   // as passed at creation (-1: derived)
    int64_t nnz = 0;
    int32_t max_len = 0;         // longest row (set when constructed)
    lilac_dtype dt = LILAC_F64;
    unsigned flags = 0;
    // device copies
    int32_t *d_row_ptr = nullptr;
    int32_t *d_col = nullptr;
    void *d_vals = nullptr;
    // analysis
    int32_t *d_bin_rows = nullptr;
    int32_t *d_c_row = nullptr, *d_c_k0 = nullptr, *d_c_k1 = nullptr;
    int32_t *d_s_first = nullptr;
    double *d_chunk_part = nullptr;
    Tile *d_tiles = nullptr;
    double *d_dot_part = nullptr;   // one per persistent workgroup + finaliser
    // distinct 128-byte lines of x per non-zero in sampled groups of 64
    // rows (near 1: scattered columns; -1: not measured)
    double line_ratio = -1.0;
    // column-panel layout (when use_panels)
    bool use_panels = false;
    PanelDesc pan{};
    void *d_pv = nullptr;
    uint32_t *d_prc = nullptr;
    int32_t *d_pw = nullptr;
    // hot-column layout (when use_hot)
    bool use_hot = false;
    HotDesc hot{};
    void *d_hv = nullptr;
    uint32_t *d_hrc = nullptr;
    uint16_t *d_hkey = nullptr;
    uint16_t *d_hrmap = nullptr;    // rows: key of each row in its block
    int32_t *d_hb = nullptr;        // brow | bent | bsplit
    // band layout (when use_band)
    bool use_band = false;
    BandDesc band{};
    uint32_t *d_brc = nullptr;
    int32_t *d_bb = nullptr;        // brow | bent | cbase
    std::vector<int32_t> bin_off;   // NCLASS+1
    int64_t nchunks = 0;
    int32_t nsplit = 0;
    int32_t ntiles = 0;
    int32_t grid = 0;               // workgroups of the tile kernel
    int32_t fin_blocks = 0;         // workgroups of the finaliser
    Plan plan;
    // remembered host arrays (LILAC_KEEP_HOST or raw-call cache)
    const int32_t *h_row_ptr = nullptr, *h_col = nullptr;
    const void *h_vals = nullptr;
    bool dirty_struct = false, dirty_vals = false;
    int64_t dev_bytes = 0;
    CgState *cg = nullptr;
    PrState *pr = nullptr;
};

size_t dtype_size(lilac_dtype dt);

// Whether the product runs on a layout of its own (column panels or hot
// columns) rather than on the row-class tiles.
inline bool own_layout(const CsrHandle &h)
{
    return h.use_panels || h.use_hot || h.use_band;
}

// ---- errors ---------------------------------------------------------------
struct Error {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const std::string &msg);
void hip_check(hipError_t e, const char *what, const char *file, int line);
#define HIPC(x) ::lilac::hip_check((x), #x, __FILE__, __LINE__)

// ---- device memory with a byte budget -----------------------------------
// Every device allocation of the library goes through dev_alloc, which
// charges it to the library-wide budget (LILAC_HBM_BUDGET) and, when the
// calling thread has an account set, to that account and each of its
// parents; an allocation that would take any of them past its limit fails
// with LILAC_ERR_BUDGET and allocates nothing.  dev_free returns the bytes
// to the accounts charged at allocation, whichever thread frees.  Accounts
// are read and changed only under lib_mutex().
struct Account {
    int64_t limit = INT64_MAX;
    int64_t in_use = 0;
    int64_t peak = 0;
    Account *parent = nullptr;
};
// The calling thread's current account (nullptr: none).
Account *&thread_account();
void *dev_alloc(size_t bytes);
void dev_free(void *p);

// Temporaries of a handle build (freed before the build returns).  A thread
// that installs a TmpCache takes them from one grow-only buffer of at most
// `limit` bytes, charged to `acct`, so that its builds call no hipFree
// (which waits for every stream of the device); without one, or for a
// larger or second temporary, they are ordinary allocations.
struct TmpCache {
    void *p = nullptr;
    size_t cap = 0, limit = 0;
    bool busy = false;
    Account *acct = nullptr;
};
TmpCache *&thread_tmp_cache();
void *tmp_alloc(size_t bytes);
void tmp_free(void *p);
void tmp_cache_release(TmpCache &t);   // frees the buffer
int device_cu_count();

// ---- kernel launchers (kernels.hip) --------------------------------------
void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
void launch_fill_bytes_zero(void *p, int64_t bytes, hipStream_t s);
void launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
// HBM stream ceiling (read, or copy when dst is set) over bytes/16 pieces.
void launch_stream(const void *src, void *dst, int64_t bytes, int32_t groups,
                   uint32_t *sink, hipStream_t s);
void launch_validate(int32_t rows, const int32_t *rp, int64_t nnz,
                     const int32_t *col, int32_t cols_given, int32_t *status,
                     hipStream_t s);
void launch_bin_count(int32_t rows, const int32_t *rp, const Thresholds &th,
                      int32_t *hist, int32_t nblk, hipStream_t s);
// Exclusive prefix sum of a[0..n) in place; *total (if non-null) receives
// the sum.  Beyond 65536 elements it takes a temporary buffer and waits for
// the stream: analysis only, never inside a captured graph.
void launch_scan_excl(int32_t *a, int64_t n, int32_t *total, hipStream_t s);
void launch_bin_scatter(int32_t rows, const int32_t *rp, const Thresholds &th,
                        const int32_t *hist, int32_t nblk, int32_t *bin_rows,
                        hipStream_t s);
void launch_chunk_count(int32_t nsplit, const int32_t *split_rows,
                        const int32_t *rp, int32_t chunk, int32_t *cnt,
                        hipStream_t s);
void launch_chunk_fill(int32_t nsplit, const int32_t *split_rows,
                       const int32_t *rp, int32_t chunk, const int32_t *s_first,
                       int32_t *c_row, int32_t *c_k0, int32_t *c_k1,
                       hipStream_t s);

// Product over the tiles of one matrix (GROUPED = false, desc passed by
// value) or of many (desc table in device memory).  With dot_part non-null,
// workgroup g also writes dot_part[g] = sum over its rows of w[i]*y[i] and
// the finaliser writes dot_part[grid + b].
void launch_spmv_tiles(lilac_dtype dt, const Tile *tiles, int32_t ntiles,
                       int32_t grid, const MatDesc &single,
                       const MatDesc *mats, const Epi &epi, double *dot_part,
                       hipStream_t s);
// Column-panel product (see PanelDesc); dot_part (or null) receives one
// partial of sum w[i]*y[i] per workgroup.
void launch_spmv_panels(lilac_dtype dt, const PanelDesc &pd, const void *x,
                        void *y, const Epi &epi, const void *w, double *dot_part,
                        hipStream_t s);
void launch_panel_count(const PanelDesc &pd, const int32_t *rp,
                        const int32_t *col, int32_t *cnt, hipStream_t s);
void launch_panel_scatter(lilac_dtype dt, const PanelDesc &pd, const int32_t *rp,
                          const int32_t *col, const void *vals, const int32_t *ptr,
                          void *pv, uint32_t *prc, hipStream_t s);
void launch_panel_wptr(const PanelDesc &pd, const int32_t *ptr, int32_t *wptr,
                       hipStream_t s);
// Column-panel products of nmat matrices in one launch of nblocks
// workgroups: matrix j owns workgroups [prefix[j], prefix[j+1]).  Each
// result equals the single-matrix launch bit for bit.
void launch_spmv_panels_grouped(lilac_dtype dt, const PanelDesc *descs,
                                const PanelIO *io, const int32_t *prefix,
                                int32_t nmat, int32_t nblocks, hipStream_t s);
// Band product (see BandDesc): one workgroup per row block; dot_part (or
// null) receives one partial per block.
void launch_spmv_band(lilac_dtype dt, const BandDesc &bd, const void *x, void *y,
                      const Epi &epi, const void *w, double *dot_part, hipStream_t s);
// Band products of nmat matrices in one launch (as for column panels).
void launch_spmv_band_grouped(lilac_dtype dt, const BandDesc *descs, const PanelIO *io,
                              const int32_t *prefix, int32_t nmat, int32_t nblocks,
                              hipStream_t s);
// lo[i], hi[i] = smallest and largest column of row i (INT_MAX, -1 if empty).
void launch_row_span(int32_t rows, const int32_t *rp, const int32_t *col, int32_t *lo,
                     int32_t *hi, hipStream_t s);
void launch_band_pack(const BandDesc &bd, const int32_t *rp, const int32_t *col,
                      uint32_t *rc, hipStream_t s);
// For ngroups groups of 64 consecutive rows spread over the matrix:
// out[2g] = non-zeros looked at (at most 8192), out[2g+1] = distinct
// (col >> shift) among them, hashed into 16384 bins.
void launch_line_reuse(int32_t rows, const int32_t *rp, const int32_t *col,
                       int32_t ngroups, int32_t shift, int32_t *out, hipStream_t s);
// Lets the panel kernels use the whole LDS of a CU (once per process).
void panels_prepare();
// Hot-column product (see HotDesc): hd.grid persistent workgroups take the
// row blocks in turn; dot_part (or null) receives one partial per workgroup.
void launch_spmv_hot(lilac_dtype dt, const HotDesc &hd, const void *x, void *y,
                     const Epi &epi, const void *w, double *dot_part, hipStream_t s);
// cnt[r] = entries of row r with a column below hd.hot.
void launch_hot_count(const HotDesc &hd, const int32_t *rp, const int32_t *col,
                      int32_t *cnt, hipStream_t s);
// bsplit from the block bounds and the exclusive scan hx of the hot counts.
void launch_hot_split(const HotDesc &hd, const int32_t *hx, int32_t *bsplit,
                      hipStream_t s);
void launch_hot_scatter(lilac_dtype dt, const HotDesc &hd, const int32_t *rp,
                        const int32_t *col, const void *vals, const int32_t *hx,
                        void *hv, uint32_t *hrc, uint16_t *hkey, hipStream_t s);
// Finaliser for split rows: single matrix (items == null, n = nsplit) or a
// list of (matrix, split row) items for grouped launches.
void launch_split_finalize(lilac_dtype dt, const int32_t *items, int32_t n,
                           const MatDesc &single, const MatDesc *mats,
                           const Epi &epi, double *dot_part, hipStream_t s);

// Product over several matrices whose own tile lists are concatenated
// virtually: tile v belongs to matrix j with prefix[j] <= v < prefix[j+1].
void launch_spmv_segments(lilac_dtype dt, const MatDesc *mats,
                          const int32_t *prefix, int32_t nseg, int32_t total,
                          int32_t grid, hipStream_t s);

// Many CG solves advanced together, one iteration per call sequence, in
// the Chronopoulos-Gear arrangement of the single-matrix solve: init once
// (x = 0, r = b, p = s = 0), then after each product w = A r the partial
// sums of r.w (rw) and one step that forms beta, alpha and updates
// p = r + beta p, s = w + beta s, x += alpha p, r -= alpha s.
struct CgSeg {
    const double *b;
    double *x, *r, *p, *w, *s;
    double *rw_part;    // nb partial sums of r.w
    double *rr_part;    // 2*nb partial sums of r.r (by iteration parity)
    double *sc;         // gamma[2], alpha[2] (by iteration parity)
    int32_t *done;      // set once the solve stopped (gamma or p.Ap zero)
    int64_t n;
    int32_t nb;         // workgroups of this solve (fixed by n)
    int32_t iter;       // iteration index k of this step
    int32_t blk0;       // first workgroup of this solve in the launch
    int32_t nrw;        // r.w partials the product wrote (0: k_cgb_rw writes nb)
};
int32_t cg_seg_blocks(int64_t n);
void launch_cgb_init(const CgSeg *segs, int32_t nseg, int32_t blocks, hipStream_t s);
void launch_cgb_rw(const CgSeg *segs, int32_t nseg, int32_t blocks, hipStream_t s);
void launch_cgb_step(const CgSeg *segs, int32_t nseg, int32_t blocks, hipStream_t s);

void launch_dot_parts(int64_t n, const double *a, const double *b,
                      double *part, int32_t nparts, hipStream_t s);
void launch_dot_parts_f32(int64_t n, const float *a, const float *b,
                          double *part, int32_t nparts, hipStream_t s);

// One level of a breadth-first search as a Boolean product over the tiles:
// every row v with level[v] == -1 that has a column u with level[u] == depth
// gets level depth+1; *changed is set to 1 if any row did.
void launch_bfs_step(const Tile *tiles, int32_t ntiles, int32_t grid,
                     const MatDesc &m, int32_t *level, int32_t depth,
                     int32_t *changed, hipStream_t s);

// Relabelling of a graph's vertices by decreasing out-degree (locality of the
// gathered vector): deg[u] = entries in column u; key = bucket of deg
// (powers of two, largest first); newid = stable position by key.
void launch_count_cols(int64_t nnz, const int32_t *col, int32_t *deg, hipStream_t s);
void launch_degree_keys(int32_t n, const int32_t *deg, int32_t *key, hipStream_t s);
constexpr int kDegKeys = 33;
void launch_key_hist(int32_t n, const int32_t *key, int32_t *hist, int32_t nblk,
                     hipStream_t s);
void launch_key_scatter(int32_t n, const int32_t *key, const int32_t *hist,
                        int32_t nblk, int32_t *newid, hipStream_t s);
// Permuted copy: row newid[v] of the output is row v of the input with its
// columns renamed by newid (entries keep their order).
void launch_perm_lengths(int32_t rows, const int32_t *rp, const int32_t *newid,
                         int32_t *len2, hipStream_t s);
void launch_perm_entries(lilac_dtype dt, int32_t rows, int64_t nnz, const int32_t *rp,
                         const int32_t *col, const void *vals, const int32_t *newid,
                         const int32_t *rp2, int32_t *col2, void *vals2, hipStream_t s);
// out[newid[v]] = in[v] (to = true) or out[v] = in[newid[v]] (to = false)
void launch_permute_f32(int32_t n, const int32_t *newid, const float *in, float *out,
                        bool to, hipStream_t s);

// Jagged Diagonal Storage product, every sum in diagonal order without
// contraction (bitwise equal to the sequential definition).
void launch_spmv_jds(int32_t rows, int32_t max_len, int32_t nnz,
                     const int32_t *iperm, const int32_t *nzcnt,
                     const int32_t *jd_ptr, const int32_t *jd_col,
                     const double *jd_val, const double *x, double *y,
                     hipStream_t s);
void launch_invert_perm(int32_t rows, const int32_t *perm, int32_t *iperm,
                        hipStream_t s);
void launch_sum_parts(const double *part, int32_t nparts, double *out,
                      hipStream_t s);
void launch_sum_parts_f32(const double *part, int32_t nparts, float *out,
                          hipStream_t s);
void launch_copy_f64(int64_t n, const double *src, double *dst, hipStream_t s);
void launch_copy_f32(int64_t n, const float *src, float *dst, hipStream_t s);

// CG building blocks (device scalars in `CgScalars`)
struct CgScalars {
    double rho;                 // r.r (of the final residual, or at the stop)
    double gamma[2], alpha[2];  // r.r and alpha of the last two iterations
    int32_t done, iters;
};
// A conjugate gradient solve is k_cg_init, then per iteration the product
// w = A r with the w.r partials fused into it and k_cg_step, then
// k_cg_final (see kernels.hip).  rr holds r.r partials for two parities
// (kDotParts each), so no partial is written by one workgroup while others
// read it.
void launch_cg_init(int64_t n, const double *b, double *x, double *r, double *p,
                    double *sv, double *rr, int32_t nparts, CgScalars *sc, hipStream_t s);
void launch_cg_step(int64_t n, CgScalars *sc, const double *w, double *p, double *sv,
                    double *x, double *r, const double *dot_part, int32_t ndot, double *rr,
                    int32_t nparts, int32_t k, hipStream_t s);
void launch_cg_final(CgScalars *sc, const double *rr, int32_t nparts, int32_t par,
                     hipStream_t s);
int32_t blas1_parts(int64_t n);
// Workgroups of the tile kernel resident per compute unit.
int occupancy_tiles(lilac_dtype dt);
bool is_device_ptr(const void *p);

// ---- runtime services shared with the request server ----------------------
std::recursive_mutex &lib_mutex();
void set_last_error(const std::string &msg);
int lib_device();
// inputs_ready: device inputs are complete (the caller synchronised the
// stream that wrote them), so no device-wide wait is needed.
CsrHandle *create_handle(int rows, int cols, int64_t nnz, const int32_t *rp,
                         const int32_t *col, const void *vals, lilac_dtype dt,
                         unsigned flags, bool inputs_ready = false);
// A handle that takes over device arrays allocated with dev_alloc and
// already holding the matrix: rp[rows+1], col and vals with room for
// padded_nnz(nnz) entries.  They belong to the handle from the call on
// (freed with it, also when the call fails).  Blocking.
int64_t padded_nnz(int64_t nnz);
// The checks and the analysis run on stream s (null: the library's stream).
CsrHandle *create_handle_adopt(int rows, int cols, int64_t nnz, int32_t *rp,
                               int32_t *col, void *vals, lilac_dtype dt,
                               hipStream_t s = nullptr);
void destroy_handle(CsrHandle *h);
MatDesc make_desc(const CsrHandle &h, const void *x, void *y, const void *w,
                  double *chunk_part);
void spmv_enqueue(const CsrHandle &h, const void *x, void *y, const Epi &epi,
                  const void *w, bool dot, hipStream_t s);
void run_cg(CsrHandle &h, const double *b, double *x, int iters,
            unsigned flags, hipStream_t s, double *rho_out, int *iters_done);
// Allocates the handle's CG state now (otherwise done on the first solve).
void handle_cg_prepare(CsrHandle &h);
int tile_grid(lilac_dtype dt);   // persistent workgroups for a grouped launch

// ---- CSR -> JDS (jds.hip) ---------------------------------------------------
// Longest row of the handle's matrix (d_tmp: one device int of scratch).
// Blocking.
int32_t jds_max_len(const CsrHandle &h, int32_t *d_tmp, hipStream_t s);
// The JDS arrays of the handle's matrix into device outputs perm[rows],
// nzcnt[rows], jd_ptr[max_len+1], jd_col[nnz], jd_val[nnz] (handle's dtype).
// Blocking.
void jds_convert(const CsrHandle &h, int32_t max_len, int32_t *perm, int32_t *nzcnt,
                 int32_t *jd_ptr, int32_t *jd_col, void *jd_val, hipStream_t s);

}  // namespace lilac

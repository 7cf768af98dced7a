// Host runtime of liblilac.so: library context, device memory with a byte
// budget, CSR handles (upload, validation, analysis, work tiles), the raw
// pointer marshaling cache, CG and PageRank drivers (captured as HIP graphs),
// grouped batched products, the autotuner and the C ABI entry points.
#include <algorithm>
#include <queue>
#include <type_traits>
#include <cctype>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "lilac_internal.h"
#include "marshal.h"

namespace lilac {

// ===================================================================== errors

static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }

void fail(int code, const std::string &msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char *what, const char *file, int line)
{
    if (e == hipSuccess)
        return;
    const int code = (e == hipErrorOutOfMemory) ? LILAC_ERR_OOM : LILAC_ERR_DEVICE;
    const char *f = std::strrchr(file, '/');
    fail(code, std::string(what) + ": " + hipGetErrorString(e) + " (" +
                   (f ? f + 1 : file) + ":" + std::to_string(line) + ")");
}

size_t dtype_size(lilac_dtype dt) { return dt == LILAC_F32 ? 4 : 8; }

// ==================================================================== context

// The library's persistent state: the paper's PersistentVariables, created
// by the first call (BeforeFirstExecution) and torn down by lilac_finalize
// or at exit (AfterLastExecution).
struct Context {
    int device = -1;
    int cu = 0;
    hipStream_t stream = nullptr;   // the library's own stream
    hipStream_t cap = nullptr;      // stream used only for graph capture
    int64_t budget = INT64_MAX;
    int64_t in_use = 0;
    struct Charge {
        size_t bytes;
        Account *acct;
    };
    std::unordered_map<void *, Charge> sizes;
    // scratch for the raw calls
    void *x_buf = nullptr, *y_buf = nullptr;
    size_t x_cap = 0, y_cap = 0;
    double *dot_part = nullptr;     // kDotParts + 1 (result)
    double *dot_a = nullptr, *dot_b = nullptr;
    size_t dot_cap = 0;
    int32_t *status = nullptr;      // 2 ints for validation
    int32_t *total = nullptr;       // 1 int for scans
    int occ[2] = {0, 0};            // tile-kernel workgroups per CU (f64, f32)
};

static std::recursive_mutex g_mu;
std::recursive_mutex &lib_mutex() { return g_mu; }
static Context *g_ctx = nullptr;
static bool g_exit_registered = false;

static int64_t parse_bytes(const char *s)
{
    char *end = nullptr;
    double v = std::strtod(s, &end);
    if (end && *end) {
        switch (*end) {
        case 'k': case 'K': v *= 1024.0; break;
        case 'm': case 'M': v *= 1024.0 * 1024.0; break;
        case 'g': case 'G': v *= 1024.0 * 1024.0 * 1024.0; break;
        case 't': case 'T': v *= 1024.0 * 1024.0 * 1024.0 * 1024.0; break;
        default: break;
        }
    }
    return v > 0 ? (int64_t)v : INT64_MAX;
}

void release_all_raw();
void release_group_plans();
void tune_cache_load();

static void at_exit_hook()
{
    // Host-side tear-down only: the device memory goes with the process, and
    // HIP calls from exit handlers can race the runtime's own shutdown.
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    marshal_reset();
}

static char *scratch_on_current_device();

static Context &init_ctx(int device)
{
    if (g_ctx)
        return *g_ctx;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        fail(LILAC_ERR_DEVICE, "no HIP device available");
    }
    auto *c = new Context();
    if (device < 0)
        HIPC(hipGetDevice(&device));
    if (device >= ndev) {
        delete c;
        fail(LILAC_ERR_ARG, "device index out of range");
    }
    HIPC(hipSetDevice(device));
    c->device = device;
    hipDeviceProp_t prop;
    HIPC(hipGetDeviceProperties(&prop, device));
    c->cu = prop.multiProcessorCount;
    HIPC(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIPC(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    (void)scratch_on_current_device();  // the fixed CG state's address
    if (const char *b = std::getenv("LILAC_HBM_BUDGET"))
        c->budget = parse_bytes(b);
    g_ctx = c;
    c->status = (int32_t *)dev_alloc(2 * sizeof(int32_t));
    c->total = (int32_t *)dev_alloc(sizeof(int32_t));
    c->dot_part = (double *)dev_alloc((kDotParts + 1) * sizeof(double));
    if (!g_exit_registered) {
        std::atexit(at_exit_hook);
        g_exit_registered = true;
    }
    tune_cache_load();
    return *c;
}

static Context &ctx()
{
    if (!g_ctx)
        return init_ctx(-1);
    return *g_ctx;
}

int device_cu_count() { return ctx().cu; }
int lib_device() { return ctx().device; }

Account *&thread_account()
{
    static thread_local Account *a = nullptr;
    return a;
}

void *dev_alloc(size_t bytes)
{
    std::lock_guard<std::recursive_mutex> lk(g_mu);
    Context &c = *g_ctx;
    if (bytes == 0)
        bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    if (c.in_use + (int64_t)bytes > c.budget)
        fail(LILAC_ERR_BUDGET, "allocation of " + std::to_string(bytes) +
                                   " bytes exceeds the HBM budget (" +
                                   std::to_string(c.in_use) + " of " +
                                   std::to_string(c.budget) + " in use)");
    Account *acct = thread_account();
    for (Account *a = acct; a; a = a->parent)
        if (a->in_use + (int64_t)bytes > a->limit)
            fail(LILAC_ERR_BUDGET, "allocation of " + std::to_string(bytes) +
                                       " bytes exceeds an account's limit (" +
                                       std::to_string(a->in_use) + " of " +
                                       std::to_string(a->limit) + " in use)");
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(LILAC_ERR_OOM, "hipMalloc of " + std::to_string(bytes) +
                                " bytes failed: " + hipGetErrorString(e));
    }
    c.sizes[p] = Context::Charge{bytes, acct};
    c.in_use += (int64_t)bytes;
    for (Account *a = acct; a; a = a->parent) {
        a->in_use += (int64_t)bytes;
        a->peak = std::max(a->peak, a->in_use);
    }
    return p;
}

void dev_free(void *p)
{
    if (!p || !g_ctx)
        return;
    {
        std::lock_guard<std::recursive_mutex> lk(g_mu);
        Context &c = *g_ctx;
        auto it = c.sizes.find(p);
        if (it != c.sizes.end()) {
            c.in_use -= (int64_t)it->second.bytes;
            for (Account *a = it->second.acct; a; a = a->parent)
                a->in_use -= (int64_t)it->second.bytes;
            c.sizes.erase(it);
        }
    }
    // waits for outstanding work on the device, so not under the lock:
    // other threads keep allocating meanwhile
    (void)hipFree(p);
}

TmpCache *&thread_tmp_cache()
{
    static thread_local TmpCache *t = nullptr;
    return t;
}

void *tmp_alloc(size_t bytes)
{
    TmpCache *t = thread_tmp_cache();
    bytes = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    if (!t || t->busy || bytes > t->limit)
        return dev_alloc(bytes);
    if (t->cap < bytes) {
        // grow to the next MiB (at most the limit); the old buffer is idle
        const size_t want = std::min(t->limit, (bytes + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1));
        Account *saved = thread_account();
        thread_account() = t->acct;
        try {
            dev_free(t->p);
            t->p = nullptr;
            t->cap = 0;
            t->p = dev_alloc(want);
            t->cap = want;
        } catch (...) {
            thread_account() = saved;
            throw;
        }
        thread_account() = saved;
    }
    t->busy = true;
    return t->p;
}

void tmp_free(void *p)
{
    TmpCache *t = thread_tmp_cache();
    if (t && p && p == t->p && t->busy) {
        t->busy = false;
        return;
    }
    dev_free(p);
}

void tmp_cache_release(TmpCache &t)
{
    dev_free(t.p);
    t.p = nullptr;
    t.cap = 0;
    t.busy = false;
}

template <typename T>
static void dev_free_reset(T *&p)
{
    dev_free((void *)p);
    p = nullptr;
}

bool is_device_ptr(const void *p)
{
    if (!p)
        return false;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

static void copy_in(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    if (bytes == 0)
        return;
    HIPC(hipMemcpyAsync(dst, src, bytes,
                        is_device_ptr(src) ? hipMemcpyDeviceToDevice
                                           : hipMemcpyHostToDevice,
                        s));
}

static int tile_occupancy(lilac_dtype dt);

// ============================================================ plan / tiles

// Persistent workgroups of the tile kernel per CU by default: four ran
// faster than eight or more on every matrix shape measured (long and short
// rows, local and scattered columns), and than two or three.
constexpr int kTileGroupsPerCu = 4;

// Default row classes: two non-zeros per lane where a lane loads single
// elements (groups of 1 to 4 lanes), eight where it loads 16-byte vectors
// (8 to 32 lanes: rows of up to 64, 128 and 256), more rows in flight per
// wavefront than one or two vectors per lane give.
Plan default_plan()
{
    Plan p;
    const int32_t up[NCLASS] = {2, 4, 8, 64, 128, 256, 1024, 8192, INT_MAX};
    const int32_t rpg[NCLASS] = {1, 1, 1, 1, 1, 1, 2, 1, 1};
    for (int c = 0; c < NCLASS; ++c) {
        p.upper[c] = up[c];
        p.rpg[c] = rpg[c];
    }
    p.chunk = 4096;
    p.grid_per_cu = kTileGroupsPerCu;
    p.layout = LAYOUT_AUTO;
    return p;
}

static void check_plan(const Plan &p)
{
    for (int c = 0; c + 1 < NCLASS - 1; ++c)
        if (p.upper[c] > p.upper[c + 1])
            fail(LILAC_ERR_ARG, "class bounds must be non-decreasing");
    if (p.upper[0] < 0)
        fail(LILAC_ERR_ARG, "class bounds must be >= 0");
    static const int lanes[NCLASS] = {1, 2, 4, 8, 16, 32, 64, 64, 1};
    for (int c = 0; c < NCLASS; ++c)
        if (p.rpg[c] < 1 || p.rpg[c] > lanes[c])
            fail(LILAC_ERR_ARG, "rows per group must be in [1, lanes of the class]"
                                " (one for the single-lane and split classes)");
    if (p.chunk < 256 || p.chunk > (1 << 24))
        fail(LILAC_ERR_ARG, "chunk must be in [256, 2^24]");
    if (p.grid_per_cu < 1 || p.grid_per_cu > 32)
        fail(LILAC_ERR_ARG, "grid_per_cu must be in [1, 32]");
    if (p.layout < LAYOUT_AUTO || p.layout > LAYOUT_BAND)
        fail(LILAC_ERR_ARG, "unknown layout");
}

static const int kLanes[NCLASS] = {1, 2, 4, 8, 16, 32, 64, kBlock, kBlock};

struct HandleExtra {
    std::vector<Tile> tiles;   // host copy of the handle's tile list
};
static std::unordered_map<const CsrHandle *, HandleExtra> g_extra;

static void free_analysis(CsrHandle &h)
{
    dev_free_reset(h.d_bin_rows);
    dev_free_reset(h.d_c_row);
    dev_free_reset(h.d_c_k0);
    dev_free_reset(h.d_c_k1);
    dev_free_reset(h.d_s_first);
    dev_free_reset(h.d_chunk_part);
    dev_free_reset(h.d_tiles);
    dev_free_reset(h.d_dot_part);
    dev_free_reset(h.d_pv);
    dev_free_reset(h.d_prc);
    dev_free_reset(h.d_pw);
    dev_free_reset(h.d_hv);
    dev_free_reset(h.d_hrc);
    dev_free_reset(h.d_hkey);
    dev_free_reset(h.d_hrmap);
    dev_free_reset(h.d_hb);
    dev_free_reset(h.d_brc);
    dev_free_reset(h.d_bb);
    h.use_band = false;
    h.band = BandDesc{};
    h.use_panels = false;
    h.pan = PanelDesc{};
    h.use_hot = false;
    h.hot = HotDesc{};
    h.ntiles = 0;
    h.nchunks = 0;
    h.nsplit = 0;
    h.grid = 0;
    h.fin_blocks = 0;
}

static int64_t analysis_bytes(const CsrHandle &h)
{
    int64_t b = (int64_t)h.rows * 4 + h.nchunks * (3 * 4 + 8) +
                (int64_t)(h.nsplit + 1) * 4 + (int64_t)h.ntiles * sizeof(Tile) +
                (int64_t)(h.grid + h.fin_blocks) * 8;
    if (h.use_panels)
        b += (h.nnz + kPad) * ((int64_t)dtype_size(h.dt) + 4) +
             (int64_t)h.pan.nblk * h.pan.np * (kPanelWaves + 1) * 4;
    if (h.use_hot)
        b += (h.nnz + kPad) * ((int64_t)dtype_size(h.dt) + 6) + (int64_t)h.rows * 2 +
             (int64_t)(4 * h.hot.nblk + h.hot.grid + 3) * 4;
    if (h.use_band)
        b += (h.nnz + kPad) * 4 + (int64_t)(3 * h.band.nblk + 2) * 4;
    return b;
}

static int32_t panel_rows(const CsrHandle &h);
// Columns per panel: a panel of x and the row sums of a block fill the LDS.
static int32_t panel_cols(const CsrHandle &h)
{
    return panel_width((int)dtype_size(h.dt), panel_rows(h));
}
static int64_t panel_count(const CsrHandle &h)
{
    return h.cols > 0 ? ((int64_t)h.cols + panel_cols(h) - 1) / panel_cols(h) : 0;
}

// Rows per block of the column-panel layout: enough blocks for every CU,
// but at least as many rows as make up the bytes of one copy of x (each
// block copies all of x into LDS once), and at most kPanelMaxRb.
static int32_t panel_rows(const CsrHandle &h)
{
    if (h.rows == 0)
        return 1;
    const double vs = (double)dtype_size(h.dt);
    const double row_bytes = std::max(1.0, (double)h.nnz / h.rows * (vs + 4.0));
    const int64_t by_cu = ((int64_t)h.rows + device_cu_count() - 1) / device_cu_count();
    const int64_t by_x = (int64_t)std::ceil((double)h.cols * vs / row_bytes);
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(kPanelMaxRb, std::max(by_cu, by_x)));
}

// A matrix is gather-heavy when its non-zeros touch nearly one distinct
// cache line of x each (scattered columns): then the row-class tiles are
// bound by the gathers, and copying x through LDS pays.
constexpr double kGatherHeavy = 0.3;
// Smallest matrix given the column-panel or band layout automatically;
// smaller ones stay on the row-class tiles (one grouped launch takes them
// all in a batch).
constexpr int64_t kOwnLayoutMinNnz = 16384;

// Whether the column-panel layout suits the matrix: gather-heavy, at most
// 64 panels, no row longer than the wavefront class (1024), and the copies
// of x (one per row block, served from L2) at most four times the matrix
// bytes.  Other matrices stay on the row-class tiles.
static bool panels_eligible(const CsrHandle &h)
{
    if (h.rows == 0 || h.nnz < kOwnLayoutMinNnz)
        return false;
    const int64_t np = panel_count(h);
    if (np < 1 || np > kPanelMaxPanels)
        return false;
    if (h.bin_off[NCLASS] - h.bin_off[C_W64 + 1] > 0)
        return false;  // rows longer than the wavefront class bound
    if (h.line_ratio < kGatherHeavy)
        return false;
    const double vs = (double)dtype_size(h.dt);
    const int32_t rb = panel_rows(h);
    const double nblk = std::ceil((double)h.rows / rb);
    const double stage = nblk * (double)h.cols * vs;
    return stage <= 4.0 * (double)h.nnz * (vs + 4.0);
}

// Distinct x lines per non-zero over up to 256 sampled groups of 64 rows.
static double measure_line_ratio(const CsrHandle &h, hipStream_t s)
{
    if (h.rows == 0 || h.nnz == 0)
        return 0.0;
    const int32_t ngroups = (int32_t)std::min<int64_t>(256, ((int64_t)h.rows + 63) / 64);
    int32_t *d = (int32_t *)tmp_alloc((size_t)ngroups * 8);
    std::vector<int32_t> out((size_t)ngroups * 2);
    try {
        launch_line_reuse(h.rows, h.d_row_ptr, h.d_col, ngroups,
                          h.dt == LILAC_F64 ? 4 : 5, d, s);
        HIPC(hipMemcpyAsync(out.data(), d, out.size() * 4, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
    } catch (...) {
        tmp_free(d);
        throw;
    }
    tmp_free(d);
    int64_t e = 0, l = 0;
    for (int32_t g = 0; g < ngroups; ++g) {
        e += out[2 * g];
        l += out[2 * g + 1];
    }
    return e > 0 ? (double)l / (double)e : 0.0;
}

static int64_t scan_total(int32_t *a, int64_t n, hipStream_t s);

// Builds the column-panel copy of the matrix (see PanelDesc).
static void build_panels(CsrHandle &h, hipStream_t s)
{
    PanelDesc pd{};
    pd.rows = h.rows;
    pd.cols = h.cols;
    pd.pw = panel_cols(h);
    pd.np = (int32_t)panel_count(h);
    if (pd.np < 1 || pd.np > kPanelMaxPanels)
        fail(LILAC_ERR_DEVICE, "column-panel layout needs 1 to 64 panels");
    panels_prepare();
    pd.rb = panel_rows(h);
    pd.nblk = (int32_t)((h.rows + pd.rb - 1) / pd.rb);
    pd.rw = (pd.rb + kPanelWaves - 1) / kPanelWaves;
    const int64_t nptr = (int64_t)pd.nblk * pd.np * (pd.rb + 1);
    int32_t *ptr = (int32_t *)tmp_alloc((size_t)nptr * 4);
    try {
        launch_fill_i32(ptr, nptr, 0, s);
        launch_panel_count(pd, h.d_row_ptr, h.d_col, ptr, s);
        const int64_t total = scan_total(ptr, nptr, s);
        if (total != h.nnz)
            fail(LILAC_ERR_DEVICE, "panel layout lost entries");
        const size_t vs = dtype_size(h.dt);
        h.d_pv = dev_alloc((size_t)(h.nnz + kPad) * vs);
        h.d_prc = (uint32_t *)dev_alloc((size_t)(h.nnz + kPad) * 4);
        launch_fill_bytes_zero((char *)h.d_pv + h.nnz * vs, kPad * vs, s);
        launch_fill_bytes_zero((char *)(h.d_prc + h.nnz), kPad * 4, s);
        launch_panel_scatter(h.dt, pd, h.d_row_ptr, h.d_col, h.d_vals, ptr, h.d_pv,
                             h.d_prc, s);
        const int64_t nw = (int64_t)pd.nblk * pd.np * (kPanelWaves + 1);
        h.d_pw = (int32_t *)dev_alloc((size_t)nw * 4);
        launch_panel_wptr(pd, ptr, h.d_pw, s);
        HIPC(hipStreamSynchronize(s));
    } catch (...) {
        tmp_free(ptr);
        throw;
    }
    tmp_free(ptr);
    pd.vals = h.d_pv;
    pd.rc = h.d_prc;
    pd.wptr = h.d_pw;
    h.pan = pd;
    h.use_panels = true;
}

// Whether the hot-column layout can be built: it needs entries.
static bool hot_possible(const CsrHandle &h)
{
    return h.rows > 0 && h.nnz > 0 && h.cols > 0;
}

// Builds the hot-column copy of the matrix (see HotDesc).  Block bounds and
// row keys are chosen on the host from row_ptr: a new block starts before a
// non-empty row when the current one has kHotRows non-empty rows, or when it
// has at least one workgroup's share of the entries or kHotSpan rows (few,
// large blocks cost the fewest barriers; the assignment below balances
// them).  Empty rows take no key, so a block of a graph's sparse tail
// (where most rows are empty) spans more rows than kHotRows.
static void build_hot(CsrHandle &h, hipStream_t s)
{
    Context &c = ctx();
    HotDesc hd{};
    hd.rows = h.rows;
    hd.cols = h.cols;
    hd.hot = std::min<int32_t>(h.cols, hot_width((int)dtype_size(h.dt)));
    panels_prepare();
    std::vector<int32_t> rp((size_t)h.rows + 1);
    HIPC(hipMemcpyAsync(rp.data(), h.d_row_ptr, rp.size() * 4, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    const int64_t target = std::max<int64_t>(16384, h.nnz / (int64_t)c.cu);
    std::vector<int32_t> brow{0};
    std::vector<uint16_t> rmap((size_t)h.rows);
    int32_t start = 0, keys = 0;
    for (int32_t r = 0; r < h.rows; ++r) {
        const bool filled = rp[r + 1] > rp[r];
        if (r > start && ((filled && keys >= kHotRows) || r - start >= kHotSpan ||
                          (int64_t)rp[r] - rp[start] >= target)) {
            brow.push_back(r);
            start = r;
            keys = 0;
        }
        rmap[r] = filled ? (uint16_t)keys++ : kHotEmpty;
    }
    brow.push_back(h.rows);
    hd.nblk = (int32_t)brow.size() - 1;
    hd.grid = std::min<int32_t>(hd.nblk, c.cu);
    // blocks to workgroups: longest first, each to the least loaded
    // workgroup so far (work = entries + rows), then each workgroup's blocks
    // in ascending order.  Blocks differ a lot (the densest rows come first
    // after relabelling), so taking every grid-th block leaves some
    // workgroups a quarter more work than the mean.
    std::vector<int32_t> owner((size_t)hd.nblk);
    {
        auto work = [&](int32_t b) {
            return (int64_t)rp[brow[b + 1]] - rp[brow[b]] + (brow[b + 1] - brow[b]);
        };
        std::vector<int32_t> order((size_t)hd.nblk);
        for (int32_t b = 0; b < hd.nblk; ++b)
            order[b] = b;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return work(a) > work(b); });
        typedef std::pair<int64_t, int32_t> Load;   // (work so far, workgroup)
        std::priority_queue<Load, std::vector<Load>, std::greater<Load>> least;
        for (int32_t g = 0; g < hd.grid; ++g)
            least.push(Load(0, g));
        for (int32_t b : order) {
            Load l = least.top();
            least.pop();
            owner[b] = l.second;
            l.first += work(b);
            least.push(l);
        }
    }
    const size_t nb1 = (size_t)hd.nblk + 1;
    std::vector<int32_t> hb(3 * nb1 - 1 + (size_t)hd.grid + 1 + hd.nblk);
    for (int32_t b = 0; b <= hd.nblk; ++b) {
        hb[b] = brow[b];
        hb[nb1 + b] = rp[brow[b]];
    }
    int32_t *gptr = hb.data() + 3 * nb1 - 1;
    int32_t *gblk = gptr + hd.grid + 1;
    for (int32_t b = 0; b < hd.nblk; ++b)
        ++gptr[owner[b] + 1];
    for (int32_t g = 0; g < hd.grid; ++g)
        gptr[g + 1] += gptr[g];
    {
        std::vector<int32_t> fill(gptr, gptr + hd.grid);
        for (int32_t b = 0; b < hd.nblk; ++b)
            gblk[fill[owner[b]]++] = b;
    }
    h.d_hb = (int32_t *)dev_alloc(hb.size() * 4);
    HIPC(hipMemcpyAsync(h.d_hb, hb.data(), hb.size() * 4, hipMemcpyHostToDevice, s));
    h.d_hrmap = (uint16_t *)dev_alloc(rmap.size() * 2);
    HIPC(hipMemcpyAsync(h.d_hrmap, rmap.data(), rmap.size() * 2, hipMemcpyHostToDevice, s));
    hd.rmap = h.d_hrmap;
    hd.brow = h.d_hb;
    hd.bent = h.d_hb + nb1;
    int32_t *bsplit = h.d_hb + 2 * nb1;
    hd.bsplit = bsplit;
    hd.gptr = h.d_hb + 3 * nb1 - 1;
    hd.gblk = hd.gptr + hd.grid + 1;
    int32_t *hx = (int32_t *)tmp_alloc((size_t)(h.rows + 1) * 4);
    try {
        launch_fill_i32(hx + h.rows, 1, 0, s);
        launch_hot_count(hd, h.d_row_ptr, h.d_col, hx, s);
        scan_total(hx, (int64_t)h.rows + 1, s);
        launch_hot_split(hd, hx, bsplit, s);
        const size_t vs = dtype_size(h.dt);
        h.d_hv = dev_alloc((size_t)(h.nnz + kPad) * vs);
        h.d_hrc = (uint32_t *)dev_alloc((size_t)(h.nnz + kPad) * 4);
        h.d_hkey = (uint16_t *)dev_alloc((size_t)(h.nnz + kPad) * 2);
        launch_fill_bytes_zero((char *)h.d_hv + h.nnz * vs, kPad * vs, s);
        launch_fill_bytes_zero((char *)(h.d_hrc + h.nnz), kPad * 4, s);
        // keys of hot entries are never used; keep every byte defined
        launch_fill_bytes_zero(h.d_hkey, (h.nnz + kPad) * 2, s);
        launch_hot_scatter(h.dt, hd, h.d_row_ptr, h.d_col, h.d_vals, hx, h.d_hv,
                           h.d_hrc, h.d_hkey, s);
        HIPC(hipStreamSynchronize(s));
    } catch (...) {
        tmp_free(hx);
        throw;
    }
    tmp_free(hx);
    hd.vals = h.d_hv;
    hd.rc = h.d_hrc;
    hd.key = h.d_hkey;
    h.hot = hd;
    h.use_hot = true;
}

// Builds the band copy of the matrix (see BandDesc) if every row spans
// fewer than 65536 columns; returns whether it did.  Block bounds are chosen
// on the host: a new block starts when the current one has kBandRows rows,
// `target` entries or more, or would span 65536 columns or more.
// Fewest non-zeros per band block, on average, for the automatic choice.
constexpr int64_t kBandMinEntries = 1024;

static bool build_band(CsrHandle &h, hipStream_t s, bool automatic)
{
    if (h.rows == 0 || h.nnz == 0)
        return false;
    std::vector<int32_t> lo((size_t)h.rows), hi((size_t)h.rows), rp((size_t)h.rows + 1);
    int32_t *d = (int32_t *)tmp_alloc((size_t)h.rows * 8);
    try {
        launch_row_span(h.rows, h.d_row_ptr, h.d_col, d, d + h.rows, s);
        HIPC(hipMemcpyAsync(lo.data(), d, (size_t)h.rows * 4, hipMemcpyDeviceToHost, s));
        HIPC(hipMemcpyAsync(hi.data(), d + h.rows, (size_t)h.rows * 4,
                            hipMemcpyDeviceToHost, s));
        HIPC(hipMemcpyAsync(rp.data(), h.d_row_ptr, rp.size() * 4, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
    } catch (...) {
        tmp_free(d);
        throw;
    }
    tmp_free(d);
    // about eight blocks per CU (they run eight at a time on one), between
    // 2048 entries (short chains for small matrices) and 32768
    const int64_t target = std::min<int64_t>(
        32768, std::max<int64_t>(2048, h.nnz / ((int64_t)ctx().cu * 8)));
    std::vector<int32_t> brow{0}, cbase;
    int32_t start = 0;
    int64_t bmin = INT64_MAX, bmax = -1;
    for (int32_t r = 0; r < h.rows; ++r) {
        if (hi[r] >= 0 && (int64_t)hi[r] - lo[r] >= 65536)
            return false;  // one row alone is too wide
        const int64_t nmin = hi[r] >= 0 ? std::min<int64_t>(bmin, lo[r]) : bmin;
        const int64_t nmax = hi[r] >= 0 ? std::max<int64_t>(bmax, hi[r]) : bmax;
        const bool wide = nmax >= 0 && nmax - nmin >= 65536;
        if (r > start && (r - start >= kBandRows || (int64_t)rp[r] - rp[start] >= target ||
                          wide)) {
            cbase.push_back(bmax >= 0 ? (int32_t)bmin : 0);
            brow.push_back(r);
            start = r;
            bmin = hi[r] >= 0 ? lo[r] : INT64_MAX;
            bmax = hi[r];
        } else {
            bmin = nmin;
            bmax = nmax;
        }
    }
    cbase.push_back(bmax >= 0 ? (int32_t)bmin : 0);
    brow.push_back(h.rows);
    // chosen automatically, the blocks must stay long: rows whose columns
    // are local to each row but not to their neighbours (windows at
    // scattered offsets) cut a block at nearly every row, and a workgroup
    // per few entries is slower than the row-class tiles
    if (automatic && h.nnz < kBandMinEntries * (int64_t)cbase.size())
        return false;
    BandDesc bd{};
    bd.rows = h.rows;
    bd.cols = h.cols;
    bd.nblk = (int32_t)cbase.size();
    std::vector<int32_t> hb((size_t)3 * bd.nblk + 2);
    for (int32_t b = 0; b <= bd.nblk; ++b) {
        hb[b] = brow[b];
        hb[bd.nblk + 1 + b] = rp[brow[b]];
    }
    for (int32_t b = 0; b < bd.nblk; ++b)
        hb[2 * (bd.nblk + 1) + b] = cbase[b];
    h.d_bb = (int32_t *)dev_alloc(hb.size() * 4);
    HIPC(hipMemcpyAsync(h.d_bb, hb.data(), hb.size() * 4, hipMemcpyHostToDevice, s));
    bd.brow = h.d_bb;
    bd.bent = h.d_bb + bd.nblk + 1;
    bd.cbase = h.d_bb + 2 * (bd.nblk + 1);
    h.d_brc = (uint32_t *)dev_alloc((size_t)(h.nnz + kPad) * 4);
    launch_fill_bytes_zero((char *)(h.d_brc + h.nnz), kPad * 4, s);
    launch_band_pack(bd, h.d_row_ptr, h.d_col, h.d_brc, s);
    HIPC(hipStreamSynchronize(s));
    bd.vals = h.d_vals;
    bd.rc = h.d_brc;
    h.band = bd;
    h.use_band = true;
    return true;
}

// Exclusive scan of a[0..n) in place; returns the total.
static int64_t scan_total(int32_t *a, int64_t n, hipStream_t s)
{
    Context &c = ctx();
    launch_scan_excl(a, n, c.total, s);
    int32_t total = 0;
    HIPC(hipMemcpyAsync(&total, c.total, 4, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    return total;
}

// Row-length analysis: class of every row, class-ordered row list, chunk
// table for split rows, and the tile list of one product.  Runs once per
// matrix structure (and again after a plan change).
static void drop_graphs(CsrHandle &h);
void forget_handle_in_groups(const CsrHandle *h);

static void analyse(CsrHandle &h, hipStream_t s)
{
    drop_graphs(h);
    forget_handle_in_groups(&h);
    free_analysis(h);
    Context &c = ctx();
    h.bin_off.assign(NCLASS + 1, 0);
    std::vector<Tile> tiles;
    std::vector<int32_t> host_rows;
    if (h.rows > 0) {
        Thresholds th;
        for (int k = 0; k < NCLASS; ++k)
            th.upper[k] = h.plan.upper[k];
        const int32_t nblk = (h.rows + kBlock - 1) / kBlock;
        const int64_t nh = (int64_t)NCLASS * nblk;
        int32_t *hist = (int32_t *)tmp_alloc(nh * sizeof(int32_t));
        h.d_bin_rows = (int32_t *)dev_alloc((size_t)h.rows * sizeof(int32_t));
        try {
            launch_bin_count(h.rows, h.d_row_ptr, th, hist, nblk, s);
            launch_scan_excl(hist, nh, nullptr, s);
            launch_bin_scatter(h.rows, h.d_row_ptr, th, hist, nblk, h.d_bin_rows, s);
            std::vector<int32_t> hh(nh);
            HIPC(hipMemcpyAsync(hh.data(), hist, nh * sizeof(int32_t),
                                hipMemcpyDeviceToHost, s));
            host_rows.resize(h.rows);
            HIPC(hipMemcpyAsync(host_rows.data(), h.d_bin_rows,
                                (size_t)h.rows * sizeof(int32_t),
                                hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            for (int k = 0; k < NCLASS; ++k)
                h.bin_off[k] = hh[(size_t)k * nblk];
            h.bin_off[NCLASS] = h.rows;
        } catch (...) {
            tmp_free(hist);
            throw;
        }
        tmp_free(hist);

        const int32_t split_begin = h.bin_off[C_SPLIT];
        h.nsplit = h.rows - split_begin;
        if (h.nsplit > 0) {
            h.d_s_first = (int32_t *)dev_alloc((size_t)(h.nsplit + 1) * 4);
            launch_chunk_count(h.nsplit, h.d_bin_rows + split_begin, h.d_row_ptr,
                               h.plan.chunk, h.d_s_first, s);
            launch_scan_excl(h.d_s_first, h.nsplit + 1, c.total, s);
            int32_t total = 0;
            HIPC(hipMemcpyAsync(&total, c.total, 4, hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            h.nchunks = total;
            h.d_c_row = (int32_t *)dev_alloc((size_t)total * 4);
            h.d_c_k0 = (int32_t *)dev_alloc((size_t)total * 4);
            h.d_c_k1 = (int32_t *)dev_alloc((size_t)total * 4);
            h.d_chunk_part = (double *)dev_alloc((size_t)total * 8);
            launch_chunk_fill(h.nsplit, h.d_bin_rows + split_begin, h.d_row_ptr,
                              h.plan.chunk, h.d_s_first, h.d_c_row, h.d_c_k0,
                              h.d_c_k1, s);
        }
        // Tiles, longest work first: split chunks, whole-workgroup rows, then
        // lane classes from 64 lanes down to 1.
        for (int64_t ch = 0; ch < h.nchunks; ++ch)
            tiles.push_back(Tile{C_SPLIT, 0, (int32_t)ch, 1});
        for (int cls = C_WG; cls >= C_W1; --cls) {
            const int32_t a = h.bin_off[cls], e = h.bin_off[cls + 1];
            const int32_t groups = (cls == C_WG) ? 1 : kBlock / kLanes[cls];
            const int32_t per = groups * h.plan.rpg[cls];
            for (int32_t r = a; r < e; r += per) {
                const int32_t cnt = std::min(per, e - r);
                // rows listed in ascending order: consecutive iff the span
                // equals the count
                if (host_rows[r + cnt - 1] - host_rows[r] == cnt - 1)
                    tiles.push_back(Tile{cls | kTileContig, 0, host_rows[r], cnt});
                else
                    tiles.push_back(Tile{cls, 0, r, cnt});
            }
        }
    }
    h.ntiles = (int32_t)tiles.size();
    if (h.ntiles > 0) {
        h.d_tiles = (Tile *)dev_alloc(tiles.size() * sizeof(Tile));
        HIPC(hipMemcpyAsync(h.d_tiles, tiles.data(), tiles.size() * sizeof(Tile),
                            hipMemcpyHostToDevice, s));
        const int occ = std::max(1, std::min(h.plan.grid_per_cu, tile_occupancy(h.dt)));
        h.grid = std::min<int32_t>(h.ntiles, c.cu * occ);
    }
    h.fin_blocks = (h.nsplit + kBlock - 1) / kBlock;
    // a forced panel layout only needs a bounded number of panels; the
    // automatic choice also needs the matrix to suit it
    if (h.line_ratio < 0.0)
        h.line_ratio = measure_line_ratio(h, s);
    const int64_t np_req = panel_count(h);
    const bool want_panels =
        (h.plan.layout == LAYOUT_PANELS && np_req <= kPanelMaxPanels) ||
        (h.plan.layout == LAYOUT_AUTO && panels_eligible(h));
    // the band layout: on request, or automatically for matrices whose
    // columns are local (not gather-heavy) and whose rows are not all short
    // enough for one lane each
    const bool want_band =
        h.plan.layout == LAYOUT_BAND ||
        (h.plan.layout == LAYOUT_AUTO && !want_panels && h.nnz >= kOwnLayoutMinNnz &&
         h.line_ratio < kGatherHeavy);
    if (h.plan.layout == LAYOUT_HOT && hot_possible(h)) {
        build_hot(h, s);
        h.grid = h.hot.grid;   // one fused-dot partial per workgroup
        h.fin_blocks = 0;
    } else if (want_panels && h.rows > 0 && h.nnz > 0) {
        build_panels(h, s);
        h.grid = h.pan.nblk;   // one fused-dot partial per row block
        h.fin_blocks = 0;
    } else if (want_band && build_band(h, s, h.plan.layout == LAYOUT_AUTO)) {
        h.grid = h.band.nblk;  // one fused-dot partial per row block
        h.fin_blocks = 0;
    }
    h.d_dot_part = (double *)dev_alloc((size_t)(std::max(h.grid, 1) + h.fin_blocks + 1) * 8);
    HIPC(hipStreamSynchronize(s));
    g_extra[&h].tiles = std::move(tiles);
}

// ============================================================ handle create

struct TuneKey;
bool tune_cache_lookup(const CsrHandle &h, Plan &out);

static void upload_values(CsrHandle &h, const void *vals, hipStream_t s)
{
    copy_in(h.d_vals, vals, (size_t)h.nnz * dtype_size(h.dt), s);
}

int64_t padded_nnz(int64_t nnz)
{
    return ((nnz + kPad - 1) / kPad) * kPad + kPad;
}

// rp/col/vals == the handle's own arrays (adopted): nothing to copy.
static void construct(CsrHandle &h, int cols_given, const int32_t *rp,
                      const int32_t *col, const void *vals, hipStream_t s)
{
    Context &c = ctx();
    const size_t vs = dtype_size(h.dt);
    const int64_t npad = padded_nnz(h.nnz);
    if (!h.d_row_ptr) {
        h.d_row_ptr = (int32_t *)dev_alloc((size_t)(h.rows + 1) * 4);
        h.d_col = (int32_t *)dev_alloc((size_t)npad * 4);
        h.d_vals = dev_alloc((size_t)npad * vs);
    }
    h.dev_bytes = (int64_t)(h.rows + 1) * 4 + npad * (4 + (int64_t)vs);
    if (rp != h.d_row_ptr)
        copy_in(h.d_row_ptr, rp, (size_t)(h.rows + 1) * 4, s);
    if (col != h.d_col)
        copy_in(h.d_col, col, (size_t)h.nnz * 4, s);
    if (vals != h.d_vals)
        upload_values(h, vals, s);
    // padding past nnz is read (and discarded) by nothing, but keep it defined
    launch_fill_i32(h.d_col + h.nnz, npad - h.nnz, 0, s);
    launch_fill_bytes_zero((char *)h.d_vals + h.nnz * vs, (npad - h.nnz) * vs, s);
    // validation + column count (one pass over row_ptr and col_idx)
    launch_fill_i32(c.status, 1, 0, s);
    launch_fill_i32(c.status + 1, 1, -1, s);
    launch_validate(h.rows, h.d_row_ptr, h.nnz, h.d_col, cols_given, c.status, s);
    int32_t st[2] = {0, -1};
    HIPC(hipMemcpyAsync(st, c.status, sizeof(st), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (st[0]) {
        std::string why;
        if (st[0] & 1) why += " row_ptr[0] != 0;";
        if (st[0] & 2) why += " row_ptr decreases;";
        if (st[0] & 4) why += " row_ptr[rows] != nnz;";
        if (st[0] & 8) why += " column index out of range;";
        fail(LILAC_ERR_CSR, "invalid CSR:" + why);
    }
    h.cols = cols_given >= 0 ? cols_given : st[1] + 1;
    h.max_len = jds_max_len(h, c.total, s);
    h.line_ratio = -1.0;  // measured again for the new structure
    Plan tuned;
    if (tune_cache_lookup(h, tuned))
        h.plan = tuned;
    analyse(h, s);
    h.dev_bytes += analysis_bytes(h);
    h.dirty_struct = h.dirty_vals = false;
}

void destroy_handle(CsrHandle *h);

CsrHandle *create_handle(int rows, int cols, int64_t nnz,
                                const int32_t *rp, const int32_t *col,
                                const void *vals, lilac_dtype dt,
                                unsigned flags, bool inputs_ready)
{
    if (rows < 0)
        fail(LILAC_ERR_ARG, "rows must be >= 0");
    if (nnz < 0 || nnz > (int64_t)INT32_MAX - 8192)
        fail(LILAC_ERR_ARG, "nnz must be in [0, 2^31 - 8192)");
    if (cols < -1)
        cols = -1;
    if (!rp)
        fail(LILAC_ERR_ARG, "row_ptr is NULL");
    if (nnz > 0 && (!col || !vals))
        fail(LILAC_ERR_ARG, "col_idx or vals is NULL");
    if (dt != LILAC_F64 && dt != LILAC_F32)
        fail(LILAC_ERR_ARG, "unknown dtype");
    Context &c = ctx();
    // device inputs may still be in flight on the caller's streams
    if (!inputs_ready && (is_device_ptr(rp) || is_device_ptr(col) || is_device_ptr(vals)))
        HIPC(hipDeviceSynchronize());
    auto *h = new CsrHandle();
    h->rows = rows;
    h->nnz = nnz;
    h->dt = dt;
    h->flags = flags;
    h->cols_given = cols;
    h->plan = default_plan();
    try {
        construct(*h, cols, rp, col, vals, c.stream);
    } catch (...) {
        destroy_handle(h);
        throw;
    }
    if (flags & LILAC_KEEP_HOST) {
        h->h_row_ptr = rp;
        h->h_col = col;
        h->h_vals = vals;
    }
    return h;
}

CsrHandle *create_handle_adopt(int rows, int cols, int64_t nnz, int32_t *rp,
                               int32_t *col, void *vals, lilac_dtype dt, hipStream_t s)
{
    auto *h = new CsrHandle();
    h->d_row_ptr = rp;
    h->d_col = col;
    h->d_vals = vals;
    h->rows = rows;
    h->nnz = nnz;
    h->dt = dt;
    h->cols_given = cols < -1 ? -1 : cols;
    h->plan = default_plan();
    try {
        if (rows < 0 || nnz < 0 || nnz > (int64_t)INT32_MAX - 8192 || !rp || !col || !vals)
            fail(LILAC_ERR_ARG, "bad adopted arrays");
        if (dt != LILAC_F64 && dt != LILAC_F32)
            fail(LILAC_ERR_ARG, "unknown dtype");
        construct(*h, h->cols_given, rp, col, vals, s ? s : ctx().stream);
    } catch (...) {
        destroy_handle(h);
        throw;
    }
    return h;
}

struct CgState {
    int64_t n = 0;
    double *r = nullptr, *p = nullptr, *sv = nullptr, *w = nullptr, *part = nullptr;
    CgScalars *sc = nullptr;
    struct G {
        const double *b;
        double *x;
        int iters;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<G> graphs;
};

struct PrState {
    float *tmp = nullptr;
    // vertices relabelled by decreasing out-degree (large graphs)
    CsrHandle *g = nullptr;
    int32_t *newid = nullptr;
    float *xp = nullptr;
    struct G {
        float *x;
        int iters;
        float d;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<G> graphs;
};

static void drop_graphs(CsrHandle &h)
{
    if (h.pr && h.pr->g) {
        // the relabelled copy follows the matrix: rebuild it on next use
        destroy_handle(h.pr->g);
        h.pr->g = nullptr;
        dev_free(h.pr->newid);
        dev_free(h.pr->xp);
        h.pr->newid = nullptr;
        h.pr->xp = nullptr;
    }
    if (h.cg) {
        for (auto &g : h.cg->graphs) {
            (void)hipGraphExecDestroy(g.exec);
            (void)hipGraphDestroy(g.graph);
        }
        h.cg->graphs.clear();
    }
    if (h.pr) {
        for (auto &g : h.pr->graphs) {
            (void)hipGraphExecDestroy(g.exec);
            (void)hipGraphDestroy(g.graph);
        }
        h.pr->graphs.clear();
    }
}

void destroy_handle(CsrHandle *h)
{
    if (!h)
        return;
    if (g_ctx)
        (void)hipStreamSynchronize(g_ctx->stream);
    marshal_forget(h);
    forget_handle_in_groups(h);
    drop_graphs(*h);
    if (h->cg) {
        dev_free(h->cg->r);
        dev_free(h->cg->p);
        dev_free(h->cg->sv);
        dev_free(h->cg->w);
        dev_free(h->cg->part);
        dev_free(h->cg->sc);
        delete h->cg;
    }
    if (h->pr) {
        dev_free(h->pr->tmp);
        dev_free(h->pr->newid);
        dev_free(h->pr->xp);
        if (h->pr->g)
            destroy_handle(h->pr->g);
        delete h->pr;
    }
    free_analysis(*h);
    dev_free(h->d_row_ptr);
    dev_free(h->d_col);
    dev_free(h->d_vals);
    g_extra.erase(h);
    delete h;
}

// New values also feed the copies made from the CSR arrays (column panels,
// hot columns, the relabelled PageRank graph): rebuild those.
static void values_changed(CsrHandle &h, hipStream_t s)
{
    if (h.use_panels || h.use_hot) {  // the band layout reads the CSR values
        h.dev_bytes -= analysis_bytes(h);
        analyse(h, s);
        h.dev_bytes += analysis_bytes(h);
    } else if (h.pr && h.pr->g) {
        drop_graphs(h);
    }
}

// Bring a handle up to date before use (ReadObject: re-construct after a
// structural change, update after a value change).
static void refresh(CsrHandle &h, hipStream_t s)
{
    if (h.dirty_struct) {
        if (!h.h_row_ptr)
            fail(LILAC_ERR_STATE, "handle invalidated without remembered host arrays");
        drop_graphs(h);
        forget_handle_in_groups(&h);
        construct(h, h.cols_given, h.h_row_ptr, h.h_col, h.h_vals, s);
    } else if (h.dirty_vals) {
        upload_values(h, h.h_vals, s);
        h.dirty_vals = false;
        values_changed(h, s);
    }
}

// ================================================================ products

MatDesc make_desc(const CsrHandle &h, const void *x, void *y,
                         const void *w, double *chunk_part)
{
    MatDesc d;
    d.row_ptr = h.d_row_ptr;
    d.col = h.d_col;
    d.vals = h.d_vals;
    d.bin_rows = h.d_bin_rows;
    d.c_k0 = h.d_c_k0;
    d.c_k1 = h.d_c_k1;
    d.s_first = h.d_s_first;
    d.c_row = h.d_c_row;
    d.x = x;
    d.y = y;
    d.w = w;
    d.chunk_part = chunk_part;
    d.split_begin = h.bin_off.empty() ? 0 : h.bin_off[C_SPLIT];
    d.nsplit = h.nsplit;
    d.tiles = h.d_tiles;
    d.ntiles = h.ntiles;
    d.pad = 0;
    return d;
}

void spmv_enqueue(const CsrHandle &h, const void *x, void *y,
                         const Epi &epi, const void *w, bool dot,
                         hipStream_t s)
{
    if (h.rows == 0)
        return;
    if (h.use_panels) {
        launch_spmv_panels(h.dt, h.pan, x, y, epi, w, dot ? h.d_dot_part : nullptr, s);
        return;
    }
    if (h.use_hot) {
        launch_spmv_hot(h.dt, h.hot, x, y, epi, w, dot ? h.d_dot_part : nullptr, s);
        return;
    }
    if (h.use_band) {
        launch_spmv_band(h.dt, h.band, x, y, epi, w, dot ? h.d_dot_part : nullptr, s);
        return;
    }
    const MatDesc d = make_desc(h, x, y, w, h.d_chunk_part);
    launch_spmv_tiles(h.dt, h.d_tiles, h.ntiles, h.grid, d, nullptr, epi,
                      dot ? h.d_dot_part : nullptr, s);
    if (h.nsplit > 0)
        launch_split_finalize(h.dt, nullptr, h.nsplit, d, nullptr, epi,
                              dot ? h.d_dot_part + h.grid : nullptr, s);
}

static Epi epi_none() { return Epi{EPI_NONE, 0, 0.0, 0.0}; }

int tile_grid(lilac_dtype dt)
{
    return ctx().cu * std::max(1, std::min(kTileGroupsPerCu, tile_occupancy(dt)));
}

// Workgroups of the tile kernel that fit on one CU at once.
static int tile_occupancy(lilac_dtype dt)
{
    Context &c = *g_ctx;
    int &o = c.occ[dt == LILAC_F32 ? 1 : 0];
    if (o == 0) {
        o = occupancy_tiles(dt);
        if (o <= 0)
            o = 4;
    }
    return o;
}

// =============================================================== raw calls

struct RawKey {
    const void *rp, *col, *vals;
    int32_t rows;
    int64_t nnz;
    int dt;
    bool operator<(const RawKey &o) const
    {
        return std::tie(rp, col, vals, rows, nnz, dt) <
               std::tie(o.rp, o.col, o.vals, o.rows, o.nnz, o.dt);
    }
};
static std::map<RawKey, CsrHandle *> g_raw;

void release_all_raw()
{
    for (auto &kv : g_raw)
        destroy_handle(kv.second);
    g_raw.clear();
}

static int marshal_mode()
{
    const char *m = std::getenv("LILAC_MARSHAL");
    if (!m)
        return 0;
    if (!std::strcmp(m, "naive"))
        return 1;
    if (!std::strcmp(m, "protect"))
        return 2;
    return 0;
}

static void *grow_buffer(void *&buf, size_t &cap, size_t bytes)
{
    if (bytes > cap) {
        dev_free(buf);
        buf = nullptr;
        cap = 0;
        buf = dev_alloc(bytes);
        cap = bytes;
    }
    return buf;
}

static void raw_spmv(int rows, const int32_t *rp, const int32_t *col,
                     const void *vals, const void *x, void *y, lilac_dtype dt)
{
    if (rows < 0)
        fail(LILAC_ERR_ARG, "rows must be >= 0");
    if (!rp || !y)
        fail(LILAC_ERR_ARG, "row_ptr or y is NULL");
    Context &c = ctx();
    hipStream_t s = c.stream;
    if (rows == 0)
        return;
    int32_t last = 0;
    const bool rp_dev = is_device_ptr(rp);
    // a blocking call: device operands written on other streams must be done
    if (rp_dev || is_device_ptr(x) || is_device_ptr(y) || is_device_ptr(vals))
        HIPC(hipDeviceSynchronize());
    if (rp_dev) {
        HIPC(hipMemcpyAsync(&last, rp + rows, 4, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
    } else {
        last = rp[rows];
    }
    if (last < 0)
        fail(LILAC_ERR_CSR, "invalid CSR: row_ptr[rows] < 0");
    const int64_t nnz = last;
    const int mode = marshal_mode();
    CsrHandle *h = nullptr;
    std::unique_ptr<CsrHandle, void (*)(CsrHandle *)> temp(nullptr, destroy_handle);
    if (mode == 1) {
        temp.reset(create_handle(rows, -1, nnz, rp, col, vals, dt, 0));
        h = temp.get();
    } else {
        RawKey key{rp, col, vals, rows, nnz, (int)dt};
        auto it = g_raw.find(key);
        if (it == g_raw.end()) {
            h = create_handle(rows, -1, nnz, rp, col, vals, dt, LILAC_KEEP_HOST);
            g_raw[key] = h;
            if (mode == 2) {
                if (!rp_dev)
                    marshal_track_range(h, MARSHAL_STRUCT, rp, (size_t)(rows + 1) * 4);
                if (col && !is_device_ptr(col))
                    marshal_track_range(h, MARSHAL_STRUCT, col, (size_t)nnz * 4);
                if (vals && !is_device_ptr(vals))
                    marshal_track_range(h, MARSHAL_VALS, vals, (size_t)nnz * dtype_size(dt));
            }
        } else {
            h = it->second;
            if (mode == 2) {
                const int k = marshal_take_dirty(h);
                if (k & MARSHAL_STRUCT)
                    h->dirty_struct = true;
                if (k & MARSHAL_VALS)
                    h->dirty_vals = true;
            }
            const bool was_dirty = h->dirty_struct || h->dirty_vals;
            refresh(*h, s);
            if (mode == 2 && was_dirty)
                marshal_arm(h);
        }
    }
    const size_t vs = dtype_size(dt);
    const void *dx = x;
    if (h->cols > 0 && !x)
        fail(LILAC_ERR_ARG, "x is NULL");
    if (x && !is_device_ptr(x)) {
        void *b = grow_buffer(c.x_buf, c.x_cap, (size_t)h->cols * vs);
        HIPC(hipMemcpyAsync(b, x, (size_t)h->cols * vs, hipMemcpyHostToDevice, s));
        dx = b;
    }
    const bool y_dev = is_device_ptr(y);
    void *dy = y_dev ? y : grow_buffer(c.y_buf, c.y_cap, (size_t)rows * vs);
    spmv_enqueue(*h, dx, dy, epi_none(), nullptr, false, s);
    if (!y_dev)
        HIPC(hipMemcpyAsync(y, dy, (size_t)rows * vs, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
}

static void invalidate_ptr(const void *ptr)
{
    const char *p = (const char *)ptr;
    for (auto &kv : g_raw) {
        const RawKey &k = kv.first;
        CsrHandle *h = kv.second;
        const size_t vs = dtype_size((lilac_dtype)k.dt);
        auto inside = [&](const void *base, size_t bytes) {
            const char *b = (const char *)base;
            return b && p >= b && p < b + std::max<size_t>(bytes, 1);
        };
        if (inside(k.rp, (size_t)(k.rows + 1) * 4) || inside(k.col, (size_t)k.nnz * 4))
            h->dirty_struct = true;
        else if (inside(k.vals, (size_t)k.nnz * vs))
            h->dirty_vals = true;
    }
}

// ===================================================================== dot

template <typename T>
static double raw_dot(int64_t n, const T *a, const T *b)
{
    if (n < 0)
        fail(LILAC_ERR_ARG, "n must be >= 0");
    if (n == 0)
        return 0.0;
    if (!a || !b)
        fail(LILAC_ERR_ARG, "a or b is NULL");
    Context &c = ctx();
    hipStream_t s = c.stream;
    const T *da = a, *db = b;
    const size_t bytes = (size_t)n * sizeof(T);
    const bool ad = is_device_ptr(a), bd = is_device_ptr(b);
    if (ad || bd)
        HIPC(hipDeviceSynchronize());
    if (!ad || !bd) {
        if (bytes > c.dot_cap) {
            dev_free_reset(c.dot_a);
            dev_free_reset(c.dot_b);
            c.dot_cap = 0;
            c.dot_a = (double *)dev_alloc(bytes);
            c.dot_b = (double *)dev_alloc(bytes);
            c.dot_cap = bytes;
        }
        if (!ad) {
            HIPC(hipMemcpyAsync(c.dot_a, a, bytes, hipMemcpyHostToDevice, s));
            da = (const T *)c.dot_a;
        }
        if (!bd) {
            HIPC(hipMemcpyAsync(c.dot_b, b, bytes, hipMemcpyHostToDevice, s));
            db = (const T *)c.dot_b;
        }
    }
    const int32_t np = blas1_parts(n);
    if constexpr (std::is_same<T, float>::value)
        launch_dot_parts_f32(n, da, db, c.dot_part, np, s);
    else
        launch_dot_parts(n, da, db, c.dot_part, np, s);
    launch_sum_parts(c.dot_part, np, c.dot_part + kDotParts, s);
    double r = 0.0;
    HIPC(hipMemcpyAsync(&r, c.dot_part + kDotParts, 8, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    return r;
}

// ====================================================================== CG

static void cg_prepare(CsrHandle &h)
{
    if (h.cg)
        return;
    auto *st = new CgState();
    st->n = h.rows;
    try {
        st->r = (double *)dev_alloc((size_t)h.rows * 8);
        st->p = (double *)dev_alloc((size_t)h.rows * 8);
        st->sv = (double *)dev_alloc((size_t)h.rows * 8);
        st->w = (double *)dev_alloc((size_t)h.rows * 8);
        st->part = (double *)dev_alloc((size_t)2 * kDotParts * 8);
        st->sc = (CgScalars *)dev_alloc(sizeof(CgScalars));
    } catch (...) {
        dev_free(st->r);
        dev_free(st->p);
        dev_free(st->sv);
        dev_free(st->w);
        dev_free(st->part);
        delete st;
        throw;
    }
    h.cg = st;
}

void handle_cg_prepare(CsrHandle &h) { cg_prepare(h); }

// One whole solve: initialisation, then `iters` iterations of two kernels
// (the product w = A r with the w.r partials fused into it; the scalars and
// the p, s, x, r updates with the next r.r partials), then the final r.r.
// Scalars never leave the device.  r, p, sv (s = A p), w hold rows doubles,
// part 2 * kDotParts, sc one CgScalars; the initialisation writes
// everything later launches read.
static void cg_enqueue_state(const CsrHandle &h, const double *b, double *x, int iters,
                             double *r, double *p, double *sv, double *w, double *part,
                             CgScalars *sc, hipStream_t s)
{
    const int64_t n = h.rows;
    const int32_t np = blas1_parts(n);
    const int32_t ndot = h.grid + h.fin_blocks;
    launch_cg_init(n, b, x, r, p, sv, part, np, sc, s);
    for (int it = 0; it < iters; ++it) {
        spmv_enqueue(h, r, w, epi_none(), r, true, s);
        launch_cg_step(n, sc, w, p, sv, x, r, h.d_dot_part, ndot, part, np, it, s);
    }
    launch_cg_final(sc, part, np, iters & 1, s);
}

static void cg_enqueue(const CsrHandle &h, const double *b, double *x,
                       int iters, hipStream_t s)
{
    const CgState &st = *h.cg;
    cg_enqueue_state(h, b, x, iters, st.r, st.p, st.sv, st.w, st.part, st.sc, s);
}

// ------------------------------------------------ CG without allocation
//
// For callers that cannot allocate device memory (work under HIP graph
// capture, tight serving loops): the CG state (r, p, s, w, the r.r partials
// and the scalars) lives in one fixed device array instead of the handle's
// state, which is allocated on first use.  The array holds the state of a
// matrix of at most kNoAllocRows rows; every GPU the library runs on keeps
// its own copy until the process ends.  In host code `scratch` is only a
// stand-in for the symbol: its device address, per device, comes from
// hipGetSymbolAddress and only that address is handed to kernels.
constexpr int64_t kNoAllocRows = 1 << 20;
constexpr size_t kNoAllocPart = 2 * kDotParts;
constexpr size_t kNoAllocBytes =
    4 * (size_t)kNoAllocRows * 8 + kNoAllocPart * 8 + sizeof(CgScalars);
static __device__ __align__(256) char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
static char *scratch_on_current_device()
{
    int dev = -1;
    HIPC(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        fail(LILAC_ERR_DEVICE, "device index beyond the fixed-state table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            fail(LILAC_ERR_DEVICE, std::string("hipGetSymbolAddress of the fixed CG "
                                               "state failed: ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = (char *)ptr;
    }
    return g_scratch_ptr[dev];
}

template <typename Enq>
static void capture(hipGraph_t &graph, hipGraphExec_t &exec, Enq enq)
{
    Context &c = ctx();
    HIPC(hipStreamBeginCapture(c.cap, hipStreamCaptureModeRelaxed));
    try {
        enq(c.cap);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(c.cap, &g);
        if (g)
            (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        throw;
    }
    HIPC(hipStreamEndCapture(c.cap, &graph));
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        hip_check(e, "hipGraphInstantiate", __FILE__, __LINE__);
    }
}

void run_cg(CsrHandle &h, const double *b, double *x, int iters,
                   unsigned flags, hipStream_t s, double *rho_out,
                   int *iters_done)
{
    if (h.dt != LILAC_F64)
        fail(LILAC_ERR_UNSUPPORTED, "CG needs a float64 handle");
    if (h.rows != h.cols)
        fail(LILAC_ERR_ARG, "CG needs a square matrix");
    if (iters < 0)
        fail(LILAC_ERR_ARG, "iters must be >= 0");
    if (h.rows > 0 && (!b || !x))
        fail(LILAC_ERR_ARG, "b or x is NULL");
    if (h.rows > 0 && (!is_device_ptr(b) || !is_device_ptr(x)))
        fail(LILAC_ERR_ARG, "b and x must be device arrays");
    refresh(h, s);
    if (h.rows == 0) {
        if (rho_out)
            *rho_out = 0.0;
        if (iters_done)
            *iters_done = 0;
        return;
    }
    cg_prepare(h);
    if (flags & LILAC_CG_GRAPH) {
        CgState &st = *h.cg;
        CgState::G *hit = nullptr;
        for (auto &g : st.graphs)
            if (g.b == b && g.x == x && g.iters == iters)
                hit = &g;
        if (!hit) {
            if (st.graphs.size() >= 4) {
                (void)hipGraphExecDestroy(st.graphs.front().exec);
                (void)hipGraphDestroy(st.graphs.front().graph);
                st.graphs.erase(st.graphs.begin());
            }
            CgState::G g{b, x, iters, nullptr, nullptr};
            capture(g.graph, g.exec,
                    [&](hipStream_t cs) { cg_enqueue(h, b, x, iters, cs); });
            st.graphs.push_back(g);
            hit = &st.graphs.back();
        }
        HIPC(hipGraphLaunch(hit->exec, s));
    } else {
        cg_enqueue(h, b, x, iters, s);
    }
    if (rho_out || iters_done) {
        CgScalars sc;
        HIPC(hipMemcpyAsync(&sc, h.cg->sc, sizeof(sc), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        if (rho_out)
            *rho_out = sc.rho;
        if (iters_done)
            *iters_done = sc.iters;
    }
}

// ================================================================ PageRank

// Graphs with at least this many vertices are iterated on a copy relabelled
// by out-degree.
constexpr int32_t kRelabelRows = 65536;

// Copy of a square graph matrix with its vertices renamed in decreasing
// out-degree order (stable): the most gathered entries of x come first,
// where the hot-column layout keeps them in LDS.  (P A P^T)(P x) = P (A x).
static void build_relabel(CsrHandle &h, PrState &st)
{
    Context &c = ctx();
    hipStream_t s = c.stream;
    const int32_t n = h.rows;
    const int32_t nblk = (n + kBlock - 1) / kBlock;
    int32_t *deg = nullptr, *key = nullptr, *hist = nullptr, *rp2 = nullptr,
            *col2 = nullptr;
    void *vals2 = nullptr;
    try {
        deg = (int32_t *)dev_alloc((size_t)n * 4);
        key = (int32_t *)dev_alloc((size_t)n * 4);
        hist = (int32_t *)dev_alloc((size_t)kDegKeys * nblk * 4);
        st.newid = (int32_t *)dev_alloc((size_t)n * 4);
        launch_fill_i32(deg, n, 0, s);
        launch_count_cols(h.nnz, h.d_col, deg, s);
        launch_degree_keys(n, deg, key, s);
        launch_key_hist(n, key, hist, nblk, s);
        launch_scan_excl(hist, (int64_t)kDegKeys * nblk, nullptr, s);
        launch_key_scatter(n, key, hist, nblk, st.newid, s);
        rp2 = (int32_t *)dev_alloc((size_t)(n + 1) * 4);
        launch_perm_lengths(n, h.d_row_ptr, st.newid, rp2, s);
        const int64_t total = scan_total(rp2, (int64_t)n + 1, s);
        if (total != h.nnz)
            fail(LILAC_ERR_DEVICE, "relabelled copy lost entries");
        col2 = (int32_t *)dev_alloc((size_t)std::max<int64_t>(h.nnz, 1) * 4);
        vals2 = dev_alloc((size_t)std::max<int64_t>(h.nnz, 1) * 4);
        launch_perm_entries(h.dt, n, h.nnz, h.d_row_ptr, h.d_col, h.d_vals, st.newid,
                            rp2, col2, vals2, s);
        HIPC(hipStreamSynchronize(s));
        st.g = create_handle(n, h.cols, h.nnz, rp2, col2, vals2, h.dt, 0);
        if (hot_possible(*st.g)) {
            // after relabelling the most gathered columns come first: keep
            // them in LDS (hot-column layout)
            CsrHandle &g = *st.g;
            g.dev_bytes -= analysis_bytes(g);
            g.plan.layout = LAYOUT_HOT;
            analyse(g, s);
            g.dev_bytes += analysis_bytes(g);
        }
        st.xp = (float *)dev_alloc((size_t)n * 4);
    } catch (...) {
        dev_free(deg);
        dev_free(key);
        dev_free(hist);
        dev_free(rp2);
        dev_free(col2);
        dev_free(vals2);
        throw;
    }
    dev_free(deg);
    dev_free(key);
    dev_free(hist);
    dev_free(rp2);
    dev_free(col2);
    dev_free(vals2);
}

static void run_pagerank(CsrHandle &h, float d, int iters, float *x,
                         hipStream_t s)
{
    if (h.dt != LILAC_F32)
        fail(LILAC_ERR_UNSUPPORTED, "PageRank needs a float32 handle");
    if (h.rows != h.cols && h.nnz > 0 && h.cols > h.rows)
        fail(LILAC_ERR_ARG, "PageRank needs a square matrix");
    if (iters < 0)
        fail(LILAC_ERR_ARG, "iters must be >= 0");
    if (h.rows == 0 || iters == 0)
        return;
    if (!x || !is_device_ptr(x))
        fail(LILAC_ERR_ARG, "x_inout must be a device array");
    refresh(h, s);
    if (!h.pr) {
        auto *st = new PrState();
        try {
            st->tmp = (float *)dev_alloc((size_t)h.rows * 4);
        } catch (...) {
            delete st;
            throw;
        }
        h.pr = st;
    }
    PrState &st = *h.pr;
    PrState::G *hit = nullptr;
    for (auto &g : st.graphs)
        if (g.x == x && g.iters == iters && g.d == d)
            hit = &g;
    if (!hit) {
        if (st.graphs.size() >= 4) {
            (void)hipGraphExecDestroy(st.graphs.front().exec);
            (void)hipGraphDestroy(st.graphs.front().graph);
            st.graphs.erase(st.graphs.begin());
        }
        PrState::G g{x, iters, d, nullptr, nullptr};
        const Epi epi{EPI_PAGERANK, 0, (double)d,
                      (1.0 - (double)d) / (double)h.rows};
        const bool relabel = h.rows >= kRelabelRows && h.cols <= h.rows;
        if (relabel && !st.g)
            build_relabel(h, st);
        capture(g.graph, g.exec, [&](hipStream_t cs) {
            if (relabel) {
                // iterate on the relabelled copy: x' = P x, ..., x = P^T x'
                launch_permute_f32(h.rows, st.newid, x, st.xp, true, cs);
                float *cur = st.xp, *nxt = st.tmp;
                for (int it = 0; it < iters; ++it) {
                    spmv_enqueue(*st.g, cur, nxt, epi, nullptr, false, cs);
                    std::swap(cur, nxt);
                }
                launch_permute_f32(h.rows, st.newid, cur, x, false, cs);
                return;
            }
            float *cur = x, *nxt = st.tmp;
            for (int it = 0; it < iters; ++it) {
                spmv_enqueue(h, cur, nxt, epi, nullptr, false, cs);
                std::swap(cur, nxt);
            }
            if (cur != x)
                launch_copy_f32(h.rows, cur, x, cs);
        });
        st.graphs.push_back(g);
        hit = &st.graphs.back();
    }
    HIPC(hipGraphLaunch(hit->exec, s));
}

// ================================================================= batched

struct GroupPlan {
    std::vector<const CsrHandle *> hs;
    std::vector<const void *> xs;
    std::vector<void *> ys;
    lilac_dtype dt;
    MatDesc *d_mats = nullptr;
    Tile *d_tiles = nullptr;
    int32_t *d_items = nullptr;
    double *d_chunk = nullptr;
    int32_t ntiles = 0, grid = 0, nitems = 0;
    // column-panel matrices of the group: one grouped launch
    PanelDesc *d_pdesc = nullptr;
    PanelIO *d_pio = nullptr;
    int32_t *d_pprefix = nullptr;
    int32_t npm = 0, pblocks = 0;
    // band matrices of the group: one grouped launch
    BandDesc *d_bdesc = nullptr;
    PanelIO *d_bio = nullptr;
    int32_t *d_bprefix = nullptr;
    int32_t nbm = 0, bblocks = 0;
};
static std::vector<GroupPlan *> g_groups;

static void free_group(GroupPlan *g)
{
    dev_free(g->d_mats);
    dev_free(g->d_tiles);
    dev_free(g->d_items);
    dev_free(g->d_chunk);
    dev_free(g->d_pdesc);
    dev_free(g->d_pio);
    dev_free(g->d_pprefix);
    dev_free(g->d_bdesc);
    dev_free(g->d_bio);
    dev_free(g->d_bprefix);
    delete g;
}

void release_group_plans()
{
    for (auto *g : g_groups)
        free_group(g);
    g_groups.clear();
}

void forget_handle_in_groups(const CsrHandle *h)
{
    for (size_t i = 0; i < g_groups.size();) {
        GroupPlan *g = g_groups[i];
        if (std::find(g->hs.begin(), g->hs.end(), h) != g->hs.end()) {
            free_group(g);
            g_groups.erase(g_groups.begin() + i);
        } else {
            ++i;
        }
    }
}

// One work list over all matrices: tiles of every matrix, class by class
// from the longest work down, so the persistent workgroups drain the big
// items first.  Each matrix keeps its own plan (and so its own reduction
// order); split rows get chunk-partial space private to this group.
static GroupPlan *build_group(int count, const lilac_csr_t *hs,
                              const void *const *xs, void *const *ys,
                              hipStream_t s)
{
    auto *g = new GroupPlan();
    g->dt = ((const CsrHandle *)hs[0])->dt;
    std::vector<MatDesc> descs(count);
    std::vector<int64_t> chunk_off(count, 0);
    int64_t nchunk_total = 0;
    for (int j = 0; j < count; ++j) {
        const CsrHandle *h = (const CsrHandle *)hs[j];
        g->hs.push_back(h);
        g->xs.push_back(xs[j]);
        g->ys.push_back(ys[j]);
        chunk_off[j] = nchunk_total;
        nchunk_total += h->nchunks;
    }
    std::vector<int32_t> items;
    try {
        if (nchunk_total > 0)
            g->d_chunk = (double *)dev_alloc((size_t)nchunk_total * 8);
        for (int j = 0; j < count; ++j) {
            const CsrHandle *h = g->hs[j];
            descs[j] = make_desc(*h, xs[j], ys[j], nullptr,
                                 g->d_chunk ? g->d_chunk + chunk_off[j] : nullptr);
            if (own_layout(*h))
                continue;  // launched on its own layout
            for (int32_t k = 0; k < h->nsplit; ++k) {
                items.push_back(j);
                items.push_back(k);
            }
        }
        std::vector<Tile> tiles;
        for (int cls = C_SPLIT; cls >= C_W1; --cls)
            for (int j = 0; j < count; ++j)
                for (const Tile &t : g_extra[g->hs[j]].tiles)
                    if (!own_layout(*g->hs[j]))
                    if ((t.cls & kTileClassMask) == cls) {
                        Tile u = t;
                        u.mat = j;
                        tiles.push_back(u);
                    }
        g->ntiles = (int32_t)tiles.size();
        g->nitems = (int32_t)(items.size() / 2);
        g->d_mats = (MatDesc *)dev_alloc(descs.size() * sizeof(MatDesc));
        HIPC(hipMemcpyAsync(g->d_mats, descs.data(), descs.size() * sizeof(MatDesc),
                            hipMemcpyHostToDevice, s));
        if (g->ntiles) {
            g->d_tiles = (Tile *)dev_alloc(tiles.size() * sizeof(Tile));
            HIPC(hipMemcpyAsync(g->d_tiles, tiles.data(), tiles.size() * sizeof(Tile),
                                hipMemcpyHostToDevice, s));
        }
        if (g->nitems) {
            g->d_items = (int32_t *)dev_alloc(items.size() * 4);
            HIPC(hipMemcpyAsync(g->d_items, items.data(), items.size() * 4,
                                hipMemcpyHostToDevice, s));
        }
        // the grouped launches take the matrices with the most non-zeros per
        // block first, so that the last workgroups to start are short ones
        auto heavy_first = [&](bool panels) {
            std::vector<int> order;
            for (int j = 0; j < count; ++j) {
                const CsrHandle *h = g->hs[j];
                if ((panels ? h->use_panels : h->use_band) && h->rows > 0)
                    order.push_back(j);
            }
            auto per_block = [&](int j) {
                const CsrHandle *h = g->hs[j];
                return (double)h->nnz / (double)std::max(1, panels ? h->pan.nblk : h->band.nblk);
            };
            std::stable_sort(order.begin(), order.end(),
                             [&](int a, int b) { return per_block(a) > per_block(b); });
            return order;
        };
        std::vector<PanelDesc> pdesc;
        std::vector<PanelIO> pio;
        std::vector<int32_t> pprefix(1, 0);
        for (int j : heavy_first(true)) {
            const CsrHandle *h = g->hs[j];
            pdesc.push_back(h->pan);
            pio.push_back(PanelIO{xs[j], ys[j]});
            pprefix.push_back(pprefix.back() + h->pan.nblk);
        }
        std::vector<BandDesc> bdesc;
        std::vector<PanelIO> bio;
        std::vector<int32_t> bprefix(1, 0);
        for (int j : heavy_first(false)) {
            const CsrHandle *h = g->hs[j];
            bdesc.push_back(h->band);
            bio.push_back(PanelIO{xs[j], ys[j]});
            bprefix.push_back(bprefix.back() + h->band.nblk);
        }
        g->nbm = (int32_t)bdesc.size();
        g->bblocks = bprefix.back();
        if (g->nbm) {
            g->d_bdesc = (BandDesc *)dev_alloc(bdesc.size() * sizeof(BandDesc));
            g->d_bio = (PanelIO *)dev_alloc(bio.size() * sizeof(PanelIO));
            g->d_bprefix = (int32_t *)dev_alloc(bprefix.size() * 4);
            HIPC(hipMemcpyAsync(g->d_bdesc, bdesc.data(), bdesc.size() * sizeof(BandDesc),
                                hipMemcpyHostToDevice, s));
            HIPC(hipMemcpyAsync(g->d_bio, bio.data(), bio.size() * sizeof(PanelIO),
                                hipMemcpyHostToDevice, s));
            HIPC(hipMemcpyAsync(g->d_bprefix, bprefix.data(), bprefix.size() * 4,
                                hipMemcpyHostToDevice, s));
        }
        g->npm = (int32_t)pdesc.size();
        g->pblocks = pprefix.back();
        if (g->npm) {
            g->d_pdesc = (PanelDesc *)dev_alloc(pdesc.size() * sizeof(PanelDesc));
            g->d_pio = (PanelIO *)dev_alloc(pio.size() * sizeof(PanelIO));
            g->d_pprefix = (int32_t *)dev_alloc(pprefix.size() * 4);
            HIPC(hipMemcpyAsync(g->d_pdesc, pdesc.data(), pdesc.size() * sizeof(PanelDesc),
                                hipMemcpyHostToDevice, s));
            HIPC(hipMemcpyAsync(g->d_pio, pio.data(), pio.size() * sizeof(PanelIO),
                                hipMemcpyHostToDevice, s));
            HIPC(hipMemcpyAsync(g->d_pprefix, pprefix.data(), pprefix.size() * 4,
                                hipMemcpyHostToDevice, s));
        }
        HIPC(hipStreamSynchronize(s));
    } catch (...) {
        free_group(g);
        throw;
    }
    const int occ = std::max(1, std::min(kTileGroupsPerCu, tile_occupancy(g->dt)));
    g->grid = std::min<int32_t>(g->ntiles, ctx().cu * occ);
    return g;
}

static void run_batched(int count, const lilac_csr_t *hs, const void *const *xs,
                        void *const *ys, hipStream_t s)
{
    if (count < 0)
        fail(LILAC_ERR_ARG, "count must be >= 0");
    if (count == 0)
        return;
    if (!hs || !xs || !ys)
        fail(LILAC_ERR_ARG, "NULL array");
    const lilac_dtype dt = ((const CsrHandle *)hs[0])->dt;
    for (int j = 0; j < count; ++j) {
        CsrHandle *h = (CsrHandle *)hs[j];
        if (!h)
            fail(LILAC_ERR_ARG, "NULL handle");
        if (h->dt != dt)
            fail(LILAC_ERR_ARG, "all handles of a batch must share one dtype");
        if (h->rows > 0 && (!ys[j] || (h->cols > 0 && !xs[j])))
            fail(LILAC_ERR_ARG, "NULL vector in batch");
        refresh(*h, s);
    }
    GroupPlan *hit = nullptr;
    for (auto *g : g_groups) {
        if ((int)g->hs.size() != count)
            continue;
        bool same = true;
        for (int j = 0; j < count && same; ++j)
            same = g->hs[j] == (const CsrHandle *)hs[j] && g->xs[j] == xs[j] &&
                   g->ys[j] == ys[j];
        if (same) {
            hit = g;
            break;
        }
    }
    if (!hit) {
        if (g_groups.size() >= 8) {
            free_group(g_groups.front());
            g_groups.erase(g_groups.begin());
        }
        hit = build_group(count, hs, xs, ys, s);
        g_groups.push_back(hit);
    }
    MatDesc none{};
    launch_spmv_tiles(hit->dt, hit->d_tiles, hit->ntiles, hit->grid, none,
                      hit->d_mats, epi_none(), nullptr, s);
    if (hit->nitems)
        launch_split_finalize(hit->dt, hit->d_items, hit->nitems, none,
                              hit->d_mats, epi_none(), nullptr, s);
    // column-panel and band matrices: one grouped launch each, whose blocks
    // run exactly as in each matrix's single call; hot-column matrices: their
    // own launch
    launch_spmv_panels_grouped(hit->dt, hit->d_pdesc, hit->d_pio, hit->d_pprefix,
                               hit->npm, hit->pblocks, s);
    launch_spmv_band_grouped(hit->dt, hit->d_bdesc, hit->d_bio, hit->d_bprefix,
                             hit->nbm, hit->bblocks, s);
    for (int j = 0; j < count; ++j) {
        const CsrHandle *h = hit->hs[j];
        if (h->use_hot)
            spmv_enqueue(*h, xs[j], ys[j], epi_none(), nullptr, false, s);
    }
}

// ================================================================ tuning

// Shape class of a matrix: dtype, log2 of rows, twice log2 of the mean row
// length, and the row class of its longest row under the default bounds
// (known before the analysis, so a new handle finds its class's plan).
// Handles of one class share a plan.
static std::string tune_key(const CsrHandle &h)
{
    const double mean = h.rows ? (double)h.nnz / h.rows : 0.0;
    const Plan d = default_plan();
    int top = 0;
    while (top < NCLASS - 1 && h.max_len > d.upper[top])
        ++top;
    char buf[96];
    std::snprintf(buf, sizeof(buf), "%s/r%d/m%d/c%d", h.dt == LILAC_F32 ? "f32" : "f64",
                  (int)std::lround(std::log2(std::max(1, h.rows))),
                  (int)std::lround(2.0 * std::log2(std::max(1.0, mean))), top);
    return buf;
}

static std::map<std::string, Plan> g_tune;
static bool g_tune_loaded = false;

static std::string plan_to_json(const Plan &p)
{
    std::ostringstream o;
    o << "{\"upper\":[";
    for (int c = 0; c < NCLASS - 1; ++c)
        o << (c ? "," : "") << p.upper[c];
    o << "],\"rpg\":[";
    for (int c = 0; c < NCLASS; ++c)
        o << (c ? "," : "") << p.rpg[c];
    o << "],\"chunk\":" << p.chunk << ",\"grid_per_cu\":" << p.grid_per_cu
      << ",\"layout\":" << p.layout << "}";
    return o.str();
}

// Minimal reader for the cache file this library writes (one entry per
// line: "key" followed by the plan's integers in a fixed order).
void tune_cache_load()
{
    if (g_tune_loaded)
        return;
    g_tune_loaded = true;
    const char *path = std::getenv("LILAC_TUNE_CACHE");
    if (!path)
        return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        const size_t q0 = line.find('"');
        const size_t q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
        if (q1 == std::string::npos)
            continue;
        const std::string key = line.substr(q0 + 1, q1 - q0 - 1);
        std::vector<long> nums;
        std::string rest = line.substr(q1 + 1);
        for (size_t i = 0; i < rest.size();) {
            if (std::isdigit((unsigned char)rest[i]) || (rest[i] == '-' && i + 1 < rest.size() &&
                                                         std::isdigit((unsigned char)rest[i + 1]))) {
                size_t used = 0;
                nums.push_back(std::stol(rest.substr(i), &used));
                i += used;
            } else {
                ++i;
            }
        }
        if (nums.size() != (size_t)(NCLASS - 1 + NCLASS + 3))
            continue;
        Plan p = default_plan();
        size_t k = 0;
        for (int c = 0; c < NCLASS - 1; ++c)
            p.upper[c] = (int32_t)nums[k++];
        for (int c = 0; c < NCLASS; ++c)
            p.rpg[c] = (int32_t)nums[k++];
        p.chunk = (int32_t)nums[k++];
        p.grid_per_cu = (int32_t)nums[k++];
        p.layout = (int32_t)nums[k++];
        try {
            check_plan(p);
            g_tune[key] = p;
        } catch (const Error &) {
        }
    }
}

static void tune_cache_save()
{
    const char *path = std::getenv("LILAC_TUNE_CACHE");
    if (!path)
        return;
    std::ofstream f(path);
    f << "{\n";
    size_t i = 0;
    for (auto &kv : g_tune)
        f << "\"" << kv.first << "\": " << plan_to_json(kv.second)
          << (++i < g_tune.size() ? "," : "") << "\n";
    f << "}\n";
}

bool tune_cache_lookup(const CsrHandle &h, Plan &out)
{
    if (g_tune.empty())
        return false;
    // the key needs the row count, the mean and the longest row length,
    // all known before the analysis
    auto it = g_tune.find(tune_key(h));
    if (it == g_tune.end())
        return false;
    out = it->second;
    return true;
}

static double time_spmv(CsrHandle &h, const void *x, void *y, int reps)
{
    Context &c = ctx();
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    for (int i = 0; i < 2; ++i)
        spmv_enqueue(h, x, y, epi_none(), nullptr, false, c.stream);
    HIPC(hipEventRecord(e0, c.stream));
    for (int i = 0; i < reps; ++i)
        spmv_enqueue(h, x, y, epi_none(), nullptr, false, c.stream);
    HIPC(hipEventRecord(e1, c.stream));
    HIPC(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPC(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return 1000.0 * ms / reps;
}

// Coordinate search over the plan: elements per lane of the lane classes,
// the wavefront / workgroup / split bounds, the chunk size, rows per group
// of the wavefront class and the persistent grid size.  Each candidate is
// re-analysed and timed on the matrix itself.
static double tune_handle(CsrHandle &h)
{
    Context &c = ctx();
    refresh(h, c.stream);
    if (h.rows == 0)
        return 0.0;
    const size_t vs = dtype_size(h.dt);
    void *x = dev_alloc((size_t)std::max(1, h.cols) * vs);
    void *y = dev_alloc((size_t)h.rows * vs);
    launch_fill_bytes_zero(x, (int64_t)std::max(1, h.cols) * vs, c.stream);
    const int reps = h.nnz > (1 << 22) ? 10 : 30;
    Plan best = h.plan;
    double best_us = 1e300;
    auto trial = [&](const Plan &p) {
        try {
            check_plan(p);
        } catch (const Error &) {
            return;
        }
        h.plan = p;
        analyse(h, c.stream);
        const double us = time_spmv(h, x, y, reps);
        if (us < best_us) {
            best_us = us;
            best = p;
        }
    };
    try {
        trial(best);
        for (int epl : {1, 2, 4, 8}) {
            Plan p = best;
            for (int cl = C_W1; cl <= C_W32; ++cl)
                p.upper[cl] = epl * kLanes[cl];
            trial(p);
        }
        for (int w64 : {256, 512, 1024, 2048, 4096}) {
            Plan p = best;
            p.upper[C_W64] = std::max(w64, p.upper[C_W32]);
            trial(p);
        }
        for (int wg : {4096, 8192, 16384, 65536}) {
            Plan p = best;
            p.upper[C_WG] = std::max(wg, p.upper[C_W64]);
            trial(p);
        }
        for (int ch : {2048, 4096, 8192, 16384}) {
            Plan p = best;
            p.chunk = ch;
            trial(p);
        }
        for (int r : {1, 2, 4, 8}) {
            Plan p = best;
            p.rpg[C_W64] = r;
            trial(p);
        }
        for (int gp : {2, 4, 8, 16}) {
            Plan p = best;
            p.grid_per_cu = gp;
            trial(p);
        }
        for (int lay : {LAYOUT_ROWS, LAYOUT_PANELS, LAYOUT_HOT, LAYOUT_BAND}) {
            Plan p = best;
            p.layout = lay;
            if (lay == LAYOUT_PANELS && !panels_eligible(h))
                continue;
            if (lay == LAYOUT_HOT && (!hot_possible(h) || h.rows < 32768))
                continue;
            trial(p);
        }
    } catch (...) {
        dev_free(x);
        dev_free(y);
        h.plan = best;
        analyse(h, c.stream);
        throw;
    }
    dev_free(x);
    dev_free(y);
    h.plan = best;
    drop_graphs(h);
    forget_handle_in_groups(&h);
    analyse(h, c.stream);
    g_tune[tune_key(h)] = best;
    tune_cache_save();
    return best_us;
}

// ============================================================ batch tuner

// One batched call's time (ms): the median of three runs of `reps` calls.
static double time_batch(int count, const lilac_csr_t *hs, const void *const *xs,
                         void *const *ys, int reps)
{
    Context &c = ctx();
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    double t[3];
    try {
        run_batched(count, hs, xs, ys, c.stream);
        for (double &ti : t) {
            HIPC(hipEventRecord(e0, c.stream));
            for (int i = 0; i < reps; ++i)
                run_batched(count, hs, xs, ys, c.stream);
            HIPC(hipEventRecord(e1, c.stream));
            HIPC(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPC(hipEventElapsedTime(&ms, e0, e1));
            ti = ms / reps;
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::sort(t, t + 3);
    return t[1];
}

// Layout a handle's product uses now.
static int32_t effective_layout(const CsrHandle &h)
{
    return h.use_panels ? LAYOUT_PANELS : h.use_band ? LAYOUT_BAND
                                                     : h.use_hot ? LAYOUT_HOT : LAYOUT_ROWS;
}

// Autotuner for a batch: the matrices are grouped by shape class; class by
// class (most non-zeros first), each layout the grouped launch can take
// (row-class tiles, column panels, band) is tried on every matrix of the
// class and kept if the whole batched call gets at least 1% faster.  The
// chosen plan of each class goes to the tuning cache, so handles of that
// class created later start from it.  Timing the batch itself matters:
// a layout that is fastest for a matrix alone can slow the grouped launch
// down (for instance fewer row blocks than compute units alone, but just
// right among hundreds of others).
static double tune_batch(int count, const lilac_csr_t *hs, const void *const *xs,
                         void *const *ys)
{
    Context &c = ctx();
    std::map<std::string, std::vector<int>> cls;
    for (int j = 0; j < count; ++j) {
        CsrHandle *h = (CsrHandle *)hs[j];
        refresh(*h, c.stream);
        cls[tune_key(*h)].push_back(j);
    }
    std::vector<std::pair<int64_t, std::string>> order;
    for (auto &kv : cls) {
        int64_t nnz = 0;
        for (int j : kv.second)
            nnz += ((const CsrHandle *)hs[j])->nnz;
        order.emplace_back(nnz, kv.first);
    }
    std::sort(order.begin(), order.end(), std::greater<std::pair<int64_t, std::string>>());
    auto apply = [&](const std::vector<int> &members, const std::vector<Plan> &plans) {
        for (size_t k = 0; k < members.size(); ++k) {
            CsrHandle &h = *(CsrHandle *)hs[members[k]];
            drop_graphs(h);
            forget_handle_in_groups(&h);
            h.dev_bytes -= analysis_bytes(h);
            h.plan = plans[k];
            analyse(h, c.stream);
            h.dev_bytes += analysis_bytes(h);
        }
    };
    // the clocks settle under sustained load before anything is compared
    for (int i = 0; i < 20; ++i)
        run_batched(count, hs, xs, ys, c.stream);
    double best = time_batch(count, hs, xs, ys, 5);
    for (auto &o : order) {
        const std::vector<int> &members = cls[o.second];
        std::vector<Plan> cur;
        std::vector<int32_t> lay;
        for (int j : members) {
            cur.push_back(((const CsrHandle *)hs[j])->plan);
            lay.push_back(effective_layout(*(const CsrHandle *)hs[j]));
        }
        for (int32_t cand : {LAYOUT_ROWS, LAYOUT_PANELS, LAYOUT_BAND}) {
            std::vector<Plan> trial = cur;
            for (Plan &p : trial)
                p.layout = cand;
            apply(members, trial);
            bool changed = false;
            for (size_t k = 0; k < members.size(); ++k)
                changed |= effective_layout(*(const CsrHandle *)hs[members[k]]) != lay[k];
            const double t = changed ? time_batch(count, hs, xs, ys, 5) : 1e300;
            if (t < 0.99 * best) {
                best = t;
                cur = trial;
                for (size_t k = 0; k < members.size(); ++k)
                    lay[k] = effective_layout(*(const CsrHandle *)hs[members[k]]);
            } else {
                apply(members, cur);
            }
        }
        g_tune[o.second] = cur.front();
    }
    tune_cache_save();
    return best;
}

// ================================================================== C ABI

template <typename F>
static int guard(F &&f)
{
    try {
        std::lock_guard<std::recursive_mutex> lk(g_mu);
        f();
        return LILAC_OK;
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return LILAC_ERR_OOM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return LILAC_ERR_DEVICE;
    } catch (...) {
        g_last_error = "unknown error";
        return LILAC_ERR_DEVICE;
    }
}

// NULL is HIP's default (null) stream, as for other HIP libraries.
static hipStream_t pick_stream(void *s)
{
    ctx();
    return (hipStream_t)s;
}

}  // namespace lilac

using namespace lilac;

extern "C" {

int lilac_init(int device)
{
    return guard([&] { init_ctx(device); });
}

int lilac_finalize(void)
{
    return guard([&] {
        if (!g_ctx)
            return;
        (void)hipDeviceSynchronize();
        marshal_reset();
        release_all_raw();
        release_group_plans();
        Context &c = *g_ctx;
        dev_free(c.x_buf);
        dev_free(c.y_buf);
        dev_free(c.dot_a);
        dev_free(c.dot_b);
        c.x_buf = c.y_buf = nullptr;
        c.dot_a = c.dot_b = nullptr;
        c.x_cap = c.y_cap = c.dot_cap = 0;
    });
}

const char *lilac_last_error(void) { return g_last_error.c_str(); }

int lilac_version(void) { return 10000; }

int lilac_spmv_csr(int rows, const int *row_ptr, const int *col_idx,
                   const double *vals, const double *x, double *y)
{
    return guard([&] { raw_spmv(rows, row_ptr, col_idx, vals, x, y, LILAC_F64); });
}

int lilac_spmv_csr_f32(int rows, const int *row_ptr, const int *col_idx,
                       const float *vals, const float *x, float *y)
{
    return guard([&] { raw_spmv(rows, row_ptr, col_idx, vals, x, y, LILAC_F32); });
}

double lilac_dot(int64_t n, const double *a, const double *b)
{
    double r = NAN;
    const int st = guard([&] { r = raw_dot(n, a, b); });
    return st == LILAC_OK ? r : NAN;
}

float lilac_dot_f32(int64_t n, const float *a, const float *b)
{
    double r = NAN;
    const int st = guard([&] { r = raw_dot(n, a, b); });
    return st == LILAC_OK ? (float)r : NAN;
}

int lilac_invalidate(const void *ptr)
{
    return guard([&] {
        if (ptr)
            invalidate_ptr(ptr);
    });
}

int lilac_release_all(void)
{
    return guard([&] {
        if (!g_ctx)
            return;
        marshal_reset();
        release_all_raw();
    });
}

int lilac_csr_create(lilac_csr_t *h, int rows, int cols, int64_t nnz,
                     const int *row_ptr, const int *col_idx, const void *vals,
                     lilac_dtype dt, unsigned flags)
{
    return guard([&] {
        if (!h)
            fail(LILAC_ERR_ARG, "handle pointer is NULL");
        *h = nullptr;
        *h = (lilac_csr_t)create_handle(rows, cols, nnz, row_ptr, col_idx, vals,
                                        dt, flags);
    });
}

int lilac_csr_update_values(lilac_csr_t hh, const void *vals)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h || (!vals && h->nnz > 0))
            fail(LILAC_ERR_ARG, "NULL handle or vals");
        if (is_device_ptr(vals))
            HIPC(hipDeviceSynchronize());
        upload_values(*h, vals, ctx().stream);
        values_changed(*h, ctx().stream);
        HIPC(hipStreamSynchronize(ctx().stream));
        if (h->flags & LILAC_KEEP_HOST)
            h->h_vals = vals;
        h->dirty_vals = false;
    });
}

int lilac_csr_invalidate(lilac_csr_t hh)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h)
            fail(LILAC_ERR_ARG, "NULL handle");
        if (!(h->flags & LILAC_KEEP_HOST))
            fail(LILAC_ERR_STATE, "handle was created without LILAC_KEEP_HOST");
        h->dirty_struct = true;
    });
}

int lilac_csr_destroy(lilac_csr_t hh)
{
    return guard([&] { destroy_handle((CsrHandle *)hh); });
}

int lilac_csr_info(lilac_csr_t hh, lilac_csr_info_t *out)
{
    return guard([&] {
        const CsrHandle *h = (const CsrHandle *)hh;
        if (!h || !out)
            fail(LILAC_ERR_ARG, "NULL argument");
        std::memset(out, 0, sizeof(*out));
        out->rows = h->rows;
        out->cols = h->cols;
        out->nnz = h->nnz;
        out->device_bytes = h->dev_bytes;
        out->dtype = h->dt;
        out->nbins = NCLASS;
        for (int c = 0; c < NCLASS; ++c) {
            out->bin_upper[c] = h->plan.upper[c];
            out->bin_count[c] = h->bin_off.empty() ? 0 : h->bin_off[c + 1] - h->bin_off[c];
        }
        out->chunk = h->plan.chunk;
        out->nchunks = h->nchunks;
        out->ntiles = h->ntiles;
        out->layout = h->use_panels ? LAYOUT_PANELS
                      : h->use_hot  ? LAYOUT_HOT
                      : h->use_band ? LAYOUT_BAND
                                    : LAYOUT_ROWS;
        out->npanels = h->use_panels ? h->pan.np : 0;
    });
}

int lilac_csr_analysis(lilac_csr_t hh, int *bin_off, int *bin_rows, int *c_row,
                       int *c_k0, int *c_k1)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h)
            fail(LILAC_ERR_ARG, "NULL handle");
        hipStream_t s = ctx().stream;
        refresh(*h, s);
        if (bin_off)
            std::memcpy(bin_off, h->bin_off.data(), (NCLASS + 1) * sizeof(int));
        if (bin_rows && h->rows)
            HIPC(hipMemcpyAsync(bin_rows, h->d_bin_rows, (size_t)h->rows * 4,
                                hipMemcpyDeviceToHost, s));
        const size_t cb = (size_t)h->nchunks * 4;
        if (cb && c_row)
            HIPC(hipMemcpyAsync(c_row, h->d_c_row, cb, hipMemcpyDeviceToHost, s));
        if (cb && c_k0)
            HIPC(hipMemcpyAsync(c_k0, h->d_c_k0, cb, hipMemcpyDeviceToHost, s));
        if (cb && c_k1)
            HIPC(hipMemcpyAsync(c_k1, h->d_c_k1, cb, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
    });
}

int lilac_csr_set_plan(lilac_csr_t hh, const int *upper, const int *rpg, int chunk)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h)
            fail(LILAC_ERR_ARG, "NULL handle");
        Plan p = h->plan;
        if (upper)
            for (int c = 0; c < NCLASS - 1; ++c)
                p.upper[c] = upper[c];
        if (rpg)
            for (int c = 0; c < NCLASS; ++c)
                p.rpg[c] = rpg[c];
        if (chunk > 0)
            p.chunk = chunk;
        check_plan(p);
        hipStream_t s = ctx().stream;
        refresh(*h, s);
        drop_graphs(*h);
        forget_handle_in_groups(h);
        h->plan = p;
        h->dev_bytes -= analysis_bytes(*h);
        analyse(*h, s);
        h->dev_bytes += analysis_bytes(*h);
    });
}

int lilac_csr_set_layout(lilac_csr_t hh, int layout)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h)
            fail(LILAC_ERR_ARG, "NULL handle");
        Plan p = h->plan;
        p.layout = layout;
        check_plan(p);
        hipStream_t s = ctx().stream;
        refresh(*h, s);
        h->dev_bytes -= analysis_bytes(*h);
        h->plan = p;
        analyse(*h, s);
        h->dev_bytes += analysis_bytes(*h);
    });
}

int lilac_spmv(lilac_csr_t hh, const void *x, void *y, void *stream)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h)
            fail(LILAC_ERR_ARG, "NULL handle");
        if (h->rows > 0 && (!y || (h->cols > 0 && !x)))
            fail(LILAC_ERR_ARG, "NULL vector");
        hipStream_t s = pick_stream(stream);
        refresh(*h, s);
        spmv_enqueue(*h, x, y, epi_none(), nullptr, false, s);
    });
}

int lilac_spmv_dot(lilac_csr_t hh, const void *x, void *y, const void *w,
                   double *out, void *stream)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h || !out)
            fail(LILAC_ERR_ARG, "NULL argument");
        if (h->dt != LILAC_F64)
            fail(LILAC_ERR_UNSUPPORTED, "fused dot is only provided for float64");
        if (h->rows > 0 && (!y || !w || (h->cols > 0 && !x)))
            fail(LILAC_ERR_ARG, "NULL vector");
        hipStream_t s = pick_stream(stream);
        refresh(*h, s);
        if (h->rows == 0) {
            launch_fill_bytes_zero(out, 8, s);
            return;
        }
        spmv_enqueue(*h, x, y, epi_none(), w, true, s);
        launch_sum_parts(h->d_dot_part, h->grid + h->fin_blocks, out, s);
    });
}

int lilac_dot_dev(int64_t n, const void *a, const void *b, void *out, lilac_dtype dtype,
                  void *stream)
{
    return guard([&] {
        if (n < 0 || !out)
            fail(LILAC_ERR_ARG, "bad argument");
        if (dtype != LILAC_F64 && dtype != LILAC_F32)
            fail(LILAC_ERR_ARG, "unknown dtype");
        hipStream_t s = pick_stream(stream);
        if (n == 0) {
            launch_fill_bytes_zero(out, dtype == LILAC_F32 ? 4 : 8, s);
            return;
        }
        if (!a || !b)
            fail(LILAC_ERR_ARG, "NULL vector");
        Context &c = ctx();
        const int32_t np = blas1_parts(n);
        // partials in the library's scratch: calls on different streams
        // must not overlap
        if (dtype == LILAC_F32) {
            launch_dot_parts_f32(n, (const float *)a, (const float *)b, c.dot_part, np, s);
            launch_sum_parts_f32(c.dot_part, np, (float *)out, s);
        } else {
            launch_dot_parts(n, (const double *)a, (const double *)b, c.dot_part, np, s);
            launch_sum_parts(c.dot_part, np, (double *)out, s);
        }
    });
}

int lilac_cg(lilac_csr_t hh, const double *b, double *x, int iters,
             unsigned flags, void *stream, double *rho_out, int *iters_done)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h)
            fail(LILAC_ERR_ARG, "NULL handle");
        run_cg(*h, b, x, iters, flags, pick_stream(stream), rho_out, iters_done);
    });
}

int lilac_cg_noalloc(lilac_csr_t hh, const double *b, double *x, int iters, void *stream)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h)
            fail(LILAC_ERR_ARG, "NULL handle");
        if (h->dt != LILAC_F64)
            fail(LILAC_ERR_UNSUPPORTED, "CG needs a float64 handle");
        if (h->rows != h->cols)
            fail(LILAC_ERR_ARG, "CG needs a square matrix");
        if (iters < 0)
            fail(LILAC_ERR_ARG, "iters must be >= 0");
        if ((int64_t)h->rows > kNoAllocRows)
            fail(LILAC_ERR_ARG, "matrix has " + std::to_string(h->rows) +
                                    " rows; the fixed CG state holds at most " +
                                    std::to_string(kNoAllocRows));
        if (h->dirty_struct || h->dirty_vals)
            fail(LILAC_ERR_STATE, "handle has pending updates; bring it up to date "
                                  "with a call that may allocate first");
        if (h->rows == 0)
            return;
        if (!b || !x)
            fail(LILAC_ERR_ARG, "b or x is NULL");
        if (!is_device_ptr(b) || !is_device_ptr(x))
            fail(LILAC_ERR_ARG, "b and x must be device arrays");
        char *base = scratch_on_current_device();
        double *r = (double *)base;
        double *p = r + kNoAllocRows;
        double *sv = p + kNoAllocRows;
        double *w = sv + kNoAllocRows;
        double *part = w + kNoAllocRows;
        CgScalars *sc = (CgScalars *)(part + kNoAllocPart);
        cg_enqueue_state(*h, b, x, iters, r, p, sv, w, part, sc, (hipStream_t)stream);
    });
}

int lilac_pagerank(lilac_csr_t hh, float damping, int iters, float *x_inout,
                   void *stream)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h)
            fail(LILAC_ERR_ARG, "NULL handle");
        run_pagerank(*h, damping, iters, x_inout, pick_stream(stream));
    });
}

int lilac_spmv_batched(int count, const lilac_csr_t *hs, const void *const *xs,
                       void *const *ys, void *stream)
{
    return guard([&] { run_batched(count, hs, xs, ys, pick_stream(stream)); });
}

// ------------------------------------------------- 64-bit row offsets

// A matrix with int64 row offsets, kept as consecutive row parts that are
// ordinary handles (32-bit offsets rebased to each part's first entry).
struct Csr64 {
    int rows = 0, cols = 0;
    int64_t nnz = 0;
    lilac_dtype dt = LILAC_F64;
    std::vector<CsrHandle *> parts;
    std::vector<int32_t> first_row;
};

// Most non-zeros of one part: below the 32-bit handle bound with room to
// spare, or less when LILAC_PART_NNZ says so.
static int64_t part_nnz_limit()
{
    int64_t lim = ((int64_t)1 << 31) - ((int64_t)1 << 20);
    if (const char *e = std::getenv("LILAC_PART_NNZ")) {
        const long long v = std::strtoll(e, nullptr, 10);
        if (v >= 1 && v < lim)
            lim = v;
    }
    return lim;
}

static void destroy_csr64(Csr64 *m)
{
    if (!m)
        return;
    (void)hipDeviceSynchronize();
    for (CsrHandle *h : m->parts)
        destroy_handle(h);
    delete m;
}

static Csr64 *create_csr64(int rows, int cols, int64_t nnz, const int64_t *row_ptr,
                           const int32_t *col, const void *vals, lilac_dtype dt)
{
    if (rows < 0)
        fail(LILAC_ERR_ARG, "rows must be >= 0");
    if (nnz < 0)
        fail(LILAC_ERR_ARG, "nnz must be >= 0");
    if (!row_ptr)
        fail(LILAC_ERR_ARG, "row_ptr is NULL");
    if (nnz > 0 && (!col || !vals))
        fail(LILAC_ERR_ARG, "col_idx or vals is NULL");
    if (dt != LILAC_F64 && dt != LILAC_F32)
        fail(LILAC_ERR_ARG, "unknown dtype");
    // the offsets are needed on the host to cut the parts
    std::vector<int64_t> rp((size_t)rows + 1);
    if (is_device_ptr(row_ptr)) {
        HIPC(hipDeviceSynchronize());
        HIPC(hipMemcpy(rp.data(), row_ptr, rp.size() * 8, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(rp.data(), row_ptr, rp.size() * 8);
    }
    if (rp[0] != 0 || rp[rows] != nnz)
        fail(LILAC_ERR_CSR, "invalid CSR: row_ptr[0] != 0 or row_ptr[rows] != nnz");
    for (int64_t r = 0; r < rows; ++r)
        if (rp[r + 1] < rp[r])
            fail(LILAC_ERR_CSR, "invalid CSR: row_ptr decreases");
    const int64_t lim = part_nnz_limit();
    const size_t vs = dtype_size(dt);
    auto *m = new Csr64();
    m->rows = rows;
    m->nnz = nnz;
    m->dt = dt;
    try {
        int64_t r0 = 0;
        std::vector<int32_t> rb;
        while (r0 < rows) {
            if (rp[r0 + 1] - rp[r0] > lim)
                fail(LILAC_ERR_UNSUPPORTED, "a row has more non-zeros than one part holds");
            // the last row end within the bound
            const int64_t r1 =
                (int64_t)(std::upper_bound(rp.begin() + r0 + 1, rp.end(), rp[r0] + lim) -
                          rp.begin()) - 1;
            const int64_t e0 = rp[r0];
            rb.resize((size_t)(r1 - r0) + 1);
            for (int64_t r = r0; r <= r1; ++r)
                rb[(size_t)(r - r0)] = (int32_t)(rp[r] - e0);
            const int64_t pn = rp[r1] - e0;
            CsrHandle *h = create_handle((int)(r1 - r0), cols, pn, rb.data(),
                                         pn > 0 ? col + e0 : col,
                                         pn > 0 ? (const char *)vals + e0 * (int64_t)vs : vals,
                                         dt, 0);
            m->parts.push_back(h);
            m->first_row.push_back((int32_t)r0);
            m->cols = std::max(m->cols, h->cols);
            r0 = r1;
        }
        if (cols >= 0)
            m->cols = cols;
    } catch (...) {
        destroy_csr64(m);
        throw;
    }
    return m;
}

int lilac_csr64_create(lilac_csr64_t *h, int rows, int cols, int64_t nnz,
                       const int64_t *row_ptr, const int *col_idx, const void *vals,
                       lilac_dtype dt)
{
    return guard([&] {
        if (!h)
            fail(LILAC_ERR_ARG, "handle pointer is NULL");
        *h = nullptr;
        *h = (lilac_csr64_t)create_csr64(rows, cols, nnz, row_ptr, col_idx, vals, dt);
    });
}

int lilac_csr64_spmv(lilac_csr64_t hh, const void *x, void *y, void *stream)
{
    return guard([&] {
        Csr64 *m = (Csr64 *)hh;
        if (!m)
            fail(LILAC_ERR_ARG, "NULL handle");
        if (m->rows > 0 && (!y || (m->cols > 0 && !x)))
            fail(LILAC_ERR_ARG, "NULL vector");
        const size_t n = m->parts.size();
        if (n == 0)
            return;
        const size_t vs = dtype_size(m->dt);
        std::vector<lilac_csr_t> hs(n);
        std::vector<const void *> xs(n, x);
        std::vector<void *> ys(n);
        for (size_t p = 0; p < n; ++p) {
            hs[p] = (lilac_csr_t)m->parts[p];
            ys[p] = (char *)y + (int64_t)m->first_row[p] * (int64_t)vs;
        }
        run_batched((int)n, hs.data(), xs.data(), ys.data(), pick_stream(stream));
    });
}

int lilac_csr64_info(lilac_csr64_t hh, int *rows, int *cols, int64_t *nnz, int *nparts)
{
    return guard([&] {
        const Csr64 *m = (const Csr64 *)hh;
        if (!m)
            fail(LILAC_ERR_ARG, "NULL handle");
        if (rows)
            *rows = m->rows;
        if (cols)
            *cols = m->cols;
        if (nnz)
            *nnz = m->nnz;
        if (nparts)
            *nparts = (int)m->parts.size();
    });
}

int lilac_csr64_destroy(lilac_csr64_t hh)
{
    return guard([&] { destroy_csr64((Csr64 *)hh); });
}

int lilac_bfs(lilac_csr_t hh, int source, int *level, int *nlevels, void *stream)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h || !level)
            fail(LILAC_ERR_ARG, "NULL argument");
        if (h->cols > h->rows)
            fail(LILAC_ERR_ARG, "BFS needs cols <= rows (a graph's adjacency)");
        if (source < 0 || source >= h->rows)
            fail(LILAC_ERR_ARG, "source out of range");
        if (!is_device_ptr(level))
            fail(LILAC_ERR_ARG, "level must be a device array");
        hipStream_t s = pick_stream(stream);
        refresh(*h, s);
        Context &c = ctx();
        launch_fill_i32(level, h->rows, -1, s);
        launch_fill_i32(level + source, 1, 0, s);
        const MatDesc m = make_desc(*h, nullptr, nullptr, nullptr, nullptr);
        const int32_t grid = own_layout(*h) ? tile_grid(h->dt) : h->grid;
        int32_t depth = 0;
        for (;; ++depth) {
            launch_fill_i32(c.status, 1, 0, s);
            launch_bfs_step(h->d_tiles, h->ntiles, grid, m, level, depth, c.status, s);
            int32_t changed = 0;
            HIPC(hipMemcpyAsync(&changed, c.status, 4, hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            if (!changed)
                break;
        }
        if (nlevels)
            *nlevels = depth + 1;
    });
}

int lilac_spmv_jds(int rows, int max_len, const int *perm, const int *nzcnt,
                   const int *jd_ptr, const int *jd_col, const double *jd_val,
                   const double *x, double *y)
{
    return guard([&] {
        if (rows < 0 || max_len < 0)
            fail(LILAC_ERR_ARG, "negative size");
        if (rows == 0)
            return;
        if (!perm || !nzcnt || !jd_ptr || !y || (max_len > 0 && (!jd_col || !jd_val || !x)))
            fail(LILAC_ERR_ARG, "NULL argument");
        Context &c = ctx();
        hipStream_t s = c.stream;
        const bool any_dev = is_device_ptr(perm) || is_device_ptr(nzcnt) ||
                             is_device_ptr(jd_ptr) || is_device_ptr(jd_col) ||
                             is_device_ptr(jd_val) || is_device_ptr(x) || is_device_ptr(y);
        if (any_dev)
            HIPC(hipDeviceSynchronize());
        // jd_ptr[max_len] is the number of entries
        int32_t nnz = 0;
        if (is_device_ptr(jd_ptr)) {
            HIPC(hipMemcpyAsync(&nnz, jd_ptr + max_len, 4, hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
        } else {
            nnz = jd_ptr[max_len];
        }
        if (nnz < 0)
            fail(LILAC_ERR_ARG, "jd_ptr[max_len] < 0");
        // device copies of host arrays for this call (JDS is not cached)
        std::vector<void *> tmp;
        auto dev = [&](const void *p, size_t bytes) -> const void * {
            if (!p || is_device_ptr(p))
                return p;
            void *d = dev_alloc(bytes);
            tmp.push_back(d);
            HIPC(hipMemcpyAsync(d, p, bytes, hipMemcpyHostToDevice, s));
            return d;
        };
        int32_t cols = 0;
        try {
            const int32_t *d_perm = (const int32_t *)dev(perm, (size_t)rows * 4);
            const int32_t *d_nz = (const int32_t *)dev(nzcnt, (size_t)rows * 4);
            const int32_t *d_ptr = (const int32_t *)dev(jd_ptr, (size_t)(max_len + 1) * 4);
            const int32_t *d_col = (const int32_t *)dev(jd_col, (size_t)std::max(nnz, 1) * 4);
            const double *d_val = (const double *)dev(jd_val, (size_t)std::max(nnz, 1) * 8);
            // the columns bound the x that must be present
            launch_fill_i32(c.status + 1, 1, -1, s);
            launch_fill_i32(c.status, 1, 0, s);
            launch_validate(0, c.total, nnz, d_col, -1, c.status, s);
            int32_t st[2];
            HIPC(hipMemcpyAsync(st, c.status, 8, hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            if (st[0] & 8)
                fail(LILAC_ERR_CSR, "negative column index in JDS");
            cols = st[1] + 1;
            const double *d_x = (const double *)dev(x, (size_t)std::max(cols, 1) * 8);
            int32_t *iperm = (int32_t *)dev_alloc((size_t)rows * 4);
            tmp.push_back(iperm);
            const bool y_dev = is_device_ptr(y);
            double *d_y = y_dev ? y : (double *)dev_alloc((size_t)rows * 8);
            if (!y_dev)
                tmp.push_back(d_y);
            launch_fill_i32(iperm, rows, -1, s);
            launch_invert_perm(rows, d_perm, iperm, s);
            launch_spmv_jds(rows, max_len, nnz, iperm, d_nz, d_ptr, d_col, d_val, d_x,
                            d_y, s);
            if (!y_dev)
                HIPC(hipMemcpyAsync(y, d_y, (size_t)rows * 8, hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
        } catch (...) {
            (void)hipStreamSynchronize(s);
            for (void *d : tmp)
                dev_free(d);
            throw;
        }
        for (void *d : tmp)
            dev_free(d);
    });
}

int lilac_csr_to_jds(lilac_csr_t hh, int *perm, int *nzcnt, int *jd_ptr, int jd_ptr_len,
                     int *jd_col, void *jd_val, int *max_len, void *stream)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h || !max_len)
            fail(LILAC_ERR_ARG, "NULL handle or max_len");
        Context &c = ctx();
        hipStream_t s = stream ? (hipStream_t)stream : c.stream;
        refresh(*h, s);
        const int32_t ml = jds_max_len(*h, c.total, s);
        *max_len = ml;
        if (!jd_ptr)
            return;  // size query
        if (jd_ptr_len < ml + 1)
            fail(LILAC_ERR_ARG, "jd_ptr holds fewer than max_len + 1 entries");
        if (h->rows > 0 && (!perm || !nzcnt))
            fail(LILAC_ERR_ARG, "NULL perm or nzcnt");
        if (h->nnz > 0 && (!jd_col || !jd_val))
            fail(LILAC_ERR_ARG, "NULL jd_col or jd_val");
        for (const void *p : {(const void *)perm, (const void *)nzcnt, (const void *)jd_ptr,
                              (const void *)jd_col, (const void *)jd_val})
            if (p && !is_device_ptr(p))
                fail(LILAC_ERR_ARG, "JDS outputs must be device memory");
        jds_convert(*h, ml, perm, nzcnt, jd_ptr, jd_col, jd_val, s);
    });
}

int lilac_hbm_stream(const void *src, void *dst, int64_t bytes, int groups_per_cu,
                     void *stream)
{
    return guard([&] {
        if (!src || bytes < 0 || (bytes & 15) || (((uintptr_t)src | (uintptr_t)dst) & 15))
            fail(LILAC_ERR_ARG, "src (and dst) must be 16-byte aligned, bytes a multiple of 16");
        if (groups_per_cu < 1 || groups_per_cu > 64)
            fail(LILAC_ERR_ARG, "groups_per_cu must be in [1, 64]");
        if (!is_device_ptr(src) || (dst && !is_device_ptr(dst)))
            fail(LILAC_ERR_ARG, "src and dst must be device memory");
        Context &c = ctx();
        launch_stream(src, dst, bytes, c.cu * groups_per_cu, (uint32_t *)c.total,
                      pick_stream(stream));
    });
}

int lilac_spmv_batched_tune(int count, const lilac_csr_t *hs, const void *const *xs,
                            void *const *ys, double *best_ms)
{
    return guard([&] {
        if (count < 0 || (count > 0 && (!hs || !xs || !ys)))
            fail(LILAC_ERR_ARG, "bad batch");
        for (int j = 0; j < count; ++j)
            if (!hs[j])
                fail(LILAC_ERR_ARG, "NULL handle");
        const double ms = count ? tune_batch(count, hs, xs, ys) : 0.0;
        if (best_ms)
            *best_ms = ms;
    });
}

int lilac_tune_clear(void)
{
    return guard([&] {
        tune_cache_load();   // a later load must not bring the file's plans back
        g_tune.clear();
    });
}

int lilac_csr_tune_class(lilac_csr_t hh, char *buf, int cap)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h || !buf || cap < 1)
            fail(LILAC_ERR_ARG, "NULL handle or buffer");
        const std::string k = tune_key(*h);
        if ((int)k.size() >= cap)
            fail(LILAC_ERR_ARG, "buffer too small");
        std::memcpy(buf, k.c_str(), k.size() + 1);
    });
}

int lilac_csr_tune(lilac_csr_t hh, double *best_us)
{
    return guard([&] {
        CsrHandle *h = (CsrHandle *)hh;
        if (!h)
            fail(LILAC_ERR_ARG, "NULL handle");
        const double us = tune_handle(*h);
        if (best_us)
            *best_us = us;
    });
}

}  // extern "C"

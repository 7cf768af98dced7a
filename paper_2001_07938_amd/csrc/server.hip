// Request server: continuous batching of SpMV and CG-solve requests over a
// pool of device-resident matrices.
//
// The scheduling (admission against the HBM budget, the resident pool and
// its LRU-2 eviction, request slots, batching into ticks, statistics) is the
// device-free serve::Core (serve_core.h).  This file is its executor on
// the GPU:
//  - uploads run on two threads with a stream each: the CSR arrays go from
//    pinned host memory straight into the device arrays the matrix handle
//    then takes over, and the handle's analysis and layout build follow;
//  - every device byte a matrix holds is charged to an allocator account of
//    its own whose limit is the upload's reserve, under the server's account
//    whose limit is the budget, so the budget is a hard bound, the reserve
//    is checked, and what a resident matrix holds is known exactly;
//  - requests run in two lanes with a stream each: matrices of at least
//    kHeavyNnz non-zeros (one product alone takes tens of microseconds) in
//    the heavy lane, the others in the light lane, so a short request never
//    waits out a long product in its tick;
//  - a tick is ONE grouped product over every active request of a lane (y = A x for
//    SpMV requests, q = A p for the next iteration of every active CG
//    request; row-class tiles, column panels and band blocks each in one
//    launch), then three batched kernels that advance every CG by one
//    iteration.  Each request's reductions have shapes fixed by its own
//    matrix, so a result does not depend on what it was batched with.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <vector>

#include "lilac_internal.h"
#include "serve_core.h"

namespace lilac {
namespace {

using Clock = std::chrono::steady_clock;

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               Clock::now().time_since_epoch())
        .count();
}

constexpr int kUploadThreads = 2;
constexpr int64_t kHeavyNnz = 1 << 23;
// Compute units kept for uploads: the upload streams run on these only and
// the light lane's ticks on the others, so a matrix's checks and analysis
// never queue behind a long tick (a tick's kernels can hold every CU for
// hundreds of microseconds) and short requests never wait out an upload.
// The heavy lane keeps every CU: its column-panel products launch one
// workgroup per CU and would take a second round on fewer.
constexpr int kUploadCus = 16;
// Largest build temporary an upload thread keeps between uploads (its
// builds then call no hipFree, which waits for every stream of the device).
constexpr size_t kTmpCacheLimit = (size_t)16 << 20;

// Streams on a subset of the compute units (mask bits [lo, hi)), or plain
// streams when the device is too small to split or refuses the mask.
void create_masked_stream(hipStream_t *st, int lo, int hi)
{
    const int cus = device_cu_count();
    if (cus < 4 * kUploadCus) {
        HIPC(hipStreamCreateWithFlags(st, hipStreamNonBlocking));
        return;
    }
    std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0u);
    for (int c = lo; c < hi && c < cus; ++c)
        mask[(size_t)c / 32] |= 1u << (c % 32);
    if (hipExtStreamCreateWithCUMask(st, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
        (void)hipGetLastError();   // masks refused: a plain stream serves too
        HIPC(hipStreamCreateWithFlags(st, hipStreamNonBlocking));
    }
}

struct SMatrix {
    int rows = 0, cols = 0;
    int64_t nnz = 0;
    const int32_t *rp = nullptr, *col = nullptr;   // pinned host copy
    const double *vals = nullptr;
    void *pin = nullptr;
    CsrHandle *h = nullptr;                 // set by the upload thread
    double *vin = nullptr;                  // trace-mode operand (all ones)
    Account acct;                           // every device byte it holds
    int64_t nchunks = 0;                    // of the resident handle
};

// Per-slot device workspace of an admitted request: CG vectors (r, p,
// w = A r, s), its own output vector for trace-mode requests, partials,
// the solve's scalars, chunk sums.
struct Slot {
    int64_t cap_chunks = 0;
    double *r = nullptr, *p = nullptr, *w = nullptr, *s = nullptr, *x = nullptr;
    double *rw = nullptr, *rr = nullptr;  // kBlock (r.w) and 2*kBlock (r.r) partials
    int32_t *done = nullptr;              // 256 bytes: done flag, then the scalars
    double *chunk = nullptr;
};

// A resident copy given up by the scheduler, freed by an upload thread.
struct Evicted {
    int mid = -1;
    CsrHandle *h = nullptr;
    double *vin = nullptr;
};

// Tables of one tick, in pinned memory and on the device.  Sized once for
// max_active requests.
struct TickBuf {
    hipEvent_t ev = nullptr;
    char *host = nullptr, *dev = nullptr;
    size_t cap = 0;
};

size_t per_request_table_bytes()
{
    return sizeof(MatDesc) + 4 + 2 * sizeof(CgSeg) + sizeof(PanelDesc) +
           sizeof(PanelIO) + 4 + sizeof(BandDesc) + sizeof(PanelIO) + 4;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Server;

class HipExec : public serve::Executor {
  public:
    explicit HipExec(Server *s) : S(s) {}
    int64_t now_ns() override { return lilac::now_ns(); }
    int64_t upload_reserve(int mid) override;
    void start_upload(int mid) override;
    void evict(int mid) override;
    int64_t slot_need(int slot, int mid) override;
    void prepare_slot(int slot, int mid) override;
    void release_slot(int slot) override;
    int lane_of(int mid) override;
    void launch_tick(int lane, int tick, const std::vector<serve::Request *> &reqs) override;
    bool tick_done(int lane, int tick) override;
    void wait_tick(int lane, int tick) override;
    void run_one(serve::Request *r) override;

  private:
    Server *S;
};

struct Server {
    lilac_server_config cfg{};
    bool fifo = false;
    int max_rows = 0;
    hipStream_t stream[serve::kLanes] = {};
    hipStream_t up_stream[kUploadThreads] = {};
    std::vector<SMatrix> mats;
    std::vector<Slot> slots;
    TickBuf ticks[serve::kLanes][2];
    Account acct;                  // the server's own: limit = budget
    HipExec exec{this};
    serve::Core *core = nullptr;
    std::thread sched;
    std::thread uploader[kUploadThreads];
    std::atomic<bool> stop{false};
    // uploads and frees of evicted copies; an upload starts only when no
    // free is queued or running, so that the memory a plan counted as
    // released is back before anything new is allocated
    std::mutex up_mu;
    std::condition_variable up_cv;
    std::deque<int> up_q;
    std::deque<Evicted> free_q;
    int freeing = 0;
    TmpCache tmp[kUploadThreads];
    std::atomic<bool> started{false};
    std::mutex start_mu;
};

// ------------------------------------------------------------- accounting

// Bound on the device bytes an upload of a float64 matrix holds at any
// moment: the CSR arrays (padded), the row-class analysis and its
// temporaries, the larger of the column-panel and band copies with their
// build temporaries, the trace operand, and the 256-byte rounding of each
// allocation.  Upload threads run under an account with this limit, so a
// build that needed more would fail loudly instead of passing the budget.
int64_t upload_bound(const SMatrix &m, bool cg_state)
{
    const int64_t rows = m.rows, nnz = m.nnz;
    const int64_t npad = padded_nnz(nnz);
    int64_t b = 0;
    b += (rows + 1) * 4 + npad * 12;                       // CSR
    b += rows * 28 + (nnz / 2048 + 1) * 24 + (1 << 20);    // classes, tiles, chunks, temps
    b += (nnz + kPad) * 12 + 256 * (rows + 257) + (2 << 20);  // panel or band copy + build
    b += (int64_t)std::max(1, m.cols) * 8;                 // trace operand
    if (cg_state)
        b += rows * 32 + 2 * 1024 * 8 + 256;               // CG state of the plain path
    b += 64 * 256;                                         // allocation rounding
    return b;
}

int64_t slot_bytes_for(const Server *S, int64_t chunks)
{
    const int64_t n = std::max(1, S->max_rows);
    return 5 * (int64_t)round256((size_t)n * 8) + (int64_t)round256(kBlock * 8) +
           (int64_t)round256(2 * kBlock * 8) + 256 +
           (chunks > 0 ? (int64_t)round256((size_t)chunks * 8) : 0);
}

// ------------------------------------------------------------- uploads

// Frees an evicted copy (hipFree waits for the whole device, which is why
// the scheduler does not do it itself).
void free_evicted(Server *S, const Evicted &e)
{
    std::lock_guard<std::recursive_mutex> lk(lib_mutex());
    destroy_handle(e.h);
    dev_free(e.vin);
    if (S->mats[(size_t)e.mid].acct.in_use != 0)
        fail(LILAC_ERR_DEVICE, "evicted matrix still holds device memory");
}

// Blocks until every queued eviction has given its memory back.
void wait_frees(Server *S)
{
    std::unique_lock<std::mutex> lk(S->up_mu);
    S->up_cv.wait(lk, [&] {
        return (S->free_q.empty() && S->freeing == 0) || S->stop.load();
    });
}

void upload_loop(Server *S, int t)
{
    if (hipSetDevice(lib_device()) != hipSuccess)
        return;
    hipStream_t us = S->up_stream[t];
    thread_tmp_cache() = &S->tmp[t];
    while (true) {
        int id = -1;
        Evicted ev;
        {
            std::unique_lock<std::mutex> lk(S->up_mu);
            S->up_cv.wait(lk, [&] {
                return !S->free_q.empty() || (!S->up_q.empty() && S->freeing == 0) ||
                       S->stop.load();
            });
            if (S->stop.load())
                break;
            if (!S->free_q.empty()) {
                ev = S->free_q.front();
                S->free_q.pop_front();
                S->freeing += 1;
            } else {
                id = S->up_q.front();
                S->up_q.pop_front();
            }
        }
        if (id < 0) {
            std::string why;
            try {
                free_evicted(S, ev);
            } catch (const Error &e) {
                why = e.msg;
            }
            {
                std::lock_guard<std::mutex> lk(S->up_mu);
                S->freeing -= 1;
                S->up_cv.notify_all();
            }
            if (!why.empty())
                S->core->die(why);
            continue;
        }
        SMatrix &m = S->mats[(size_t)id];
        const int64_t npad = padded_nnz(m.nnz);
        int32_t *d_rp = nullptr, *d_col = nullptr;
        double *d_vals = nullptr;
        CsrHandle *h = nullptr;
        double *vin = nullptr;
        bool ok = true;
        std::string why;
        thread_account() = &m.acct;
        try {
            {
                std::lock_guard<std::recursive_mutex> lk(lib_mutex());
                m.acct.peak = m.acct.in_use;
                d_rp = (int32_t *)dev_alloc((size_t)(m.rows + 1) * 4);
                d_col = (int32_t *)dev_alloc((size_t)npad * 4);
                d_vals = (double *)dev_alloc((size_t)npad * 8);
            }
            // the copies run without the library lock (the scheduler may
            // need it meanwhile); the arrays become the handle's own
            HIPC(hipMemcpyAsync(d_rp, m.rp, (size_t)(m.rows + 1) * 4,
                                hipMemcpyHostToDevice, us));
            if (m.nnz) {
                HIPC(hipMemcpyAsync(d_col, m.col, (size_t)m.nnz * 4,
                                    hipMemcpyHostToDevice, us));
                HIPC(hipMemcpyAsync(d_vals, m.vals, (size_t)m.nnz * 8,
                                    hipMemcpyHostToDevice, us));
            }
            HIPC(hipStreamSynchronize(us));
            std::lock_guard<std::recursive_mutex> lk(lib_mutex());
            int32_t *a = d_rp, *c = d_col;
            double *v = d_vals;
            d_rp = d_col = nullptr;
            d_vals = nullptr;
            h = create_handle_adopt(m.rows, m.cols, m.nnz, a, c, v, LILAC_F64, us);
            if (S->fifo && m.rows == m.cols && m.rows > 0)
                handle_cg_prepare(*h);   // the plain path's CG state, counted here
            vin = (double *)dev_alloc((size_t)std::max(1, m.cols) * 8);
            launch_fill_f64(vin, std::max(1, m.cols), 1.0, us);
            HIPC(hipStreamSynchronize(us));
        } catch (const Error &e) {
            ok = false;
            why = e.msg;
            std::lock_guard<std::recursive_mutex> lk(lib_mutex());
            dev_free(d_rp);
            dev_free(d_col);
            dev_free(d_vals);
            dev_free(vin);
            vin = nullptr;
            if (h)
                destroy_handle(h);
            h = nullptr;
        }
        thread_account() = nullptr;
        int64_t held = 0;
        {
            std::lock_guard<std::recursive_mutex> lk(lib_mutex());
            m.h = h;
            m.vin = vin;
            m.nchunks = h ? h->nchunks : 0;
            held = m.acct.in_use;
            m.acct.limit = INT64_MAX;   // the reserve no longer applies
        }
        S->core->upload_done(id, ok, held, why);
    }
    tmp_cache_release(S->tmp[t]);
    thread_tmp_cache() = nullptr;
}

// ------------------------------------------------------------- executor

int64_t HipExec::upload_reserve(int mid)
{
    return upload_bound(S->mats[(size_t)mid], S->fifo);
}

void HipExec::start_upload(int mid)
{
    SMatrix &m = S->mats[(size_t)mid];
    {
        std::lock_guard<std::recursive_mutex> lk(lib_mutex());
        m.acct.limit = upload_bound(m, S->fifo);
    }
    std::lock_guard<std::mutex> lk(S->up_mu);
    S->up_q.push_back(mid);
    S->up_cv.notify_one();
}

// The copy goes to the upload threads to be freed; uploads and new slot
// memory wait for that free (wait_frees), so the device never holds more
// than the plan while the scheduler moves on at once.
void HipExec::evict(int mid)
{
    SMatrix &m = S->mats[(size_t)mid];
    Evicted e;
    e.mid = mid;
    e.h = m.h;
    e.vin = m.vin;
    m.h = nullptr;
    m.vin = nullptr;
    std::lock_guard<std::mutex> lk(S->up_mu);
    S->free_q.push_back(e);
    S->up_cv.notify_all();
}

int64_t HipExec::slot_need(int slot, int mid)
{
    const Slot *sl = slot < (int)S->slots.size() ? &S->slots[(size_t)slot] : nullptr;
    const int64_t chunks =
        std::max<int64_t>(sl ? sl->cap_chunks : 0, S->mats[(size_t)mid].nchunks);
    return slot_bytes_for(S, chunks);
}

void HipExec::prepare_slot(int slot, int mid)
{
    while ((int)S->slots.size() <= slot)
        S->slots.push_back(Slot());
    Slot &sl = S->slots[(size_t)slot];
    const int64_t n = std::max(1, S->max_rows);
    const int64_t nc = S->mats[(size_t)mid].nchunks;
    if (sl.r && sl.cap_chunks >= nc)
        return;   // a slot that fits: nothing to allocate, no lock
    wait_frees(S);
    std::lock_guard<std::recursive_mutex> lk(lib_mutex());
    if (!sl.r) {
        sl.r = (double *)dev_alloc((size_t)n * 8);
        sl.p = (double *)dev_alloc((size_t)n * 8);
        sl.w = (double *)dev_alloc((size_t)n * 8);
        sl.s = (double *)dev_alloc((size_t)n * 8);
        sl.x = (double *)dev_alloc((size_t)n * 8);
        sl.rw = (double *)dev_alloc(kBlock * 8);
        sl.rr = (double *)dev_alloc(2 * kBlock * 8);
        sl.done = (int32_t *)dev_alloc(256);
    }
    if (sl.cap_chunks < nc) {
        dev_free(sl.chunk);
        sl.chunk = nullptr;
        sl.cap_chunks = 0;
        sl.chunk = (double *)dev_alloc((size_t)nc * 8);
        sl.cap_chunks = nc;
    }
}

void HipExec::release_slot(int slot)
{
    if (slot >= (int)S->slots.size())
        return;
    wait_frees(S);
    Slot &sl = S->slots[(size_t)slot];
    std::lock_guard<std::recursive_mutex> lk(lib_mutex());
    dev_free(sl.r);
    dev_free(sl.p);
    dev_free(sl.w);
    dev_free(sl.s);
    dev_free(sl.x);
    dev_free(sl.rw);
    dev_free(sl.rr);
    dev_free(sl.done);
    dev_free(sl.chunk);
    sl = Slot();
}

int HipExec::lane_of(int mid) { return S->mats[(size_t)mid].nnz >= kHeavyNnz ? 1 : 0; }

bool HipExec::tick_done(int lane, int tick)
{
    const hipError_t e = hipEventQuery(S->ticks[lane][tick].ev);
    if (e == hipErrorNotReady)
        return false;
    HIPC(e);
    return true;
}

void HipExec::wait_tick(int lane, int tick)
{
    HIPC(hipEventSynchronize(S->ticks[lane][tick].ev));
}

// Row blocks of a matrix whose grouped product can also write the r.w
// partials of a CG iteration (column panels or band, at most kBlock blocks:
// the step kernel sums them in one workgroup); 0 otherwise.
int32_t fused_rw_parts(const CsrHandle &h)
{
    const int32_t nb = h.use_panels ? h.pan.nblk : h.use_band ? h.band.nblk : 0;
    return (nb > 0 && nb <= kBlock) ? nb : 0;
}

// One batched tick over every active request of a lane.
void HipExec::launch_tick(int lane, int tick, const std::vector<serve::Request *> &reqs)
{
    TickBuf &tk = S->ticks[lane][tick];
    std::vector<MatDesc> descs;
    std::vector<int32_t> prefix(1, 0);
    std::vector<CgSeg> init, step;
    std::vector<serve::Request *> own, split;
    int32_t init_blocks = 0, step_blocks = 0;
    for (serve::Request *r : reqs) {
        SMatrix &m = S->mats[(size_t)r->mid];
        Slot &sl = S->slots[(size_t)r->slot];
        const double *in = r->in ? (const double *)r->in : m.vin;
        double *out = r->out ? (double *)r->out : sl.x;
        if (own_layout(*m.h)) {
            // matrices in a layout of their own run their own product kernel
            own.push_back(r);
        } else {
            if (r->kind == serve::kSpmv)
                descs.push_back(make_desc(*m.h, in, out, nullptr, sl.chunk));
            else
                descs.push_back(make_desc(*m.h, sl.r, sl.w, nullptr, sl.chunk));
            prefix.push_back(prefix.back() + m.h->ntiles);
            if (m.h->nsplit > 0)
                split.push_back(r);
        }
        if (r->kind == serve::kCg) {
            CgSeg sg{};
            sg.b = in;
            sg.x = out;
            sg.r = sl.r;
            sg.p = sl.p;
            sg.w = sl.w;
            sg.s = sl.s;
            sg.rw_part = sl.rw;
            sg.rr_part = sl.rr;
            sg.sc = (double *)((char *)sl.done + 64);
            sg.done = sl.done;
            sg.n = m.rows;
            sg.nb = cg_seg_blocks(m.rows);
            sg.iter = r->iter;
            sg.nrw = own_layout(*m.h) ? fused_rw_parts(*m.h) : 0;
            if (r->iter == 0) {
                sg.blk0 = init_blocks;
                init_blocks += sg.nb;
                init.push_back(sg);
            }
            sg.blk0 = step_blocks;
            step_blocks += sg.nb;
            step.push_back(sg);
        }
    }
    // column-panel and band products of the tick: one grouped launch each,
    // matrices with the most non-zeros per block first so that a launch
    // ends on short blocks
    std::vector<PanelDesc> pdesc;
    std::vector<PanelIO> pio;
    std::vector<int32_t> pprefix(1, 0);
    std::vector<BandDesc> bdesc;
    std::vector<PanelIO> bio;
    std::vector<int32_t> bprefix(1, 0);
    std::vector<serve::Request *> own_hot;
    auto per_block = [&](const serve::Request *r) {
        const CsrHandle &h = *S->mats[(size_t)r->mid].h;
        const int32_t nb = h.use_panels ? h.pan.nblk : h.use_band ? h.band.nblk : 1;
        return (double)h.nnz / (double)std::max(1, nb);
    };
    std::stable_sort(own.begin(), own.end(), [&](const serve::Request *a,
                                                 const serve::Request *b) {
        return per_block(a) > per_block(b);
    });
    for (serve::Request *r : own) {
        SMatrix &m = S->mats[(size_t)r->mid];
        Slot &sl = S->slots[(size_t)r->slot];
        const PanelIO io = (r->kind == serve::kSpmv)
                               ? PanelIO{r->in ? r->in : m.vin, r->out ? r->out : sl.x}
                               : PanelIO{sl.r, sl.w, fused_rw_parts(*m.h) ? sl.rw : nullptr};
        if (m.h->use_panels) {
            pdesc.push_back(m.h->pan);
            pio.push_back(io);
            pprefix.push_back(pprefix.back() + m.h->pan.nblk);
        } else if (m.h->use_band) {
            bdesc.push_back(m.h->band);
            bio.push_back(io);
            bprefix.push_back(bprefix.back() + m.h->band.nblk);
        } else {
            own_hot.push_back(r);
        }
    }
    const size_t b_desc = descs.size() * sizeof(MatDesc);
    const size_t b_pre = ((prefix.size() * 4 + 15) / 16) * 16;
    const size_t b_init = init.size() * sizeof(CgSeg);
    const size_t b_step = step.size() * sizeof(CgSeg);
    const size_t b_pdesc = pdesc.size() * sizeof(PanelDesc);
    const size_t b_pio = pio.size() * sizeof(PanelIO);
    const size_t b_ppre = ((pprefix.size() * 4 + 15) / 16) * 16;
    const size_t b_bdesc = bdesc.size() * sizeof(BandDesc);
    const size_t b_bio = bio.size() * sizeof(PanelIO);
    const size_t b_bpre = ((bprefix.size() * 4 + 15) / 16) * 16;
    const size_t total = b_desc + b_pre + b_init + b_step + b_pdesc + b_pio + b_ppre +
                         b_bdesc + b_bio + b_bpre;
    if (total > tk.cap)
        fail(LILAC_ERR_DEVICE, "tick tables larger than their buffer");
    size_t off = 0;
    auto put = [&](const void *src, size_t n, size_t padded) {
        if (n)
            std::memcpy(tk.host + off, src, n);
        const size_t at = off;
        off += padded;
        return at;
    };
    const size_t o_desc = put(descs.data(), b_desc, b_desc);
    const size_t o_pre = put(prefix.data(), prefix.size() * 4, b_pre);
    const size_t o_init = put(init.data(), b_init, b_init);
    const size_t o_step = put(step.data(), b_step, b_step);
    const size_t o_pdesc = put(pdesc.data(), b_pdesc, b_pdesc);
    const size_t o_pio = put(pio.data(), b_pio, b_pio);
    const size_t o_ppre = put(pprefix.data(), pprefix.size() * 4, b_ppre);
    const size_t o_bdesc = put(bdesc.data(), b_bdesc, b_bdesc);
    const size_t o_bio = put(bio.data(), b_bio, b_bio);
    const size_t o_bpre = put(bprefix.data(), bprefix.size() * 4, b_bpre);
    hipStream_t s = S->stream[lane];
    HIPC(hipMemcpyAsync(tk.dev, tk.host, off, hipMemcpyHostToDevice, s));
    const MatDesc *d_desc = (const MatDesc *)(tk.dev + o_desc);
    if (!init.empty())
        launch_cgb_init((const CgSeg *)(tk.dev + o_init), (int32_t)init.size(),
                        init_blocks, s);
    launch_spmv_segments(LILAC_F64, d_desc, (const int32_t *)(tk.dev + o_pre),
                         (int32_t)descs.size(), prefix.back(), tile_grid(LILAC_F64), s);
    launch_spmv_panels_grouped(LILAC_F64, (const PanelDesc *)(tk.dev + o_pdesc),
                               (const PanelIO *)(tk.dev + o_pio),
                               (const int32_t *)(tk.dev + o_ppre), (int32_t)pdesc.size(),
                               pprefix.back(), s);
    launch_spmv_band_grouped(LILAC_F64, (const BandDesc *)(tk.dev + o_bdesc),
                             (const PanelIO *)(tk.dev + o_bio),
                             (const int32_t *)(tk.dev + o_bpre), (int32_t)bdesc.size(),
                             bprefix.back(), s);
    for (serve::Request *r : own_hot) {
        SMatrix &m = S->mats[(size_t)r->mid];
        Slot &sl = S->slots[(size_t)r->slot];
        if (r->kind == serve::kSpmv)
            spmv_enqueue(*m.h, r->in ? r->in : m.vin, r->out ? r->out : sl.x,
                         Epi{EPI_NONE, 0, 0.0, 0.0}, nullptr, false, s);
        else
            spmv_enqueue(*m.h, sl.r, sl.w, Epi{EPI_NONE, 0, 0.0, 0.0}, nullptr, false, s);
    }
    // split rows: each request's chunk sums added up in chunk order, as the
    // single-matrix product does
    for (serve::Request *r : split) {
        SMatrix &m = S->mats[(size_t)r->mid];
        Slot &sl = S->slots[(size_t)r->slot];
        const MatDesc d = (r->kind == serve::kSpmv)
                              ? make_desc(*m.h, r->in ? r->in : m.vin,
                                          r->out ? r->out : sl.x, nullptr, sl.chunk)
                              : make_desc(*m.h, sl.r, sl.w, nullptr, sl.chunk);
        launch_split_finalize(LILAC_F64, nullptr, m.h->nsplit, d, nullptr,
                              Epi{EPI_NONE, 0, 0.0, 0.0}, nullptr, s);
    }
    if (!step.empty()) {
        const CgSeg *d_step = (const CgSeg *)(tk.dev + o_step);
        bool rw = false;   // some product did not write its r.w partials
        for (const CgSeg &sg : step)
            rw = rw || sg.nrw == 0;
        if (rw)
            launch_cgb_rw(d_step, (int32_t)step.size(), step_blocks, s);
        launch_cgb_step(d_step, (int32_t)step.size(), step_blocks, s);
    }
    HIPC(hipEventRecord(tk.ev, s));
}

// The plain path: the whole request alone with the single-matrix calls.
void HipExec::run_one(serve::Request *r)
{
    SMatrix &m = S->mats[(size_t)r->mid];
    Slot &sl = S->slots[(size_t)r->slot];
    const double *in = r->in ? (const double *)r->in : m.vin;
    double *out = r->out ? (double *)r->out : sl.x;
    hipStream_t s = S->stream[lane_of(r->mid)];   // the CUs its lane would have
    if (r->kind == serve::kSpmv) {
        spmv_enqueue(*m.h, in, out, Epi{EPI_NONE, 0, 0.0, 0.0}, nullptr, false, s);
    } else {
        // the CG state was made at upload, under the matrix's account
        thread_account() = &m.acct;
        try {
            std::lock_guard<std::recursive_mutex> lk(lib_mutex());
            run_cg(*m.h, in, out, r->iters, LILAC_CG_GRAPH, s, nullptr, nullptr);
        } catch (...) {
            thread_account() = &S->acct;
            throw;
        }
        thread_account() = &S->acct;
    }
    HIPC(hipStreamSynchronize(s));
}

// ------------------------------------------------------------- threads

void scheduler_main(Server *S)
{
    if (hipSetDevice(lib_device()) != hipSuccess) {
        S->core->die("hipSetDevice failed in the scheduler");
        return;
    }
    thread_account() = &S->acct;
    try {
        while (!S->stop.load()) {
            // with a tick on the device, look again soon (ticks end without
            // waking the scheduler); otherwise sleep until work arrives
            if (!S->core->step())
                S->core->wait_for_work(S->core->busy() ? 20000 : 200000);
        }
        S->core->shutdown();
    } catch (const Error &e) {
        S->core->die(e.msg);
    } catch (const std::exception &e) {
        S->core->die(e.what());
    }
    thread_account() = nullptr;
}

void fill_stats(Server *S, lilac_server_stats *o)
{
    const serve::Stats st = S->core->stats();
    std::memset(o, 0, sizeof(*o));
    o->completed = st.completed;
    o->spmv_done = st.spmv_done;
    o->cg_done = st.cg_done;
    o->failed = st.failed;
    o->p50_us = st.p50_us;
    o->p99_us = st.p99_us;
    o->mean_us = st.mean_us;
    o->max_us = st.max_us;
    o->wall_s = st.wall_s;
    o->req_per_s = st.req_per_s;
    o->solves_per_s = st.solves_per_s;
    o->gbytes_per_s = st.gbytes_per_s;
    o->uploads = st.uploads;
    o->evictions = st.evictions;
    o->ticks = st.ticks;
    o->planned_peak_bytes = st.planned_peak;
    o->mean_wait_us = st.mean_wait_us;
    o->mean_run_us = st.mean_run_us;
    o->waited_upload = st.waited_upload;
    std::lock_guard<std::recursive_mutex> lk(lib_mutex());
    o->peak_device_bytes = S->acct.peak;
    o->device_bytes = S->acct.in_use;
}

void free_server(Server *S)
{
    std::lock_guard<std::recursive_mutex> lk(lib_mutex());
    for (const Evicted &e : S->free_q) {
        destroy_handle(e.h);
        dev_free(e.vin);
    }
    S->free_q.clear();
    for (auto &t : S->tmp)
        tmp_cache_release(t);
    for (auto &m : S->mats) {
        if (m.h)
            destroy_handle(m.h);
        dev_free(m.vin);
        if (m.pin)
            (void)hipHostFree(m.pin);
    }
    for (auto &sl : S->slots) {
        dev_free(sl.r);
        dev_free(sl.p);
        dev_free(sl.w);
        dev_free(sl.s);
        dev_free(sl.x);
        dev_free(sl.rw);
        dev_free(sl.rr);
        dev_free(sl.done);
        dev_free(sl.chunk);
    }
    for (auto &lane : S->ticks)
        for (auto &t : lane) {
            if (t.host)
                (void)hipHostFree(t.host);
            dev_free(t.dev);
            if (t.ev)
                (void)hipEventDestroy(t.ev);
        }
    for (auto &us : S->up_stream)
        if (us)
            (void)hipStreamDestroy(us);
    for (auto &st : S->stream)
        if (st)
            (void)hipStreamDestroy(st);
    delete S->core;
    delete S;
}

// Starts the threads at the first request (matrices are all registered).
void start(Server *S)
{
    std::lock_guard<std::mutex> slk(S->start_mu);
    if (S->started.load())
        return;
    serve::Limits lim;
    lim.budget = S->cfg.hbm_budget;
    lim.max_active = S->cfg.max_active;
    lim.pool_capacity = S->cfg.pool_capacity;
    lim.fifo = S->fifo;
    {
        std::lock_guard<std::recursive_mutex> lk(lib_mutex());
        thread_account() = &S->acct;
        try {
            const size_t cap =
                round256(64 + (size_t)S->cfg.max_active * (per_request_table_bytes() + 64));
            for (auto &lane : S->ticks)
                for (auto &t : lane) {
                    HIPC(hipHostMalloc((void **)&t.host, cap, hipHostMallocDefault));
                    t.dev = (char *)dev_alloc(cap);
                    t.cap = cap;
                }
        } catch (...) {
            thread_account() = nullptr;
            throw;
        }
        thread_account() = nullptr;
        // the upload threads' build caches, charged to the server as they grow
        lim.overhead = S->acct.in_use + kUploadThreads * (int64_t)kTmpCacheLimit;
        for (auto &t : S->tmp) {
            t.limit = kTmpCacheLimit;
            t.acct = &S->acct;
        }
    }
    S->core = new serve::Core(S->exec, lim);
    for (auto &m : S->mats) {
        const int64_t sp = m.nnz * 12 + (int64_t)(m.rows + 1) * 4 +
                           (int64_t)(m.cols + m.rows) * 8;
        S->core->add_matrix(sp, sp + 9 * (int64_t)m.rows * 8);
    }
    S->sched = std::thread(scheduler_main, S);
    for (int t = 0; t < kUploadThreads; ++t)
        S->uploader[t] = std::thread(upload_loop, S, t);
    S->started.store(true);
}

}  // namespace
}  // namespace lilac

using namespace lilac;

template <typename F>
static int sguard(F &&f)
{
    try {
        f();
        return LILAC_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return LILAC_ERR_DEVICE;
    }
}

extern "C" {

int lilac_server_create(lilac_server_t *out, const lilac_server_config *cfg)
{
    return sguard([&] {
        if (!out)
            fail(LILAC_ERR_ARG, "NULL server pointer");
        *out = nullptr;
        {
            std::lock_guard<std::recursive_mutex> lk(lib_mutex());
            if (lilac_init(-1) != LILAC_OK)
                fail(LILAC_ERR_DEVICE, lilac_last_error());
        }
        auto *S = new Server();
        S->cfg.hbm_budget = (cfg && cfg->hbm_budget > 0) ? cfg->hbm_budget
                                                         : (int64_t)200 << 30;
        S->cfg.max_active = (cfg && cfg->max_active > 0) ? cfg->max_active : 256;
        S->cfg.pool_capacity = (cfg && cfg->pool_capacity > 0) ? cfg->pool_capacity : 1 << 20;
        S->cfg.fifo = cfg ? cfg->fifo : 0;
        S->fifo = S->cfg.fifo != 0;
        S->acct.limit = S->cfg.hbm_budget;
        try {
            const int cus = device_cu_count();
            create_masked_stream(&S->stream[0], kUploadCus, cus);
            HIPC(hipStreamCreateWithFlags(&S->stream[1], hipStreamNonBlocking));
            for (auto &us : S->up_stream)
                create_masked_stream(&us, 0, kUploadCus);
            for (auto &lane : S->ticks)
                for (auto &t : lane)
                    HIPC(hipEventCreateWithFlags(&t.ev, hipEventDisableTiming));
        } catch (...) {
            free_server(S);
            throw;
        }
        *out = (lilac_server_t)S;
    });
}

int lilac_server_add_matrix(lilac_server_t hs, int rows, int cols, int64_t nnz,
                            const int *row_ptr, const int *col_idx,
                            const double *vals, int *id)
{
    Server *S = (Server *)hs;
    return sguard([&] {
        if (!S || !id || rows < 0 || nnz < 0 || !row_ptr || (nnz && (!col_idx || !vals)))
            fail(LILAC_ERR_ARG, "bad argument");
        if (S->started.load())
            fail(LILAC_ERR_STATE, "add matrices before submitting requests");
        SMatrix m;
        m.rows = rows;
        m.cols = cols >= 0 ? cols : rows;
        m.nnz = nnz;
        m.acct.parent = &S->acct;
        // a pinned copy: uploads then run at DMA speed, and the caller's
        // arrays are free once this returns
        const size_t b_rp = (size_t)(rows + 1) * 4, b_col = (size_t)nnz * 4;
        const size_t b_col_pad = (b_col + 7) & ~(size_t)7;
        HIPC(hipHostMalloc(&m.pin, b_rp + b_col_pad + (size_t)nnz * 8 + 8,
                           hipHostMallocDefault));
        char *base = (char *)m.pin;
        std::memcpy(base, row_ptr, b_rp);
        if (nnz) {
            std::memcpy(base + b_rp, col_idx, b_col);
            std::memcpy(base + b_rp + b_col_pad, vals, (size_t)nnz * 8);
        }
        m.rp = (const int32_t *)base;
        m.col = (const int32_t *)(base + b_rp);
        m.vals = (const double *)(base + b_rp + b_col_pad);
        S->mats.push_back(m);
        S->max_rows = std::max(S->max_rows, std::max(m.rows, m.cols));
        *id = (int)S->mats.size() - 1;
    });
}

int lilac_server_submit(lilac_server_t hs, const lilac_request *r, uint64_t *ticket)
{
    Server *S = (Server *)hs;
    return sguard([&] {
        if (!S || !r)
            fail(LILAC_ERR_ARG, "bad argument");
        if (r->matrix < 0 || r->matrix >= (int)S->mats.size())
            fail(LILAC_ERR_ARG, "unknown matrix id");
        if (r->kind != LILAC_REQ_SPMV && r->kind != LILAC_REQ_CG)
            fail(LILAC_ERR_ARG, "unknown request kind");
        const SMatrix &m = S->mats[(size_t)r->matrix];
        if (r->kind == LILAC_REQ_CG && (r->iters <= 0 || m.rows != m.cols))
            fail(LILAC_ERR_ARG, "CG needs iters > 0 and a square matrix");
        start(S);
        if (S->core->dead())
            fail(LILAC_ERR_STATE, "server stopped after an error: " + S->core->error());
        auto *q = new serve::Request();
        q->kind = r->kind;
        q->mid = r->matrix;
        q->iters = r->iters;
        q->in = r->in;
        q->out = r->out;
        q->t_arr = r->arrival_ns > 0 ? r->arrival_ns : now_ns();
        const uint64_t t = S->core->submit(q);
        if (ticket)
            *ticket = t;
    });
}

int lilac_server_poll(lilac_server_t hs, uint64_t ticket, int *done)
{
    Server *S = (Server *)hs;
    return sguard([&] {
        if (!S || !done)
            fail(LILAC_ERR_ARG, "bad argument");
        const int st = S->core ? S->core->poll(ticket) : -2;
        if (st == -2)
            fail(LILAC_ERR_ARG, "unknown ticket");
        *done = st;
    });
}

int lilac_server_wait(lilac_server_t hs, uint64_t ticket)
{
    Server *S = (Server *)hs;
    return sguard([&] {
        if (!S)
            fail(LILAC_ERR_ARG, "bad argument");
        const int st = S->core ? S->core->wait(ticket) : -2;
        if (st == -2)
            fail(LILAC_ERR_ARG, "unknown ticket");
        if (st < 0)
            fail(LILAC_ERR_STATE, "request failed: " + S->core->error());
    });
}

int lilac_server_now(lilac_server_t hs, int64_t *ns)
{
    Server *S = (Server *)hs;
    return sguard([&] {
        if (!S || !ns)
            fail(LILAC_ERR_ARG, "bad argument");
        *ns = now_ns();
    });
}

int lilac_server_stats_get(lilac_server_t hs, lilac_server_stats *out)
{
    Server *S = (Server *)hs;
    return sguard([&] {
        if (!S || !out)
            fail(LILAC_ERR_ARG, "bad argument");
        start(S);
        fill_stats(S, out);
    });
}

int lilac_server_reset_stats(lilac_server_t hs)
{
    Server *S = (Server *)hs;
    return sguard([&] {
        if (!S)
            fail(LILAC_ERR_ARG, "bad argument");
        start(S);
        S->core->reset_stats();
        std::lock_guard<std::recursive_mutex> lk(lib_mutex());
        S->acct.peak = S->acct.in_use;
    });
}

int lilac_server_run_trace(lilac_server_t hs, int n, const int64_t *arrival_ns,
                           const int *kind, const int *matrix, int cg_iters,
                           lilac_server_stats *out)
{
    Server *S = (Server *)hs;
    return sguard([&] {
        if (!S || n < 0 || (n && (!arrival_ns || !kind || !matrix)) || cg_iters <= 0)
            fail(LILAC_ERR_ARG, "bad argument");
        for (int i = 0; i < n; ++i)
            if (matrix[i] < 0 || matrix[i] >= (int)S->mats.size() ||
                (kind[i] != LILAC_REQ_SPMV && kind[i] != LILAC_REQ_CG) ||
                (kind[i] == LILAC_REQ_CG &&
                 S->mats[(size_t)matrix[i]].rows != S->mats[(size_t)matrix[i]].cols))
                fail(LILAC_ERR_ARG, "bad request in trace");
        start(S);
        if (S->core->dead())
            fail(LILAC_ERR_STATE, "server stopped after an error: " + S->core->error());
        S->core->reset_stats();
        std::vector<uint64_t> tickets((size_t)n);
        const int64_t t0 = now_ns() + 1000000;  // start 1 ms from now
        for (int i = 0; i < n; ++i) {
            const int64_t due = t0 + arrival_ns[i];
            int64_t t = now_ns();
            if (due - t > 200000)
                std::this_thread::sleep_for(std::chrono::nanoseconds(due - t - 100000));
            while ((t = now_ns()) < due) {
            }
            auto *q = new serve::Request();
            q->kind = kind[i];
            q->mid = matrix[i];
            q->iters = cg_iters;
            q->t_arr = due;
            // trace mode: the server's operand and the slot's own output
            tickets[(size_t)i] = S->core->submit(q);
        }
        for (uint64_t tkt : tickets)
            S->core->wait(tkt);
        for (uint64_t tkt : tickets)
            S->core->forget(tkt);
        if (out)
            fill_stats(S, out);
    });
}

int lilac_server_destroy(lilac_server_t hs)
{
    Server *S = (Server *)hs;
    return sguard([&] {
        if (!S)
            return;
        S->stop.store(true);
        if (S->started.load()) {
            {
                std::lock_guard<std::mutex> lk(S->up_mu);
                S->up_cv.notify_all();
            }
            S->core->wake();
            if (S->sched.joinable())
                S->sched.join();
            for (auto &u : S->uploader) {
                {
                    std::lock_guard<std::mutex> lk(S->up_mu);
                    S->up_cv.notify_all();
                }
                if (u.joinable())
                    u.join();
            }
        }
        for (auto &st : S->stream)
            if (st)
                (void)hipStreamSynchronize(st);
        free_server(S);
    });
}

}  // extern "C"
